// Gram of the hidden matrix for the normal equations, eq. (8):
//   M = H^T H (L x L) when N >= L, M = H H^T (N x N) when N < L (the two
//   pseudoinverse forms stated before eq. 8).  Only the upper block triangle
//   is computed; each value is written to both (i, j) and (j, i), so M is
//   exactly symmetric.
//
// Every element is accumulated in one fixed order (tile k-loop, then a
// fixed-order FP64 sum over split-K chunks; no atomics), so bitwise-equal
// columns of H give bitwise-equal rows of M.  The pivoted Cholesky relies on
// that to send the Schur diagonal of a duplicated hidden node to ~0.
//
// Kernels:
//   FP64 (single problems): the FP64 GEMM's upper tiles per K chunk, then
//     gram_sum_mirror_kernel (chunk sum in FP64, mirrored).
//   gram16_kernel<T, KCONTIG>  FP32, and FP64 in the batches' grouped launches
//     (the same products in the same order), 16x16x4 MFMA, 128 x 128 tiles.
//     KCONTIG=false: operand element (row, k) at base[k*ld + row] (columns of
//       a sample-major H: the column Gram H^T H).
//     KCONTIG=true:  element (row, k) at base[row*ld + k] (rows of a
//       sample-major H for H H^T, or a node-major copy for H^T H).
//   gram_lp_kernel<HT>  BF16 or FP16 node-major copy, 32x32x16 MFMA with FP32
//     accumulation, 128 x 128 tiles.
//   gram_reduce_kernel  sums the split-K partial tiles in FP64 and mirrors.
#include "elm_internal.h"

#include <cstdlib>

#include <algorithm>
#include <cmath>
#include <mutex>

namespace elm {
namespace {

constexpr int TILE = 128;
constexpr int NT = 256;  // 4 waves in a 2 x 2 grid of 64 x 64 sub-tiles

// upper-triangular tile index t -> (bi, bj), bi <= bj, column-major over bj
__device__ inline void tile_coords(int64_t t, int& bi, int& bj) {
    int64_t c = (int64_t)((sqrt(8.0 * (double)t + 1.0) - 1.0) * 0.5);
    while (c * (c + 1) / 2 > t) --c;
    while ((c + 1) * (c + 2) / 2 <= t) ++c;
    bj = (int)c;
    bi = (int)(t - c * (c + 1) / 2);
}

template <typename T, bool KCONTIG>
__device__ __forceinline__ void gram16_body(int64_t bx, int64_t by, int64_t n, int64_t K,
                                            int64_t kc_len, const T* __restrict__ A, int64_t ld,
                                            T* __restrict__ part, int64_t ntile) {
    constexpr int BK = 16;  // samples per stage (32 for FP32 measured no faster)
    constexpr int EL = (BK * TILE) / NT;  // staged elements per thread and operand
    // two stages: the next chunk's loads are in flight while this one multiplies
    __shared__ T As[2][BK][TILE + 1];
    __shared__ T Bs[2][BK][TILE + 1];

    int bi, bj;
    tile_coords(bx, bi, bj);
    const int64_t r0 = (int64_t)bi * TILE, c0 = (int64_t)bj * TILE;
    const int64_t kbeg = by * kc_len;
    const int64_t kend = min(K, kbeg + kc_len);

    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int wm = wave >> 1, wn = wave & 1;

    typename Mfma16<T>::acc_t acc[4][4];
#pragma unroll
    for (int a = 0; a < 4; ++a)
#pragma unroll
        for (int b = 0; b < 4; ++b) acc[a][b] = typename Mfma16<T>::acc_t{};

    T va[EL], vb[EL];
    auto load = [&](int64_t k0) {
#pragma unroll
        for (int it = 0; it < EL; ++it) {
            const int e = tid + it * NT;
            int row, k;
            if (KCONTIG) { row = e / BK; k = e % BK; }
            else         { k = e / TILE; row = e % TILE; }
            const int64_t gk = k0 + k;
            const int64_t ga = r0 + row, gb = c0 + row;
            T x = T(0), y = T(0);
            if (gk < kend) {
                if (ga < n) x = KCONTIG ? A[ga * ld + gk] : A[gk * ld + ga];
                if (gb < n) y = KCONTIG ? A[gb * ld + gk] : A[gk * ld + gb];
            }
            va[it] = x;
            vb[it] = y;
        }
    };
    auto store = [&](int buf) {
#pragma unroll
        for (int it = 0; it < EL; ++it) {
            const int e = tid + it * NT;
            int row, k;
            if (KCONTIG) { row = e / BK; k = e % BK; }
            else         { k = e / TILE; row = e % TILE; }
            As[buf][k][row] = va[it];
            Bs[buf][k][row] = vb[it];
        }
    };

    if (kbeg < kend) {
        load(kbeg);
        store(0);
        __syncthreads();
        int buf = 0;
        for (int64_t k0 = kbeg; k0 < kend; k0 += BK) {
            const bool more = k0 + BK < kend;  // block-uniform
            if (more) load(k0 + BK);
#pragma unroll
            for (int kk = 0; kk < BK; kk += 4) {
                const int k = kk + (lane >> 4);
                T a[4], b[4];
#pragma unroll
                for (int q = 0; q < 4; ++q) {
                    a[q] = As[buf][k][wm * 64 + q * 16 + (lane & 15)];
                    b[q] = Bs[buf][k][wn * 64 + q * 16 + (lane & 15)];
                }
#pragma unroll
                for (int x = 0; x < 4; ++x)
#pragma unroll
                    for (int y = 0; y < 4; ++y) acc[x][y] = Mfma16<T>::op(a[x], b[y], acc[x][y]);
            }
            // the other buffer was last read before the previous barrier
            if (more) store(buf ^ 1);
            __syncthreads();
            buf ^= 1;
        }
    }

    T* out = part + (by * ntile + bx) * (TILE * TILE);
#pragma unroll
    for (int x = 0; x < 4; ++x)
#pragma unroll
        for (int y = 0; y < 4; ++y)
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                const int row = wm * 64 + x * 16 + Mfma16<T>::row(lane, v);
                const int col = wn * 64 + y * 16 + (lane & 15);
                out[row * TILE + col] = acc[x][y][v];
            }
}

template <typename T, bool KCONTIG>
__global__ __launch_bounds__(NT) void gram16_kernel(int64_t n, int64_t K, int64_t kc_len,
                                                    const T* __restrict__ A, int64_t ld,
                                                    T* __restrict__ part, int64_t ntile) {
    gram16_body<T, KCONTIG>(blockIdx.x, blockIdx.y, n, K, kc_len, A, ld, part, ntile);
}

template <typename HT> struct Mfma32;
template <> struct Mfma32<__bf16> {
    typedef bf8v vec_t;
    static __device__ inline f16v op(vec_t a, vec_t b, f16v c) {
        return __builtin_amdgcn_mfma_f32_32x32x16_bf16(a, b, c, 0, 0, 0);
    }
};
template <> struct Mfma32<_Float16> {
    typedef h8v vec_t;
    static __device__ inline f16v op(vec_t a, vec_t b, f16v c) {
        return __builtin_amdgcn_mfma_f32_32x32x16_f16(a, b, c, 0, 0, 0);
    }
};

// 32x32x16 MFMA operand/result layout (measured on gfx950): lane l holds
// A[l % 32][8 (l / 32) + e], e = 0..7, and B likewise by column; result row of
// register v is 8 (v / 4) + 4 (l / 32) + v % 4, column l % 32.

// M[i][j] = M[j][i] = sum over chunks (in chunk order, FP64) of the partial tiles
template <typename PT>
__device__ __forceinline__ void gram_reduce_body(int64_t bx, int64_t n, const PT* __restrict__ part,
                                                 int64_t ntile, int nchunk, double* __restrict__ M,
                                                 int64_t ldm) {
    int bi, bj;
    tile_coords(bx, bi, bj);
    const int64_t r0 = (int64_t)bi * TILE, c0 = (int64_t)bj * TILE;
    for (int e = threadIdx.x; e < TILE * TILE; e += NT) {
        const int row = e / TILE, col = e % TILE;
        const int64_t gi = r0 + row, gj = c0 + col;
        if (gi >= n || gj >= n || gi > gj) continue;
        double s = 0.0;
        for (int c = 0; c < nchunk; ++c)
            s += (double)part[((int64_t)c * ntile + bx) * (TILE * TILE) + e];
        M[gi * ldm + gj] = s;
        M[gj * ldm + gi] = s;
    }
}

// M = the sum over chunks (in chunk order, FP64) of the upper triangles of
// the chunk products P[c] (n x n, ld ldp, c_bs apart), written to (i, j) and
// (j, i): one 32 x 32 tile of the upper block triangle per block, its
// transpose written from LDS so both stores are whole rows
constexpr int MT = 32;
__global__ __launch_bounds__(256) void gram_sum_mirror_kernel(int64_t n, const double* __restrict__ P,
                                                              int64_t ldp, int64_t c_bs, int nchunk,
                                                              double* __restrict__ M, int64_t ldm) {
    __shared__ double t[MT][MT + 1];
    int bi, bj;
    tile_coords(blockIdx.x, bi, bj);
    const int tx = threadIdx.x & (MT - 1), ty = threadIdx.x / MT;  // 32 x 8
    const int64_t i0 = (int64_t)bi * MT, j0 = (int64_t)bj * MT;
#pragma unroll
    for (int q = 0; q < MT / 8; ++q) {
        const int li = ty + 8 * q;
        int64_t i = i0 + li, j = j0 + tx;
        if (i < n && j < n) {
            if (i > j) {  // lower half of a diagonal tile: the upper entry
                const int64_t x = i;
                i = j;
                j = x;
            }
            double v = 0.0;
            for (int c = 0; c < nchunk; ++c) v += P[(int64_t)c * c_bs + i * ldp + j];
            M[(i0 + li) * ldm + j0 + tx] = v;
            t[li][tx] = v;
        }
    }
    if (bi == bj) return;  // block-uniform: the tile is its own transpose
    __syncthreads();
#pragma unroll
    for (int q = 0; q < MT / 8; ++q) {
        const int lj = ty + 8 * q;
        const int64_t j = j0 + lj, i = i0 + tx;
        if (i < n && j < n) M[j * ldm + i] = t[tx][lj];
    }
}

template <typename PT>
__global__ __launch_bounds__(NT) void gram_reduce_kernel(int64_t n, const PT* __restrict__ part,
                                                         int64_t ntile, int nchunk,
                                                         double* __restrict__ M, int64_t ldm) {
    gram_reduce_body<PT>(blockIdx.x, n, part, ntile, nchunk, M, ldm);
}

// Split the reduction length K into chunks so the grid has enough blocks.
void plan_chunks(int64_t ntile, int64_t K, int64_t quantum, int64_t& kc_len, int& nchunk) {
    const int64_t want_blocks = 1024;
    int64_t nc = (want_blocks + ntile - 1) / ntile;
    int64_t max_nc = (K + 1023) / 1024;  // keep chunks at least ~1024 long
    if (nc > max_nc) nc = max_nc;
    if (nc > 64) nc = 64;
    if (nc < 1) nc = 1;
    kc_len = cdiv(cdiv(K, nc), quantum) * quantum;
    nchunk = (int)cdiv(K, kc_len);
}

// The default K chunks of the FP32/FP64 Gram: plan_chunks' rule, and for
// FP64 chunks of about 16384 samples (within 16 GiB of partial products),
// which keep the blocks that share a panel in step (L2 reuse).  On N = 500000,
// L = 10000 the Gram took 1109 ms in one chunk, 1029 in 8, 1013 in 16 and
// 1000 in 32; on N = 100000, L = 5000 58.9 ms in 2, 56.9 in 8 and 55.2 in 32.
static void default_chunks(int dt, int64_t n, int64_t ntile, int64_t K, int64_t& kc_len, int& nchunk) {
    plan_chunks(ntile, K, 16, kc_len, nchunk);
    if (dt == ELM_F64) {
        const int64_t cap = std::max<int64_t>(1, ((int64_t)16 << 30) / (8 * n * n));
        const int64_t want = std::min<int64_t>(std::min<int64_t>(cdiv(K, 16384), 32), cap);
        if (want > nchunk) {
            kc_len = cdiv(cdiv(K, want), 16) * 16;
            nchunk = (int)cdiv(K, kc_len);
        }
    }
}

// K chunks of the FP32/FP64 Gram: force_chunks > 0, else the tuning table's
// row for this shape, else the default rule
void gram16_chunks(int dt, int64_t n, int64_t ntile, int64_t K, int force_chunks, const Workspace& ws,
                   int64_t& kc_len, int& nchunk) {
    default_chunks(dt, n, ntile, K, kc_len, nchunk);
    int nc = force_chunks > 0 ? force_chunks : ws.find_tune(ELM_TUNE_GRAM_CHUNKS, dt, n, K);
    if (nc > 0) {
        nc = std::max(1, std::min(64, nc));
        kc_len = cdiv(cdiv(K, nc), 16) * 16;
        nchunk = (int)cdiv(K, kc_len);
    }
}

// Returns the longest run of products accumulated in T before the FP64 sum.
template <typename T, bool KCONTIG>
int64_t run_gram16(hipStream_t s, int64_t n, int64_t K, const T* A, int64_t ld, double* M,
                   int64_t ldm, Workspace& ws, int force_chunks = 0) {
    const int64_t nt = cdiv(n, TILE);
    const int64_t ntile = nt * (nt + 1) / 2;
    int64_t kc_len;
    int nchunk;
    gram16_chunks(sizeof(T) == 8 ? ELM_F64 : ELM_F32, n, ntile, K, force_chunks, ws, kc_len, nchunk);
    T* part = (T*)ws.get("gram_part", (size_t)ntile * nchunk * TILE * TILE * sizeof(T));
    {
        StageScope sc(ws.prof, ELM_STAGE_GRAM, s);
        gram16_kernel<T, KCONTIG><<<dim3((unsigned)ntile, (unsigned)nchunk), NT, 0, s>>>(
            n, K, kc_len, A, ld, part, ntile);
        ELM_LAUNCH_CHECK();
    }
    StageScope sc(ws.prof, ELM_STAGE_GRAM_REDUCE, s);
    gram_reduce_kernel<T><<<(unsigned)ntile, NT, 0, s>>>(n, part, ntile, nchunk, M, ldm);
    ELM_LAUNCH_CHECK();
    return kc_len;
}

// The FP64 Gram on the library's FP64 GEMM (its tiles and MFMA steps take
// the products of each element in the order gram16_kernel does: K chunks of
// kc_len, steps of 16 and of 4 inside them): the chunks' upper tiles in one
// batched launch (a shorter last chunk in a second), then their sum in chunk
// order and the mirror.  kcontig: operand element (row, k) at A[row * ld + k]
// (H H^T of a sample-major H); else at A[k * ld + row] (H^T H).  (On the FP32
// node-major copy the same route took twice gram16_kernel's time: the FP32
// Gram stays there.)
static void run_gram_f64(hipStream_t s, int64_t n, int64_t K, const double* A, int64_t ld, bool kcontig,
                         double* M, int64_t ldm, Workspace& ws, int force_chunks) {
    const int64_t nt = cdiv(n, TILE);
    const int64_t ntile = nt * (nt + 1) / 2;
    int64_t kc_len;
    int nchunk;
    gram16_chunks(ELM_F64, n, ntile, K, force_chunks, ws, kc_len, nchunk);
    const int64_t a_rs = kcontig ? ld : 1, a_cs = kcontig ? 1 : ld;   // A(i, k)
    const int64_t b_rs = kcontig ? 1 : ld, b_cs = kcontig ? ld : 1;   // B(k, j) = A(j, k)
    const int64_t kstep = kcontig ? 1 : ld;                           // one k further
    // a single chunk goes straight to M
    double* P = M;
    int64_t ldp = ldm, c_bs = 0;
    if (nchunk > 1) {
        P = (double*)ws.get("gram_part64", (size_t)nchunk * n * n * sizeof(double));
        ldp = n;
        c_bs = n * n;
    }
    auto gemm = [&](int64_t batch, int64_t kl, const double* Ak, double* C) {
        gemm_f64_batched(s, batch, n, n, kl, 1.0, Ak, a_rs, a_cs, kl * kstep, Ak, b_rs, b_cs, kl * kstep,
                         0.0, C, ldp, c_bs, false, false, true, nullptr);
    };
    const int64_t last = K - (int64_t)(nchunk - 1) * kc_len;
    const int nfull = last == kc_len ? nchunk : nchunk - 1;
    {
        StageScope sc(ws.prof, ELM_STAGE_GRAM, s);
        if (nfull > 0) gemm(nfull, kc_len, A, P);
        if (nfull < nchunk) gemm(1, last, A + (int64_t)nfull * kc_len * kstep, P + (int64_t)nfull * c_bs);
    }
    StageScope sc(ws.prof, ELM_STAGE_GRAM_REDUCE, s);
    const int64_t mt = cdiv(n, MT);
    gram_sum_mirror_kernel<<<(unsigned)(mt * (mt + 1) / 2), 256, 0, s>>>(n, P, ldp, c_bs, nchunk, M, ldm);
    ELM_LAUNCH_CHECK();
}

// ---------------------------------------------------------------------------
// 16-bit node-major Gram, 256 x 256 tiles (the high-throughput path).
//
// Each block owns one work item (split-K chunk, tile bi <= bj) from a table
// built on the host.  4 waves in a 2 x 2 grid each accumulate a 128 x 128
// sub-tile as 4 x 4 blocks of the 32x32x16 MFMA (256 FP32 accumulators per
// lane, in AGPRs).  K is consumed in stages of 64 samples: a stage holds
// 128 contiguous bytes of each of the 512 operand rows (64 KB), and two LDS
// buffers alternate, filled by direct global->LDS loads
// (global_load_lds_dwordx4) one stage ahead.  When the leading dimension is
// a multiple of 64 elements (the library pads its own 16-bit copies so), a
// row's stage segment is exactly one 128-byte cache line and a load
// instruction moves 8 whole lines; unaligned rows straddle two lines and
// cost about a tenth of the Gram's time.  The load path, not the MFMAs, sets
// the pace of this kernel: each load instruction occupies the CU's address
// unit for about 16 cycles, so a stage's 64 instructions are spread over the
// MFMAs of three k16 steps rather than issued in a burst that stalls the
// waves.  The loads stay in flight across the steps (explicit vmcnt and
// lgkmcnt waits with bare s_barriers: a full __syncthreads would drain them).
// Every stage issues the same number of loads (past the last full stage they
// re-read it into a buffer nobody reads again), so the wait counts are
// static.
// In LDS a tile row is 8 chunks of 16 B; chunk c of row r sits at position
// c ^ ((r >> 1) & 7): two rows share one 256-byte bank line, r % 2 picks the
// half, and the swizzle spreads the 8 row pairs of 16 consecutive rows over
// the 8 slots of a half, so the 16 rows that one quarter-wave of an operand
// read (ds_read_b128) touches hit 16 distinct 4-bank groups.  Ragged tiles
// load clamped rows on the same path; the K tail (fewer than 64 samples) and
// unaligned input take a plain path, 32 samples at a time.
// ---------------------------------------------------------------------------
constexpr int GT = 256;    // tile
constexpr int GBK = 64;    // samples per stage of the load path (128-byte row segments)
constexpr int G_OPB = GT * GBK * 2;            // bytes per operand per stage (32 KB)
constexpr int G_STB = 2 * G_OPB;               // bytes per stage (64 KB)
constexpr int GTK = 32;    // samples per step of the plain tail path
constexpr int GT_OPB = GT * GTK * 2;           // bytes per operand per tail step (16 KB)
#define G_VMCNT(N) (((N) & 15) | (((N) >> 4) << 14) | (7 << 4) | (15 << 8))
#define G_LGKMCNT(N) (15 | (3 << 14) | (7 << 4) | ((N) << 8))

typedef __attribute__((address_space(3))) void lds_void;

template <typename HT>
__device__ __forceinline__ void gram_lp256_body(const int4 wk, int64_t n, int64_t K, int64_t kc_len,
                                                const HT* __restrict__ A, int64_t ld,
                                                float* __restrict__ part) {
    __shared__ __attribute__((aligned(1024))) unsigned char smem[2 * G_STB];
    typedef typename Mfma32<HT>::vec_t vec_t;
    if (wk.x < 0) return;
    const int64_t r0 = (int64_t)wk.y * GT, c0 = (int64_t)wk.z * GT;
    const int64_t kbeg = (int64_t)wk.x * kc_len;
    const int64_t kend = min(K, kbeg + kc_len);
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int wm = wave >> 1, wn = wave & 1;
    const bool vec_ok = ((ld & 7) == 0) && ((((uintptr_t)A) & 15) == 0);

    f16v acc[4][4];
#pragma unroll
    for (int x = 0; x < 4; ++x)
#pragma unroll
        for (int y = 0; y < 4; ++y) acc[x][y] = f16v{};

#define GRAM_MMA(FA, FB)                                                                   \
    do {                                                                                   \
        _Pragma("unroll") for (int x = 0; x < 4; ++x)                                      \
            _Pragma("unroll") for (int y = 0; y < 4; ++y)                                  \
                acc[x][y] = Mfma32<HT>::op(FA[x], FB[y], acc[x][y]);                       \
    } while (0)

    // Ragged tiles take the same path: rows past n read row n - 1 (their
    // results land in partial-tile rows the reduction never reads).
    const bool interior = vec_ok;  // block-uniform
    const int64_t nfull = interior ? (kend - kbeg) / GBK : 0;
    if (nfull > 0) {
        // fragments of k16 step S (0..3) of the stage in buffer BUF
#define GRAM_READ(FA, FB, BUF, S)                                                          \
    do {                                                                                   \
        const unsigned char* sA = smem + (BUF) * G_STB;                                    \
        const unsigned char* sB = sA + G_OPB;                                              \
        _Pragma("unroll") for (int x = 0; x < 4; ++x) {                                    \
            const int ra = wm * 128 + x * 32 + (lane & 31);                                \
            const int rb = wn * 128 + x * 32 + (lane & 31);                                \
            const int c = (lane >> 5) + 2 * (S);                                           \
            FA[x] = *(const vec_t*)(sA + ra * 128 + ((c ^ ((ra >> 1) & 7)) << 4));         \
            FB[x] = *(const vec_t*)(sB + rb * 128 + ((c ^ ((rb >> 1) & 7)) << 4));         \
        }                                                                                  \
    } while (0)
        // DMA lane mapping: instruction i of wave w fills LDS bytes
        // [(4 i + w) * 1024, +1024) of an operand buffer = rows (4 i + w) * 8
        // .. +8, lane l -> row (4 i + w) * 8 + l / 8, position l % 8, which
        // holds global chunk (l % 8) ^ ((row >> 1) & 7).
        const HT* asrc[8];
        const HT* bsrc[8];
#pragma unroll
        for (int i = 0; i < 8; ++i) {
            const int row = (4 * i + wave) * 8 + (lane >> 3);
            const int c = (lane & 7) ^ ((row >> 1) & 7);
            asrc[i] = A + min(r0 + row, n - 1) * ld + c * 8;
            bsrc[i] = A + min(c0 + row, n - 1) * ld + c * 8;
        }
        const int64_t klast = kbeg + (nfull - 1) * GBK;
        // loads Q0 .. Q0 + NL - 1 of the 16 that fill stage buffer BUF with
        // samples K0 .. K0 + 63 (clamped to the last full stage): load q is
        // instruction q / 2 of operand q % 2 (A rows, then B rows)
#define GRAM_LOADS(BUF, K0, Q0, NL)                                                          \
    do {                                                                                     \
        const int64_t k_ = min((int64_t)(K0), klast);                                        \
        unsigned char* dA = smem + (BUF) * G_STB + wave * 1024;                              \
        _Pragma("unroll") for (int q = (Q0); q < (Q0) + (NL); ++q) {                         \
            const int i = q >> 1;                                                            \
            if (q & 1)                                                                       \
                __builtin_amdgcn_global_load_lds((const void*)(bsrc[i] + k_),                \
                                                 (lds_void*)(dA + G_OPB + i * 4096), 16, 0, 0); \
            else                                                                             \
                __builtin_amdgcn_global_load_lds((const void*)(asrc[i] + k_),                \
                                                 (lds_void*)(dA + i * 4096), 16, 0, 0);      \
        }                                                                                    \
    } while (0)
        // one k16 step's 16 MFMAs with loads Q0 .. Q0 + NL - 1 of stage buffer
        // BUF interleaved, evenly spaced (load t after MFMA 16 t / NL), so
        // that the load issue (about 16 cycles of the address unit per
        // instruction) overlaps the MFMAs instead of stalling the wave in a
        // burst
#define GRAM_MMA_LOADS(FA, FB, BUF, K0, Q0, NL)                                              \
    do {                                                                                     \
        const int64_t k_ = min((int64_t)(K0), klast);                                        \
        unsigned char* dA = smem + (BUF) * G_STB + wave * 1024;                              \
        _Pragma("unroll") for (int q = 0; q < 16; ++q) {                                     \
            acc[q >> 2][q & 3] = Mfma32<HT>::op(FA[q >> 2], FB[q & 3], acc[q >> 2][q & 3]);  \
            _Pragma("unroll") for (int t = 0; t < (NL); ++t) {                               \
                if ((t * 16) / (NL) == q) {                                                  \
                    const int l = (Q0) + t, i = l >> 1;                                      \
                    if (l & 1)                                                               \
                        __builtin_amdgcn_global_load_lds((const void*)(bsrc[i] + k_),        \
                                                         (lds_void*)(dA + G_OPB + i * 4096), 16, 0, 0); \
                    else                                                                     \
                        __builtin_amdgcn_global_load_lds((const void*)(asrc[i] + k_),        \
                                                         (lds_void*)(dA + i * 4096), 16, 0, 0); \
                }                                                                            \
            }                                                                                \
        }                                                                                    \
    } while (0)
        // Fragment reads are software-pipelined against the MFMAs: step s + 1
        // is read while step s multiplies, and step 0 of stage st + 1 while
        // step 3 of stage st multiplies.  The barrier before that last read
        // publishes stage st + 1 (every wave has waited for its own loads of
        // it) and retires buffer st % 2 (every wave has read its four steps).
        // The 16 loads of stage st + 2 into that buffer go out with the next
        // three steps' MFMAs: 6 with step 3 of stage st, 5 with each of steps
        // 0 and 1 of stage st + 1, and land during steps 1-3.
        constexpr int LD3 = 6, LD0 = 5, LD1 = 5;
        static_assert(LD3 + LD0 + LD1 == 16, "a stage is 16 loads per wave");
        vec_t f0a[4], f0b[4], f1a[4], f1b[4];
        GRAM_LOADS(0, kbeg, 0, 16);
        GRAM_LOADS(1, kbeg + GBK, 0, LD3);
        __builtin_amdgcn_s_waitcnt(G_VMCNT(LD3));  // stage 0 landed
        __builtin_amdgcn_s_barrier();
        GRAM_READ(f0a, f0b, 0, 0);
        // (Step 0 of stage st + 1 is read in the last iteration too, from a
        // buffer whose contents are then unused, and the loads past the last
        // stage re-read it: the counts of LDS and memory operations per
        // iteration stay static, so the wait counts stay exact across the
        // back edge.  The scheduling barriers keep the MFMAs on their side
        // of the s_barrier.)
        for (int64_t st = 0; st < nfull; ++st) {
            const int cur = (int)(st & 1);
            __builtin_amdgcn_s_waitcnt(G_LGKMCNT(0));
            GRAM_READ(f1a, f1b, cur, 1);
            __builtin_amdgcn_sched_barrier(0);
            GRAM_MMA_LOADS(f0a, f0b, cur ^ 1, kbeg + (st + 1) * GBK, LD3, LD0);
            __builtin_amdgcn_sched_barrier(0);
            __builtin_amdgcn_s_waitcnt(G_LGKMCNT(0));
            GRAM_READ(f0a, f0b, cur, 2);
            __builtin_amdgcn_sched_barrier(0);
            GRAM_MMA_LOADS(f1a, f1b, cur ^ 1, kbeg + (st + 1) * GBK, LD3 + LD0, LD1);
            __builtin_amdgcn_sched_barrier(0);
            __builtin_amdgcn_s_waitcnt(G_LGKMCNT(0));
            GRAM_READ(f1a, f1b, cur, 3);
            __builtin_amdgcn_sched_barrier(0);
            GRAM_MMA(f0a, f0b);
            __builtin_amdgcn_sched_barrier(0);
            __builtin_amdgcn_s_waitcnt(G_LGKMCNT(0));
            __builtin_amdgcn_s_waitcnt(G_VMCNT(0));  // stage st + 1 landed
            __builtin_amdgcn_s_barrier();
            __builtin_amdgcn_sched_barrier(0);
            GRAM_READ(f0a, f0b, cur ^ 1, 0);
            __builtin_amdgcn_sched_barrier(0);
            GRAM_MMA_LOADS(f1a, f1b, cur, kbeg + (st + 2) * GBK, 0, LD3);
            __builtin_amdgcn_sched_barrier(0);
        }
        __builtin_amdgcn_s_waitcnt(G_VMCNT(0));
        __builtin_amdgcn_s_barrier();
#undef GRAM_LOADS
#undef GRAM_MMA_LOADS
#undef GRAM_READ
    }
    // what the DMA path did not cover: the K tail of an interior item, or a
    // whole ragged/unaligned item, 32 samples at a time through registers
    // (LDS rows of 64 bytes, chunk c of row r at position c ^ ((r >> 2) & 3))
    for (int64_t k0 = kbeg + nfull * GBK; k0 < kend; k0 += GTK) {
        const uint16_t* A16 = (const uint16_t*)A;
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            const int q = tid + 256 * i;        // 16-byte slot in the operand buffer
            const int row = q >> 2;
            const int c = (q & 3) ^ ((row >> 2) & 3);
            uint32_t wa[4], wb[4];
#pragma unroll
            for (int e = 0; e < 4; ++e) {
                const int64_t k = k0 + c * 8 + 2 * e;
                const int64_t ga = r0 + row, gb = c0 + row;
                const uint32_t alo = (ga < n && k < kend) ? A16[ga * ld + k] : 0u;
                const uint32_t ahi = (ga < n && k + 1 < kend) ? A16[ga * ld + k + 1] : 0u;
                const uint32_t blo = (gb < n && k < kend) ? A16[gb * ld + k] : 0u;
                const uint32_t bhi = (gb < n && k + 1 < kend) ? A16[gb * ld + k + 1] : 0u;
                wa[e] = alo | (ahi << 16);
                wb[e] = blo | (bhi << 16);
            }
            *(uint4*)(smem + q * 16) = make_uint4(wa[0], wa[1], wa[2], wa[3]);
            *(uint4*)(smem + GT_OPB + q * 16) = make_uint4(wb[0], wb[1], wb[2], wb[3]);
        }
        __syncthreads();
        vec_t a0[4], b0[4], a1[4], b1[4];
#pragma unroll
        for (int x = 0; x < 4; ++x) {
            const int ra = wm * 128 + x * 32 + (lane & 31);
            const int rb = wn * 128 + x * 32 + (lane & 31);
            const int c = lane >> 5;
            const unsigned char* sA = smem;
            const unsigned char* sB = smem + GT_OPB;
            a0[x] = *(const vec_t*)(sA + ra * 64 + ((c ^ ((ra >> 2) & 3)) << 4));
            b0[x] = *(const vec_t*)(sB + rb * 64 + ((c ^ ((rb >> 2) & 3)) << 4));
            a1[x] = *(const vec_t*)(sA + ra * 64 + (((c + 2) ^ ((ra >> 2) & 3)) << 4));
            b1[x] = *(const vec_t*)(sB + rb * 64 + (((c + 2) ^ ((rb >> 2) & 3)) << 4));
        }
        GRAM_MMA(a0, b0);
        GRAM_MMA(a1, b1);
        __syncthreads();
    }
#undef GRAM_MMA

    float* out = part + (int64_t)wk.w * (GT * GT);
#pragma unroll
    for (int x = 0; x < 4; ++x)
#pragma unroll
        for (int y = 0; y < 4; ++y)
#pragma unroll
            for (int v = 0; v < 16; ++v) {
                const int row = wm * 128 + x * 32 + 8 * (v >> 2) + 4 * (lane >> 5) + (v & 3);
                const int col = wn * 128 + y * 32 + (lane & 31);
                out[row * GT + col] = acc[x][y][v];
            }
}

template <typename HT>
__global__ __launch_bounds__(256) void gram_lp256_kernel(int64_t n, int64_t K, int64_t kc_len,
                                                         const HT* __restrict__ A, int64_t ld,
                                                         float* __restrict__ part,
                                                         const int4* __restrict__ work) {
    gram_lp256_body<HT>(work[blockIdx.x], n, K, kc_len, A, ld, part);
}

// The same work items without a table: block b is split b / ntile, upper tile
// b % ntile, partial slot b (one launch covers every item in item order).
template <typename HT>
__global__ __launch_bounds__(256) void gram_lp256_direct_kernel(int64_t n, int64_t K, int64_t kc_len,
                                                                const HT* __restrict__ A, int64_t ld,
                                                                float* __restrict__ part, int64_t ntile) {
    const int64_t b = blockIdx.x;
    int bi, bj;
    tile_coords(b % ntile, bi, bj);
    gram_lp256_body<HT>(int4{(int)(b / ntile), bi, bj, (int)b}, n, K, kc_len, A, ld, part);
}

// M[i][j] = M[j][i] = sum over splits (in order, FP64) of the 256-tile partials;
// partial slot of (split s, tile t) is s * ntile + t.  A block sums one 32 x 32
// sub-tile (by: its position in the tile), writes its rows of M, and writes the
// mirrored rows from an LDS copy, so both stores are coalesced.
constexpr int RS = 32;                       // sub-tile of the partial sums
constexpr int RSUBS = (GT / RS) * (GT / RS); // sub-tiles per tile
__device__ __forceinline__ void gram_reduce256_body(int64_t bx, int64_t by, int64_t n,
                                                    const float* __restrict__ part, int64_t ntile,
                                                    int nsplit, double* __restrict__ M,
                                                    int64_t ldm) {
    __shared__ double sm[RS][RS + 1];
    int bi, bj;
    tile_coords(bx, bi, bj);
    const int sr = (int)(by / (GT / RS)), sc = (int)(by % (GT / RS));
    const int64_t r0 = (int64_t)bi * GT + sr * RS, c0 = (int64_t)bj * GT + sc * RS;
    // thread (row, quad): 4 consecutive columns of one row, read as 16 bytes
    // per split (the partial tiles are whole 256 x 256 arrays, so the quad is
    // in range even where the Gram is ragged); each element summed over the
    // splits in order, in FP64
    {
        const int row = threadIdx.x / (RS / 4), q4 = threadIdx.x % (RS / 4);  // 32 x 8 threads
        const int64_t gi = r0 + row;
        const int64_t e = (int64_t)(sr * RS + row) * GT + sc * RS + 4 * q4;  // first element within the tile
        double s[4] = {0.0, 0.0, 0.0, 0.0};
        if (gi < n && gi <= c0 + 4 * q4 + 3) {  // some column of the quad is kept
            for (int c = 0; c < nsplit; ++c) {
                const float4 v = *(const float4*)&part[((int64_t)c * ntile + bx) * (GT * GT) + e];
                s[0] += (double)v.x;
                s[1] += (double)v.y;
                s[2] += (double)v.z;
                s[3] += (double)v.w;
            }
        }
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            const int64_t gj = c0 + 4 * q4 + u;
            const bool on = gi < n && gj < n && gi <= gj;
            if (on) M[gi * ldm + gj] = s[u];
            sm[row][4 * q4 + u] = on ? s[u] : 0.0;
        }
    }
    __syncthreads();
    const int tx = threadIdx.x % RS, ty = threadIdx.x / RS;  // 32 x 8 threads
    for (int k = 0; k < RS; k += NT / RS) {
        const int col = ty + k;                 // sub-tile column: the mirrored row
        const int64_t gi = r0 + tx, gj = c0 + col;
        if (gi < n && gj < n && gi <= gj) M[gj * ldm + gi] = sm[tx][col];
    }
}

__global__ __launch_bounds__(NT) void gram_reduce256_kernel(int64_t n, const float* __restrict__ part,
                                                            int64_t ntile, int nsplit,
                                                            double* __restrict__ M, int64_t ldm) {
    gram_reduce256_body(blockIdx.x, blockIdx.y, n, part, ntile, nsplit, M, ldm);
}

__device__ __forceinline__ void diag_max_body(int64_t n, const double* __restrict__ M, int64_t ldm,
                                              double* __restrict__ out) {
    __shared__ double red[NT];
    double m = 0.0;
    bool nan = false;
    for (int64_t i = threadIdx.x; i < n; i += NT) {
        const double x = M[i * ldm + i];
        if (x != x || isinf(x)) nan = true;
        m = fmax(m, x);
    }
    red[threadIdx.x] = nan ? NAN : m;
    __syncthreads();
    for (int w = NT / 2; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) {
            const double a = red[threadIdx.x], b = red[threadIdx.x + w];
            red[threadIdx.x] = (a != a || b != b) ? NAN : fmax(a, b);
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) out[0] = red[0];
}

__global__ __launch_bounds__(NT) void diag_max_kernel(int64_t n, const double* __restrict__ M,
                                                      int64_t ldm, double* __restrict__ out) {
    diag_max_body(n, M, ldm, out);
}

// ---------------------------------------------------------------------------
// Grouped Grams of a batch (GramDesc): the blocks of a problem run over its
// work items exactly as its single launches would.
// ---------------------------------------------------------------------------
template <typename HT>
__global__ __launch_bounds__(256) void gram_lp256_grouped(const GramDesc* __restrict__ d,
                                                          GroupSched g) {
    int64_t lb;
    const GramDesc& q = d[group_problem(g, lb)];
    gram_lp256_body<HT>(q.work[lb], q.n, q.K, q.kc_len, (const HT*)q.A, q.ld, (float*)q.part);
}

template <typename T, bool KCONTIG>
__global__ __launch_bounds__(NT) void gram16_grouped(const GramDesc* __restrict__ d, GroupSched g) {
    int64_t lb;
    const GramDesc& q = d[group_problem(g, lb)];
    gram16_body<T, KCONTIG>(lb % q.ntile, lb / q.ntile, q.n, q.K, q.kc_len, (const T*)q.A, q.ld,
                            (T*)q.part, q.ntile);
}

template <int KIND>  // 0: 256-tile FP32 partials, 1: FP32 128-tile, 2: FP64 128-tile, 3: diagonal max
__global__ __launch_bounds__(NT) void gram_finish_grouped(const GramDesc* __restrict__ d,
                                                          GroupSched g) {
    int64_t lb;
    const GramDesc& q = d[group_problem(g, lb)];
    if constexpr (KIND == 0)
        gram_reduce256_body(lb % q.ntile, lb / q.ntile, q.n, (const float*)q.part, q.ntile, q.nsplit,
                            q.M, q.ldm);
    else if constexpr (KIND == 1)
        gram_reduce_body<float>(lb, q.n, (const float*)q.part, q.ntile, q.nsplit, q.M, q.ldm);
    else if constexpr (KIND == 2)
        gram_reduce_body<double>(lb, q.n, (const double*)q.part, q.ntile, q.nsplit, q.M, q.ldm);
    else
        diag_max_body(q.n, q.M, q.ldm, q.dmax);
}

}  // namespace

void launch_diag_max(hipStream_t s, int64_t n, const double* M, int64_t ldm, double* out) {
    diag_max_kernel<<<1, NT, 0, s>>>(n, M, ldm, out);
    ELM_LAUNCH_CHECK();
}

void launch_gram_f64_cols(hipStream_t s, int64_t N, int64_t L, const double* H, int64_t ldh,
                          double* M, int64_t ldm, Workspace& ws, int force_chunks) {
    run_gram_f64(s, L, N, H, ldh, false, M, ldm, ws, force_chunks);
}

void launch_gram_f64_rows(hipStream_t s, int64_t N, int64_t L, const double* H, int64_t ldh,
                          double* M, int64_t ldm, Workspace& ws) {
    run_gram_f64(s, N, L, H, ldh, true, M, ldm, ws, 0);
}

// Work table for the 256-tile Gram: items (split, bi, bj, slot) ordered by
// split, then by 4 x 8 patches of tiles, then dealt to XCDs in chunks of 32
// consecutive items (block b runs on XCD b % 8 as its (b / 8)-th block), so
// the blocks an XCD runs together cover one patch and share its panels in
// that XCD's L2.  b -> item = ((b/8)/32 * 8 + b%8) * 32 + (b/8)%32 is a
// bijection on [0, nb) for nb a multiple of 256.  Unused slots hold split = -1.
static std::vector<int4> gram_work_table(int64_t nt, int nsplit, int64_t ntile) {
    std::vector<int4> items;
    const int PI = 4, PJ = 8;
    for (int s = 0; s < nsplit; ++s)
        for (int64_t pj = 0; pj < nt; pj += PJ)
            for (int64_t pi = 0; pi <= pj + PJ - 1 && pi < nt; pi += PI)
                for (int64_t bj = pj; bj < std::min<int64_t>(pj + PJ, nt); ++bj)
                    for (int64_t bi = pi; bi < std::min<int64_t>(pi + PI, nt); ++bi) {
                        if (bi > bj) continue;
                        const int64_t t = bj * (bj + 1) / 2 + bi;
                        items.push_back(int4{s, (int)bi, (int)bj, (int)(s * ntile + t)});
                    }
    const int64_t nb = cdiv((int64_t)items.size(), 256) * 256;
    std::vector<int4> tab(nb, int4{-1, 0, 0, 0});
    for (int64_t b = 0; b < nb; ++b) {
        const int64_t xcd = b % 8, j = b / 8;
        const int64_t c = (j / 32) * 8 + xcd;
        const int64_t item = c * 32 + j % 32;
        if (item < (int64_t)items.size()) tab[b] = items[item];
    }
    return tab;
}

// splits of K: enough work items to fill 256 CUs in whole rounds
static int pick_splits(int64_t ntile, int64_t K) {
    if (ntile < 64) {
        // few tiles (small L): split K until about 256 blocks run, keeping
        // chunks of at least 512 samples; the partial tiles stay small
        int64_t s = (256 + ntile - 1) / ntile;
        const int64_t smax = std::max<int64_t>(1, std::min<int64_t>(64, K / 512));
        return (int)std::min(s, smax);
    }
    // Many tiles: chunks of about 24576 samples.  Shorter work items keep the
    // blocks that share panels closer in step (more L2 reuse) and shorten the
    // last, partly idle round; more splits cost one more 256 x 256 FP32
    // partial per tile each.  On L = 10000, N = 500000 the Gram kernel took
    // 55.9 ms with 4 splits, 51.3 with 10, 48.6 with 20 and 48.1 with 40 (the
    // partial sums 1.2, 1.4, 2.0 and 3.2 ms).  From that target, up to three
    // more splits are taken to fill the last round to 97%.
    const int64_t target = std::max<int64_t>(1, std::min<int64_t>(64, (K + 12288) / 24576));
    auto eff = [&](int64_t s) {
        const double items = (double)ntile * s;
        return items / (std::ceil(items / 256.0) * 256.0);
    };
    int64_t best = target;
    for (int64_t s = target; s <= std::min<int64_t>(64, target + 3); ++s)
        if (eff(s) >= 0.97) {
            best = s;
            break;
        }
    while (best > 1 && K / best < 2048) --best;
    return (int)best;
}

// K splits of the 16-bit Gram (ELM_GRAM_SPLITS, 1..64, overrides the choice)
static int gram_splits_override() {
    static const int v = [] {
        const char* e = std::getenv("ELM_GRAM_SPLITS");
        const int x = e ? std::atoi(e) : 0;
        return (x >= 1 && x <= 64) ? x : 0;
    }();
    return v;
}

int gram_default_splits(int64_t N, int64_t L) {
    const int64_t nt = cdiv(L, GT);
    return pick_splits(nt * (nt + 1) / 2, N);
}

int gram16_default_chunks(int dt, int64_t n, int64_t K) {
    const int64_t nt = cdiv(n, TILE);
    int64_t kc_len;
    int nchunk;
    default_chunks(dt, n, nt * (nt + 1) / 2, K, kc_len, nchunk);
    return nchunk;
}

// the work table of a 16-bit Gram of L nodes in nsplit_eff splits: it depends
// only on (L, splits), so it is built and uploaded once per workspace
static const int4* gram_table(hipStream_t s, int64_t L, int nsplit_eff, Workspace& ws,
                              size_t* nblocks_out) {
    const int64_t nt = cdiv(L, GT);
    const int64_t ntile = nt * (nt + 1) / 2;
    const std::string key = "gram_tab_" + std::to_string(L) + "_" + std::to_string(nsplit_eff);
    const size_t nwork = (size_t)ntile * nsplit_eff;
    const size_t nblocks = cdiv((int64_t)nwork, 256) * 256;
    int4* dtab = (int4*)ws.get(key, nblocks * sizeof(int4));
    if (!ws.has_table(key)) {
        std::vector<int4> tab = gram_work_table(nt, nsplit_eff, ntile);
        if (tab.size() != nblocks) throw Error{ELM_ERR_HIP, "Gram work table size mismatch"};
        ELM_HIP_TRY(hipMemcpyAsync(dtab, tab.data(), tab.size() * sizeof(int4), hipMemcpyHostToDevice, s));
        ELM_HIP_TRY(hipStreamSynchronize(s));  // tab is a host temporary
        ++ws.host_syncs;
        ws.tables.push_back(key);
    }
    *nblocks_out = nblocks;
    return dtab;
}

size_t gram_group_plan(hipStream_t s, elm_dtype dt, int64_t N, int64_t L, GramDesc& q,
                       Workspace& ws, int64_t* kc_out) {
    if (dt == ELM_BF16 || dt == ELM_F16) {  // launch_gram_lp_nodes' choices
        const int64_t nt = cdiv(L, GT);
        const int64_t ntile = nt * (nt + 1) / 2;
        int nsplit = gram_splits_override();
        if (nsplit <= 0) nsplit = ws.find_tune(ELM_TUNE_GRAM_SPLITS, (int)dt, L, N);
        if (nsplit <= 0) nsplit = pick_splits(ntile, N);
        const int64_t kc_len = cdiv(cdiv(N, nsplit), GBK) * GBK;
        const int nsplit_eff = (int)cdiv(N, kc_len);
        size_t nblocks = 0;
        q.work = gram_table(s, L, nsplit_eff, ws, &nblocks);
        q.kind = dt == ELM_BF16 ? GRAM_BF16 : GRAM_F16;
        q.n = L;
        q.K = N;
        q.kc_len = kc_len;
        q.ntile = ntile;
        q.nsplit = nsplit_eff;
        q.nblocks = (int64_t)nblocks;
        *kc_out = kc_len;
        return (size_t)ntile * nsplit_eff * GT * GT * sizeof(float);
    }
    // run_gram16's tiles and chunks (the FP64 route chunks alike)
    const int64_t nt = cdiv(L, TILE);
    const int64_t ntile = nt * (nt + 1) / 2;
    int64_t kc_len;
    int nchunk;
    gram16_chunks(dt == ELM_F32 ? ELM_F32 : ELM_F64, L, ntile, N, 0, ws, kc_len, nchunk);
    q.kind = dt == ELM_F32 ? GRAM_F32 : GRAM_F64;
    q.n = L;
    q.K = N;
    q.kc_len = kc_len;
    q.ntile = ntile;
    q.nsplit = nchunk;
    q.nblocks = ntile * nchunk;
    q.work = nullptr;
    *kc_out = kc_len;
    return (size_t)ntile * nchunk * TILE * TILE * (dt == ELM_F32 ? sizeof(float) : sizeof(double));
}

int64_t gram_group_blocks(int stage, const GramDesc& q) {
    if (stage == 0) return q.nblocks;
    if (stage == 1) return q.kind <= GRAM_F16 ? q.ntile * RSUBS : q.ntile;
    return 1;
}

void launch_gram_grouped(hipStream_t s, int stage, int kind, const GramDesc* d, const GroupSched& g) {
    if (g.count <= 0 || g.blocks <= 0) return;
    const unsigned grid = (unsigned)g.blocks;
    if (stage == 0) {
        switch (kind) {
            case GRAM_BF16: gram_lp256_grouped<__bf16><<<grid, 256, 0, s>>>(d, g); break;
            case GRAM_F16: gram_lp256_grouped<_Float16><<<grid, 256, 0, s>>>(d, g); break;
            case GRAM_F32: gram16_grouped<float, true><<<grid, NT, 0, s>>>(d, g); break;
            default: gram16_grouped<double, false><<<grid, NT, 0, s>>>(d, g); break;
        }
    } else if (stage == 1) {
        if (kind <= GRAM_F16) gram_finish_grouped<0><<<grid, NT, 0, s>>>(d, g);
        else if (kind == GRAM_F32) gram_finish_grouped<1><<<grid, NT, 0, s>>>(d, g);
        else gram_finish_grouped<2><<<grid, NT, 0, s>>>(d, g);
    } else {
        gram_finish_grouped<3><<<grid, NT, 0, s>>>(d, g);
    }
    ELM_LAUNCH_CHECK();
}

int64_t launch_gram_lp_nodes(hipStream_t s, elm_dtype dt, int64_t N, int64_t L, const void* Hn,
                             int64_t ldn, double* M, int64_t ldm, Workspace& ws, int force_splits) {
    if (dt == ELM_F32)
        return run_gram16<float, true>(s, L, N, (const float*)Hn, ldn, M, ldm, ws, force_splits);
    const int64_t nt = cdiv(L, GT);
    const int64_t ntile = nt * (nt + 1) / 2;
    int nsplit = force_splits;
    if (nsplit <= 0) nsplit = gram_splits_override();
    if (nsplit <= 0) nsplit = ws.find_tune(ELM_TUNE_GRAM_SPLITS, (int)dt, L, N);
    if (nsplit <= 0) nsplit = pick_splits(ntile, N);
    const int64_t kc_len = cdiv(cdiv(N, nsplit), GBK) * GBK;
    const int nsplit_eff = (int)cdiv(N, kc_len);
    size_t nblocks = 0;
    const int4* dtab = gram_table(s, L, nsplit_eff, ws, &nblocks);
    float* part = (float*)ws.get("gram_part", (size_t)ntile * nsplit_eff * GT * GT * sizeof(float));
    {
        StageScope sc(ws.prof, ELM_STAGE_GRAM, s);
        if (dt == ELM_BF16)
            gram_lp256_kernel<__bf16><<<(unsigned)nblocks, 256, 0, s>>>(L, N, kc_len, (const __bf16*)Hn, ldn,
                                                                        part, dtab);
        else
            gram_lp256_kernel<_Float16><<<(unsigned)nblocks, 256, 0, s>>>(L, N, kc_len, (const _Float16*)Hn, ldn,
                                                                          part, dtab);
        ELM_LAUNCH_CHECK();
    }
    StageScope sc(ws.prof, ELM_STAGE_GRAM_REDUCE, s);
    gram_reduce256_kernel<<<dim3((unsigned)ntile, RSUBS), NT, 0, s>>>(L, part, ntile, nsplit_eff,
                                                                            M, ldm);
    ELM_LAUNCH_CHECK();
    return kc_len;
}

// ---------------------------------------------------------------------------
// The Gram without device allocation (elm_gram_noalloc).  Its split-K partial
// tiles live in `scratch`, a file-scope device array that every GPU the
// library runs on holds until the process ends.  In host code the array's
// name is not a device address: its address on each device is looked up once
// (hipGetSymbolAddress, with that device current) and only that pointer is
// passed to kernels.  Every call on a GPU shares the array: calls that
// overlap on one GPU (several streams, several host threads) race.
// ---------------------------------------------------------------------------
static __device__ __align__(256) unsigned char scratch[GRAM_NOALLOC_SCRATCH_BYTES];

namespace {
constexpr int MAX_DEVICES = 64;
std::mutex g_scratch_mu;
void* g_scratch_ptr[MAX_DEVICES] = {};

// chunks of K for the 128-tile FP64/FP32 Gram: elm_gram's default count,
// lowered until ntile * nchunk partial tiles of `tile_bytes` fit in the scratch
bool fit_chunks(int dt, int64_t n, int64_t ntile, int64_t K, size_t tile_bytes, int64_t& kc_len,
                int& nchunk) {
    default_chunks(dt, n, ntile, K, kc_len, nchunk);
    for (int64_t nc = nchunk; nc >= 1; --nc) {
        kc_len = cdiv(cdiv(K, nc), 16) * 16;
        nchunk = (int)cdiv(K, kc_len);
        if ((size_t)ntile * nchunk * tile_bytes <= GRAM_NOALLOC_SCRATCH_BYTES) return true;
    }
    return false;
}
}  // namespace

void* noalloc_scratch(int device) {
    if (device < 0 || device >= MAX_DEVICES) throw Error{ELM_ERR_HIP, "device index out of range"};
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (!g_scratch_ptr[device]) {
        int cur = -1;
        ELM_HIP_TRY(hipGetDevice(&cur));
        if (cur != device) throw Error{ELM_ERR_HIP, "scratch lookup needs its device current"};
        void* p = nullptr;
        const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !p)
            throw Error{ELM_ERR_HIP, std::string("hipGetSymbolAddress(scratch): ") + hipGetErrorString(e)};
        g_scratch_ptr[device] = p;
    }
    return g_scratch_ptr[device];
}

void launch_gram_noalloc(hipStream_t s, int device, elm_dtype dt, int64_t N, int64_t L, const void* H,
                         int64_t ldh, double* M, int64_t ldm) {
    void* scr = noalloc_scratch(device);
    const bool transposed = N < L;
    if (dt == ELM_F64 || dt == ELM_F32) {
        // FP64 sample-major: columns (n = L, K = N) or rows (n = N, K = L);
        // FP32 node-major: n = L, K = N
        const int64_t n = transposed ? N : L, K = transposed ? L : N;
        const int64_t nt = cdiv(n, TILE);
        const int64_t ntile = nt * (nt + 1) / 2;
        const size_t tb = (size_t)TILE * TILE * (dt == ELM_F64 ? sizeof(double) : sizeof(float));
        int64_t kc_len;
        int nchunk;
        if (!fit_chunks(dt, n, ntile, K, tb, kc_len, nchunk))
            throw Error{ELM_ERR_SHAPE, "Gram order too large for the static scratch of elm_gram_noalloc"};
        dim3 grid((unsigned)ntile, (unsigned)nchunk);
        if (dt == ELM_F64) {
            double* part = (double*)scr;
            if (transposed)
                gram16_kernel<double, true><<<grid, NT, 0, s>>>(n, K, kc_len, (const double*)H, ldh, part, ntile);
            else
                gram16_kernel<double, false><<<grid, NT, 0, s>>>(n, K, kc_len, (const double*)H, ldh, part,
                                                                 ntile);
            ELM_LAUNCH_CHECK();
            gram_reduce_kernel<double><<<(unsigned)ntile, NT, 0, s>>>(n, part, ntile, nchunk, M, ldm);
        } else {
            float* part = (float*)scr;
            gram16_kernel<float, true><<<grid, NT, 0, s>>>(n, K, kc_len, (const float*)H, ldh, part, ntile);
            ELM_LAUNCH_CHECK();
            gram_reduce_kernel<float><<<(unsigned)ntile, NT, 0, s>>>(n, part, ntile, nchunk, M, ldm);
        }
        ELM_LAUNCH_CHECK();
        return;
    }
    // 16-bit node-major (n = L, K = N): the default split rule (or the
    // ELM_GRAM_SPLITS override), lowered until the partial tiles fit
    const int64_t nt = cdiv(L, GT);
    const int64_t ntile = nt * (nt + 1) / 2;
    const size_t tb = (size_t)GT * GT * sizeof(float);
    int nsplit = gram_splits_override();
    if (nsplit <= 0) nsplit = pick_splits(ntile, N);
    int64_t kc_len = 0;
    int nsplit_eff = 0;
    for (; nsplit >= 1; --nsplit) {
        kc_len = cdiv(cdiv(N, nsplit), GBK) * GBK;
        nsplit_eff = (int)cdiv(N, kc_len);
        if ((size_t)ntile * nsplit_eff * tb <= GRAM_NOALLOC_SCRATCH_BYTES) break;
    }
    if (nsplit < 1)
        throw Error{ELM_ERR_SHAPE, "Gram order too large for the static scratch of elm_gram_noalloc"};
    float* part = (float*)scr;
    const unsigned grid = (unsigned)(ntile * nsplit_eff);
    if (dt == ELM_BF16)
        gram_lp256_direct_kernel<__bf16><<<grid, 256, 0, s>>>(L, N, kc_len, (const __bf16*)H, ldh, part, ntile);
    else
        gram_lp256_direct_kernel<_Float16><<<grid, 256, 0, s>>>(L, N, kc_len, (const _Float16*)H, ldh, part, ntile);
    ELM_LAUNCH_CHECK();
    gram_reduce256_kernel<<<dim3((unsigned)ntile, RSUBS), NT, 0, s>>>(L, part, ntile, nsplit_eff, M, ldm);
    ELM_LAUNCH_CHECK();
}

}  // namespace elm
