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

#include <type_traits>

namespace elm {
namespace {

constexpr int HT = 128;  // tile: 128 samples x 128 hidden nodes
constexpr int HK = 16;   // reduction chunk over input features
constexpr int NT = 512;  // 8 waves in 2 x 4, each a 64 x 32 sub-tile of 4 x 2 MFMA blocks
constexpr int WGN = 4;   // waves across the tile's columns
constexpr int JB = HT / WGN / 16;  // 16-column MFMA blocks per wave
constexpr int HE = HK * HT / NT;   // staged X (and W) values per thread and chunk
constexpr int XCDS = 8;  // blocks are dealt round-robin to the 8 XCDs
// LDS row pitch of the k-major operand tiles: 16 elements of padding put the
// 4 k rows one MFMA operand read touches on disjoint halves of the banks
constexpr int HP = HT + 16;

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

// low-precision bits of one value (round to nearest even through round-to-odd)
template <typename T>
__device__ inline uint16_t lp16_bits(elm_dtype lp, T v) {
    if (lp == ELM_BF16) return bf16_rne_bits(narrow_odd(v));
    return __half_as_ushort(__float2half_rn(narrow_odd(v)));
}

template <typename T>
struct HiddenSmem {
    static constexpr int LOOP = 2 * 2 * HK * HP * (int)sizeof(T);  // [buf][X|W][k][i]
    static constexpr int STAGE16 = HT * (HT + 8) * 2;                   // node-major 16-bit tile
    static constexpr int STAGE32 = HT * (HT + 4) * 4;                   // node-major FP32 tile
    static constexpr int ZT = 3 * HT * HIDDEN_Z_MAX_M * 8;                 // HᵀT partials + T rows
    static constexpr int B = LOOP > STAGE32 ? LOOP : STAGE32;
    static constexpr int BYTES = B > ZT ? B : ZT;
};

// Tile (row_t, col_t) of block b: XCD x = b % 8 owns the column tiles
// x, x + 8, ..., so its L2 keeps its strips of W (d x 128 each) for the whole
// launch while the X row tiles stream past; within an XCD the column tiles of
// one row tile are consecutive, so each X tile is read once per XCD.
__device__ inline bool hidden_tile(int64_t nrow_t, int64_t ncol_t, int64_t& row_t, int64_t& col_t) {
    const int64_t b = blockIdx.x;
    const int x = (int)(b % XCDS);
    const int64_t j = b / XCDS;
    const int64_t ncx = (ncol_t - x + XCDS - 1) / XCDS;
    if (ncx <= 0) return false;
    row_t = j / ncx;
    col_t = x + XCDS * (j % ncx);
    return row_t < nrow_t;
}

// node-major copy of a tile staged in LDS: each node's 128 samples are 256 B
// (16-bit) or 512 B (FP32), written in 16-byte pieces where the tile is whole
// and aligned
__device__ inline void store_node_major(void* __restrict__ Hlp, int64_t ldlp, bool lp16,
                                        const uint16_t* st16, const float* st32, int64_t N,
                                        int64_t L, int64_t n0, int64_t j0, int tid) {
    __syncthreads();
    const int esz = lp16 ? 2 : 4;
    const int per = 16 / esz;  // elements per 16-byte piece
    const bool vec = n0 + HT <= N && (((uintptr_t)Hlp | (uintptr_t)(ldlp * esz)) & 15) == 0;
    const int pieces = HT / per;  // per node
    for (int e = tid; e < HT * pieces; e += NT) {
        const int lj = e / pieces, q = e % pieces;
        const int64_t gj = j0 + lj;
        if (gj >= L) continue;
        const int64_t gi = n0 + q * per;
        if (vec) {
            const uint4 val = lp16 ? *(const uint4*)&st16[lj * (HT + 8) + q * per]
                                   : *(const uint4*)&st32[lj * (HT + 4) + q * per];
            *(uint4*)((char*)Hlp + (gj * ldlp + gi) * esz) = val;
        } else {
            for (int u = 0; u < per; ++u) {
                if (gi + u >= N) break;
                if (lp16)
                    ((uint16_t*)Hlp)[gj * ldlp + gi + u] = st16[lj * (HT + 8) + q * per + u];
                else
                    ((float*)Hlp)[gj * ldlp + gi + u] = st32[lj * (HT + 4) + q * per + u];
            }
        }
    }
}

// Partial Z = H^T T of one tile: Zp[j][c] = sum over the tile's rows i of
// H[i][j] T[i][c] (j local to the tile's columns, written at global column
// j0 + j), in a fixed order: each lane's 16 rows, then the four row groups of
// a wave by an xor butterfly, then the two waves' halves through LDS.
template <typename A>
__device__ inline void tile_ht_times_t(const A (&acc)[4][JB], const double* __restrict__ Tg,
                                       int64_t ldt, int m, double* __restrict__ Zp, int64_t N,
                                       int64_t L, int64_t n0, int64_t j0, unsigned char* smem) {
    constexpr int MZ = HIDDEN_Z_MAX_M;
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int wm = wave / WGN, wn = wave % WGN;
    double* zs = (double*)smem;         // [2][HT][MZ]
    double* ts = zs + 2 * HT * MZ;      // the tile's rows of T, [HT][MZ]
    __syncthreads();                    // the LDS staging is free
    for (int e = tid; e < HT * m; e += NT) {  // coalesced: T rows are m contiguous values
        const int r = e / m, c = e % m;
        const int64_t gi = n0 + r;
        ts[r * MZ + c] = gi < N ? Tg[gi * ldt + c] : 0.0;
    }
    __syncthreads();
    for (int c = 0; c < m; ++c) {
        double tv[4][4];
#pragma unroll
        for (int i = 0; i < 4; ++i)
#pragma unroll
            for (int v = 0; v < 4; ++v)
                tv[i][v] = ts[(wm * 64 + i * 16 + Mfma16<double>::row(lane, v)) * MZ + c];
#pragma unroll
        for (int j = 0; j < JB; ++j) {
            double z = 0.0;
#pragma unroll
            for (int i = 0; i < 4; ++i)
#pragma unroll
                for (int v = 0; v < 4; ++v) z += acc[i][j][v] * tv[i][v];
            z += __shfl_xor(z, 16);
            z += __shfl_xor(z, 32);
            if (lane < 16) zs[(wm * HT + wn * (HT / WGN) + j * 16 + lane) * MZ + c] = z;
        }
    }
    __syncthreads();
    for (int e = tid; e < HT * m; e += NT) {
        const int col = e / m, c = e % m;
        const int64_t gj = j0 + col;
        if (gj < L) Zp[gj * m + c] = zs[col * MZ + c] + zs[(HT + col) * MZ + c];
    }
}

template <typename T>
__device__ __forceinline__ void hidden_body(int64_t row_t, int64_t col_t, int64_t N, int64_t d,
                                            int64_t L, const T* __restrict__ X, int64_t ldx,
                                            const T* __restrict__ W, int64_t ldw,
                                            const T* __restrict__ bias, T* __restrict__ H,
                                            int64_t ldh, void* __restrict__ Hlp, int64_t ldlp,
                                            elm_dtype lp_dt, const double* __restrict__ Tg,
                                            int64_t ldt, int m, double* __restrict__ Zp) {
    __shared__ __align__(16) unsigned char smem[HiddenSmem<T>::BYTES];
    typedef T Tile[HK][HP];
    Tile* Xs = (Tile*)smem;  // Xs[buf]: k-major, so an MFMA A read is 16 consecutive samples
    Tile* Ws = Xs + 2;       // Ws[buf]

    const int64_t n0 = row_t * HT, j0 = col_t * HT;
    const int tid = threadIdx.x;
    const int lane = tid & 63;
    const int wave = tid >> 6;
    const int wm = wave / WGN, wn = wave % WGN;

    // global -> register staging: HE X values (one sample, HE consecutive
    // features) and HE W values (one feature, HE consecutive nodes) per thread
    static_assert(HE * NT == HK * HT && HT % HE == 0 && HK % HE == 0, "staging split");
    const int xr = tid / (HK / HE), xk = (tid % (HK / HE)) * HE;
    const int wk = tid / (HT / HE), wj = (tid % (HT / HE)) * HE;
    const int64_t gxr = n0 + xr;
    T xv[HE], wv[HE];
    auto load_chunk = [&](int64_t k0) {
#pragma unroll
        for (int e = 0; e < HE; ++e) {
            const int64_t k = k0 + xk + e;
            xv[e] = (gxr < N && k < d) ? X[gxr * ldx + k] : T(0);
        }
        const int64_t kw = k0 + wk;
#pragma unroll
        for (int e = 0; e < HE; ++e) {
            const int64_t j = j0 + wj + e;
            wv[e] = (kw < d && j < L) ? W[kw * ldw + j] : T(0);
        }
    };
    auto store_chunk = [&](int buf) {
#pragma unroll
        for (int e = 0; e < HE; ++e) Xs[buf][xk + e][xr] = xv[e];
#pragma unroll
        for (int e = 0; e < HE; ++e) Ws[buf][wk][wj + e] = wv[e];
    };

    typename Mfma16<T>::acc_t acc[4][JB];
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int j = 0; j < JB; ++j) acc[i][j] = typename Mfma16<T>::acc_t{};

    const int64_t nchunk = (d + HK - 1) / HK;
    load_chunk(0);
    store_chunk(0);
    __syncthreads();
    for (int64_t c = 0; c < nchunk; ++c) {
        const int buf = (int)(c & 1);
        const bool more = c + 1 < nchunk;
        if (more) load_chunk((c + 1) * HK);  // in flight during the MFMAs below
#pragma unroll
        for (int kk = 0; kk < HK; kk += 4) {
            const int k = kk + (lane >> 4);
            T a[4], bb[JB];
#pragma unroll
            for (int i = 0; i < 4; ++i) a[i] = Xs[buf][k][wm * 64 + i * 16 + (lane & 15)];
#pragma unroll
            for (int j = 0; j < JB; ++j) bb[j] = Ws[buf][k][wn * (HT / WGN) + j * 16 + (lane & 15)];
#pragma unroll
            for (int i = 0; i < 4; ++i)
#pragma unroll
                for (int j = 0; j < JB; ++j) acc[i][j] = Mfma16<T>::op(a[i], bb[j], acc[i][j]);
        }
        if (more) store_chunk(buf ^ 1);
        __syncthreads();
    }

    // epilogue: bias, sigmoid, the sample-major store, and the low-precision
    // values staged node-major in LDS (the loop buffers are free now)
    const bool lp16 = Hlp && lp_dt != ELM_F32;
    const bool lp32 = Hlp && lp_dt == ELM_F32;
    uint16_t* st16 = (uint16_t*)smem;  // [node][HT + 8]
    float* st32 = (float*)smem;        // [node][HT + 4]
#pragma unroll
    for (int j = 0; j < JB; ++j) {
        const int lj = wn * (HT / WGN) + j * 16 + (lane & 15);
        const int64_t gj = j0 + lj;
        const T bj_val = gj < L ? bias[gj] : T(0);
#pragma unroll
        for (int i = 0; i < 4; ++i) {
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                const int li = wm * 64 + i * 16 + Mfma16<T>::row(lane, v);
                const int64_t gi = n0 + li;
                const T h = sigmoid(acc[i][j][v] + bj_val);
                // not read again until the refinement: a streaming store
                if (H && gi < N && gj < L) __builtin_nontemporal_store(h, &H[gi * ldh + gj]);
                if (lp16) st16[lj * (HT + 8) + li] = lp16_bits<T>(lp_dt, h);
                if (lp32) st32[lj * (HT + 4) + li] = (float)h;
                acc[i][j][v] = h;
            }
        }
    }
    if (Hlp) store_node_major(Hlp, ldlp, lp16, st16, st32, N, L, n0, j0, tid);
    if constexpr (std::is_same<T, double>::value)
        if (Zp) tile_ht_times_t(acc, Tg, ldt, m, Zp + row_t * L * m, N, L, n0, j0, smem);
}

template <typename T>
__global__ __launch_bounds__(NT, 4) void hidden_kernel(int64_t N, int64_t d, int64_t L,
                                                       int64_t nrow_t, int64_t ncol_t,
                                                       const T* __restrict__ X, int64_t ldx,
                                                       const T* __restrict__ W, int64_t ldw,
                                                       const T* __restrict__ bias,
                                                       T* __restrict__ H, int64_t ldh,
                                                       void* __restrict__ Hlp, int64_t ldlp,
                                                       elm_dtype lp_dt, const double* __restrict__ Tg,
                                                       int64_t ldt, int m, double* __restrict__ Zp) {
    int64_t row_t, col_t;
    if (!hidden_tile(nrow_t, ncol_t, row_t, col_t)) return;
    hidden_body<T>(row_t, col_t, N, d, L, X, ldx, W, ldw, bias, H, ldh, Hlp, ldlp, lp_dt, Tg, ldt, m,
                   Zp);
}

// the hidden layers of a batch (FP64 inputs): the blocks of a problem run
// over its tiles, column tiles of a row tile consecutive
__global__ __launch_bounds__(NT, 4) void hidden_grouped(const HiddenDesc* __restrict__ dd,
                                                        GroupSched g) {
    int64_t lb;
    const HiddenDesc& q = dd[group_problem(g, lb)];
    const int64_t ncol_t = cdiv(q.L, HT);
    hidden_body<double>(lb / ncol_t, lb % ncol_t, q.N, q.d, q.L, q.X, q.ldx, q.W, q.ldw, q.b, q.H,
                        q.ldh, q.Hlp, q.ldlp, q.lp_dt, q.T, q.ldt, q.m, q.Zp);
}

}  // namespace

int64_t hidden_group_blocks(const HiddenDesc& q) { return cdiv(q.N, HT) * cdiv(q.L, HT); }

void launch_hidden_grouped(hipStream_t s, const HiddenDesc* d, const GroupSched& g) {
    if (g.count <= 0 || g.blocks <= 0) return;
    hidden_grouped<<<(unsigned)g.blocks, NT, 0, s>>>(d, g);
    ELM_LAUNCH_CHECK();
}

void launch_hidden(hipStream_t s, elm_dtype dt, int64_t N, int64_t d, int64_t L, const void* X,
                   int64_t ldx, const void* W, int64_t ldw, const void* b, void* H, int64_t ldh,
                   void* Hlp, int64_t ldlp, elm_dtype lp_dt, const double* T, int64_t ldt, int64_t m,
                   double* Zpart) {
    const int64_t nrow_t = cdiv(N, HT), ncol_t = cdiv(L, HT);
    const int64_t per_xcd = nrow_t * cdiv(ncol_t, XCDS);  // work items of the busiest XCD
    const unsigned grid = (unsigned)(XCDS * per_xcd);
    if (Zpart && (dt != ELM_F64 || m < 1 || m > HIDDEN_Z_MAX_M || !T))
        throw Error{ELM_ERR_INVALID_ARG, "fused H^T T needs FP64 inputs, T, and 1 <= m <= 8"};
    if (dt == ELM_F64) {
        hidden_kernel<double><<<grid, NT, 0, s>>>(N, d, L, nrow_t, ncol_t, (const double*)X, ldx,
                                                  (const double*)W, ldw, (const double*)b,
                                                  (double*)H, ldh, Hlp, ldlp, lp_dt, T, ldt, (int)m,
                                                  Zpart);
    } else {
        hidden_kernel<float><<<grid, NT, 0, s>>>(N, d, L, nrow_t, ncol_t, (const float*)X, ldx,
                                                 (const float*)W, ldw, (const float*)b, (float*)H,
                                                 ldh, Hlp, ldlp, lp_dt, nullptr, 0, 0, nullptr);
    }
    ELM_LAUNCH_CHECK();
}

int64_t hidden_row_tiles(int64_t N) { return cdiv(N, HT); }

}  // namespace elm
