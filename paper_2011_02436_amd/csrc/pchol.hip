// Rank step of the RBP-ELM algorithm (Section 3, eq. 6; algorithm steps 3-4):
// a permutation P that puts r = rank(H) linearly independent columns first,
// found by a greedy diagonally pivoted Cholesky of the FP64 Gram,
//   P^T M P ~= R^T R,  R = [R11 R12] (r x n, upper trapezoidal).
// At step k the pivot is the remaining index with the largest Schur-complement
// diagonal, lowest original index on an exact tie; the factorisation stops
// when that diagonal is <= tau.
//
// GPU organisation (right-looking, blocked by panels of NB pivots):
//   panel_start   d = diag(S) of the current trailing matrix S, per-block argmax
//   step (x NB)   reduce the argmax partials -> pivot p; every remaining
//                 position a gets its panel row entry
//                   P[t][a] = (S[p][a] - sum_{t'<t} P[t'][p] P[t'][a]) / sqrt(d[p])
//                 and d[a] -= P[t][a]^2; new per-block argmax partials.  One
//                 launch per pivot: the kernel boundary is the grid-wide
//                 barrier that the exact greedy choice needs.
//   scatter       panel rows into R (columns by original index)
//   compact       drop the panel's pivots from the remaining-index list
//   trailing      S' = S[rem, rem] - P[:, rem]^T P[:, rem] on FP64 MFMA,
//                 upper tiles mirrored, written compacted
// After the last panel, `finalize` appends the rejected indices to the pivot
// order and `gather` permutes R's columns into pivot order.  Kernels read a
// device-side "done" flag first, so the host can enqueue every panel without
// waiting for the rank.
#include "elm_internal.h"

#include <algorithm>
#include <climits>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <cmath>

namespace elm {
namespace {

constexpr int PT = 256;     // threads per block, step kernels
constexpr int NB = 256;     // widest panel
static_assert(NB <= 8 * 32, "a step covers at most 8 groups of 32 panel rows");
constexpr int64_t MID_MAX = 4096;  // orders up to this use narrower panels
constexpr int TT = 128;     // trailing-update tile
enum { ST_DONE = 0, ST_RANK = 1, ST_BAD = 2, ST_CUR = 3, ST_NREM = 4, ST_N = 5 };

__device__ inline bool better(double v1, int o1, double v2, int o2) {
    return v1 > v2 || (v1 == v2 && o1 < o2);
}

// One argmax candidate: Schur diagonal v, original index o, position p.
struct __align__(16) Part {
    double v;
    int o;
    int p;
};

__device__ inline Part part_none() { return Part{-INFINITY, INT_MAX, -1}; }

__device__ inline void part_take(Part& b, const Part& x) {
    if (better(x.v, x.o, b.v, b.o)) b = x;
}

// all lanes of the wave end with the wave-wide best
__device__ inline void wave_argmax(Part& b) {
    for (int off = 32; off > 0; off >>= 1) {
        Part x;
        x.v = __shfl_xor(b.v, off);
        x.o = __shfl_xor(b.o, off);
        x.p = __shfl_xor(b.p, off);
        part_take(b, x);
    }
}

// block-wide best, written to out[bx] by thread 0.  `better` is a
// strict total order on (v, o) with distinct original indices, so the result
// does not depend on the combination order.
__device__ inline void block_argmax_store(Part b, Part* __restrict__ out, int bx) {
    __shared__ Part wbest[PT / 64];
    wave_argmax(b);
    if ((threadIdx.x & 63) == 0) wbest[threadIdx.x >> 6] = b;
    __syncthreads();
    if (threadIdx.x == 0) {
        Part r = wbest[0];
#pragma unroll
        for (int w = 1; w < PT / 64; ++w) part_take(r, wbest[w]);
        out[bx] = r;
    }
}

// pivot statistics: last accepted pivot, largest Schur diagonal at the stop
// (-inf when every position is accepted), largest Gram diagonal
enum { PS_LAST = 0, PS_REJECT = 1, PS_MAX = 2, PS_N = 3 };

__device__ __forceinline__ void init_body(int64_t a, int64_t n, int* rem0, int* state, double* pstats) {
    if (a < n) rem0[a] = (int)a;
    if (a < ST_N) state[a] = 0;
    if (a == 0) {
        pstats[PS_LAST] = INFINITY;
        pstats[PS_REJECT] = -INFINITY;
        pstats[PS_MAX] = 0.0;
    }
}

__global__ void fill_kernel(double* p, int64_t count, double v) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < count;
         i += (int64_t)gridDim.x * blockDim.x)
        p[i] = v;
}

__device__ __forceinline__ void panel_start_body(int bx, int64_t n_rem, const double* __restrict__ S,
                                        int64_t lds, double* __restrict__ d,
                                        int* __restrict__ chosen, const int* rem0, const int* rem1,
                                        Part* __restrict__ out, int* state) {
    if (state[ST_DONE]) return;
    const int* rem = state[ST_CUR] ? rem1 : rem0;
    const int64_t a = (int64_t)bx * PT + threadIdx.x;
    Part b = part_none();
    if (a < n_rem) {
        const double x = S[a * lds + a];
        d[a] = x;
        chosen[a] = 0;
        if (!isfinite(x)) state[ST_BAD] = 1;
        b = Part{x, rem[a], (int)a};
    }
    block_argmax_store(b, out, bx);
}

// One pivot.  G lanes share each remaining position a; lane group g holds
// panel rows [16 g, 16 g + 16) of the dot product
//   P[t][a] = (S[p][a] - sum_{q<t} P[q][p] P[q][a]) / sqrt(d[p]),
// so every lane issues at most 16 + 16 loads and the kernel is two dependent
// memory round trips: (flags, argmax partials, d, chosen, rem, P[.][a]) and,
// once the pivot p is known, (S[p][a], P[.][p]).  The partial sums are
// combined by an xor butterfly, so every lane holds the same bits and the
// order of operations is the same for every position: identical columns of
// the Gram stay bitwise identical.
template <int G, int R>
__device__ __forceinline__ void step_body(int bx, int64_t k, int t, int64_t n_rem,
                                 const double* __restrict__ S, int64_t lds, double* __restrict__ P,
                                 int64_t ldp, double* __restrict__ d, int* __restrict__ chosen,
                                 const int* rem0, const int* rem1, const Part* __restrict__ in,
                                 int nparts, Part* __restrict__ out, int* state, double tau,
                                 int* __restrict__ piv, double* __restrict__ pstats) {
    constexpr int CPW = 64 / G;  // positions per wave
    constexpr int CPB = CPW * (PT / 64);
    constexpr int PIN = 8;  // argmax partials per lane loaded in the first batch
    const int lane = threadIdx.x & 63;
    const int g = lane / CPW;
    const int64_t a = (int64_t)bx * CPB + (threadIdx.x >> 6) * CPW + lane % CPW;
    const int64_t ac = a < n_rem ? a : n_rem - 1;  // in-bounds twin for the batched loads
    const int q0 = R * g;

    // round trip 1: nothing here depends on the pivot
    const int done = state[ST_DONE];
    const int cur = state[ST_CUR];
    Part pin[PIN];
#pragma unroll
    for (int j = 0; j < PIN; ++j) {
        const int i = lane + 64 * j;
        pin[j] = i < nparts ? in[i] : part_none();
    }
    double y[R];
#pragma unroll
    for (int u = 0; u < R; ++u) y[u] = (q0 + u < t) ? P[(int64_t)(q0 + u) * ldp + ac] : 0.0;
    const double d_a = d[ac];
    const int ch = chosen[ac];
    const int ra = cur ? rem1[ac] : rem0[ac];

    Part best = part_none();
#pragma unroll
    for (int j = 0; j < PIN; ++j) part_take(best, pin[j]);
    for (int i = lane + 64 * PIN; i < nparts; i += 64) part_take(best, in[i]);
    if (done) return;
    wave_argmax(best);
    const int bp = __builtin_amdgcn_readfirstlane(best.p);
    const int bo = __builtin_amdgcn_readfirstlane(best.o);
    const double bv = best.v;
    if (!(bv > tau)) {  // largest remaining Schur diagonal at or below tau: rank = k
        if (bx == 0 && threadIdx.x == 0) {
            state[ST_RANK] = (int)k;
            state[ST_NREM] = (int)n_rem;
            state[ST_DONE] = 1;
            pstats[PS_REJECT] = bv;
            if (k == 0) pstats[PS_MAX] = bv;
        }
        return;
    }

    // round trip 2: the pivot's Schur row entry and panel column
    const double s0 = S[(int64_t)bp * lds + ac];
    double x[R];
#pragma unroll
    for (int u = 0; u < R; ++u) x[u] = (q0 + u < t) ? P[(int64_t)(q0 + u) * ldp + bp] : 0.0;
    double part = 0.0;
#pragma unroll
    for (int u = 0; u < R; ++u) part += x[u] * y[u];
#pragma unroll
    for (int off = CPW; off < 64; off <<= 1) part += __shfl_xor(part, off);

    const double rpp = sqrt(bv);
    Part cand = part_none();
    if (a < n_rem) {
        if (a == bp) {
            if (g == 0) {
                P[(int64_t)t * ldp + a] = rpp;
                chosen[a] = 1;
            }
        } else if (ch) {
            if (g == 0) P[(int64_t)t * ldp + a] = 0.0;
        } else {
            const double val = (s0 - part) / rpp;
            const double da = d_a - val * val;
            if (g == 0) {
                P[(int64_t)t * ldp + a] = val;
                d[a] = da;
                cand = Part{da, ra, (int)a};
            }
        }
    }
    block_argmax_store(cand, out, bx);
    if (bx == 0 && threadIdx.x == 0) {
        piv[k] = bo;
        pstats[PS_LAST] = bv;  // accepted pivots are non-increasing
        if (k == 0) pstats[PS_MAX] = bv;
    }
}

// panel rows -> R, columns by original index
__device__ __forceinline__ void scatter_body(int bx, int64_t t, int64_t ps, int nbp, int64_t n_rem,
                                    const double* __restrict__ P, int64_t ldp, const int* rem0,
                                    const int* rem1, double* __restrict__ Rorig, int64_t ldr,
                                    const int* state) {
    const int* rem = state[ST_CUR] ? rem1 : rem0;
    int64_t t_act = nbp;
    if (state[ST_DONE]) {
        t_act = (int64_t)state[ST_RANK] - ps;
        if (t_act < 0) t_act = 0;
        if (t_act > nbp) t_act = nbp;
    }
    if (t >= t_act) return;
    const int64_t a = (int64_t)bx * blockDim.x + threadIdx.x;
    if (a < n_rem) Rorig[(ps + t) * ldr + rem[a]] = P[t * ldp + a];
}

// Stable compaction of the positions whose flag is 0: out[j] = in[i], idx[j] = i.
// One block of 1024 threads; returns the count.
__device__ int64_t block_compact(int64_t n, const int* __restrict__ flag, const int* __restrict__ in,
                                 int* __restrict__ out, int* __restrict__ idx) {
    __shared__ int wsum[16];
    __shared__ int64_t base;
    if (threadIdx.x == 0) base = 0;
    __syncthreads();
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    for (int64_t c0 = 0; c0 < n; c0 += 1024) {
        const int64_t i = c0 + threadIdx.x;
        const int keep = (i < n && !flag[i]) ? 1 : 0;
        // inclusive scan within the wave
        int x = keep;
        for (int off = 1; off < 64; off <<= 1) {
            int y = __shfl_up(x, off);
            if (lane >= off) x += y;
        }
        if (lane == 63) wsum[w] = x;
        __syncthreads();
        int before = 0;
        for (int q = 0; q < w; ++q) before += wsum[q];
        int total = 0;
        for (int q = 0; q < 16; ++q) total += wsum[q];
        if (keep) {
            const int64_t j = base + before + x - 1;
            out[j] = in[i];
            if (idx) idx[j] = (int)i;
        }
        __syncthreads();
        if (threadIdx.x == 0) base += total;
        __syncthreads();
    }
    return base;
}

__device__ __forceinline__ void compact_body(int64_t n_rem, const int* __restrict__ chosen, int* rem0,
                                    int* rem1, int* __restrict__ map, int* state) {
    if (state[ST_DONE]) return;
    const int cur = state[ST_CUR];
    const int* in = cur ? rem1 : rem0;
    int* out = cur ? rem0 : rem1;
    block_compact(n_rem, chosen, in, out, map);
    __syncthreads();
    if (threadIdx.x == 0) state[ST_CUR] = cur ^ 1;
}

// tail of the pivot order: the rejected indices, in their current order
__device__ __forceinline__ void finalize_body(int64_t n, const int* __restrict__ chosen, const int* rem0,
                                     const int* rem1, int* __restrict__ piv, int* state) {
    if (!state[ST_DONE]) {
        if (threadIdx.x == 0) state[ST_RANK] = (int)n;
        return;
    }
    // chosen[] and the live index list still describe the panel that stopped
    const int* rem = state[ST_CUR] ? rem1 : rem0;
    const int64_t r = state[ST_RANK];
    block_compact(state[ST_NREM], chosen, rem, piv + r, nullptr);
}

// S'[a][b] = S[q(a)][q(b)] - sum_t P[t][q(a)] P[t][q(b)], upper TT x TT
// tiles, mirrored.  4 waves in 2 x 2, each (TT/2)^2 as 16 x 16 FP64 MFMA
// blocks; the panel rows are gathered through the compaction map into
// k-major LDS tiles, double-buffered through registers.
__device__ __forceinline__ void trailing_body(int bx, int64_t n_new, const double* __restrict__ S,
                                     int64_t lds, double* __restrict__ Sn, int64_t ldsn,
                                     const double* __restrict__ P, int64_t ldp, int nbp,
                                     const int* __restrict__ map, const int* state) {
    if (state[ST_DONE]) return;
    constexpr int BK = 16;
    constexpr int PP = TT + 16;           // LDS pitch: 4 k rows of an operand read on disjoint banks
    constexpr int EPT = TT * BK / 256;    // panel entries per thread per operand tile
    constexpr int WB = TT / 32;
    // operand tiles As[buf][k][i], Bs[buf][k][j]; reused for the mirror staging
    __shared__ double smem_tr[2 * 2 * BK * PP];
    typedef double OpTile[BK][PP];
    OpTile* As = (OpTile*)smem_tr;
    OpTile* Bs = As + 2;
    __shared__ int qa[TT], qb[TT];

    // tile index -> (bi <= bj)
    const int64_t tix = bx;
    int64_t c = (int64_t)((sqrt(8.0 * (double)tix + 1.0) - 1.0) * 0.5);
    while (c * (c + 1) / 2 > tix) --c;
    while ((c + 1) * (c + 2) / 2 <= tix) ++c;
    const int64_t bj = c, bi = tix - c * (c + 1) / 2;
    const int64_t r0 = bi * TT, c0 = bj * TT;

    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int wm = wave >> 1, wn = wave & 1;
    if (tid < TT) {
        qa[tid] = (r0 + tid < n_new) ? map[r0 + tid] : 0;
        qb[tid] = (c0 + tid < n_new) ? map[c0 + tid] : 0;
    }
    __syncthreads();

    // thread -> panel row k, positions i .. i + EPT - 1 of the tile
    const int lk = (tid * EPT) / TT, li0 = (tid * EPT) % TT;
    double av[EPT], bv[EPT];
    // qa/qb hold valid positions for every slot (slots past n_new read
    // position 0; their results are never stored), so only the panel row
    // needs masking, and only in a chunk that runs past nbp (block-uniform):
    // per-lane guarded loads would compile to branches that wait on each load
    auto load = [&](int k0) {
        if (k0 + BK <= nbp) {
            const double* prow = P + (int64_t)(k0 + lk) * ldp;
#pragma unroll
            for (int e = 0; e < EPT; ++e) {
                av[e] = prow[qa[li0 + e]];
                bv[e] = prow[qb[li0 + e]];
            }
        } else {
            const bool kin = k0 + lk < nbp;
            const double* prow = P + (int64_t)(kin ? k0 + lk : 0) * ldp;
#pragma unroll
            for (int e = 0; e < EPT; ++e) {
                av[e] = kin ? prow[qa[li0 + e]] : 0.0;
                bv[e] = kin ? prow[qb[li0 + e]] : 0.0;
            }
        }
    };
    auto store = [&](int buf) {
#pragma unroll
        for (int e = 0; e < EPT; ++e) {
            As[buf][lk][li0 + e] = av[e];
            Bs[buf][lk][li0 + e] = bv[e];
        }
    };

    d4v acc[WB][WB];
#pragma unroll
    for (int x = 0; x < WB; ++x)
#pragma unroll
        for (int y = 0; y < WB; ++y) acc[x][y] = d4v{};

    load(0);
    store(0);
    __syncthreads();
    int buf = 0;
    for (int k0 = 0; k0 < nbp; k0 += BK) {
        const bool more = k0 + BK < nbp;
        if (more) load(k0 + BK);
#pragma unroll
        for (int kk = 0; kk < BK; kk += 4) {
            const int k = kk + (lane >> 4);
            double a[WB], b[WB];
#pragma unroll
            for (int x = 0; x < WB; ++x) a[x] = As[buf][k][wm * (TT / 2) + x * 16 + (lane & 15)];
#pragma unroll
            for (int y = 0; y < WB; ++y) b[y] = Bs[buf][k][wn * (TT / 2) + y * 16 + (lane & 15)];
#pragma unroll
            for (int x = 0; x < WB; ++x)
#pragma unroll
                for (int y = 0; y < WB; ++y) acc[x][y] = Mfma16<double>::op(a[x], b[y], acc[x][y]);
        }
        if (more) store(buf ^ 1);
        __syncthreads();
        buf ^= 1;
    }
    // upper tile in place; its mirror goes through LDS (half a tile at a
    // time, in the free operand buffers) so that both are written as rows
    double (*Tm)[TT + 1] = (double (*)[TT + 1])smem_tr;  // [TT / 2][TT + 1]
    static_assert(sizeof(smem_tr) >= sizeof(double) * (TT / 2) * (TT + 1), "mirror staging");
#pragma unroll
    for (int x = 0; x < WB; ++x)
#pragma unroll
        for (int y = 0; y < WB; ++y)
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                const int li = wm * (TT / 2) + x * 16 + Mfma16<double>::row(lane, v);
                const int lj = wn * (TT / 2) + y * 16 + (lane & 15);
                const int64_t gi = r0 + li, gj = c0 + lj;
                const bool ok = gi < n_new && gj < n_new && gi <= gj;
                const double val = ok ? S[(int64_t)qa[li] * lds + qb[lj]] - acc[x][y][v] : 0.0;
                if (ok) Sn[gi * ldsn + gj] = val;
                acc[x][y][v] = val;
            }
    for (int h = 0; h < 2; ++h) {
        __syncthreads();  // the operand buffers (then the previous half) are free
        if (wn == h) {
#pragma unroll
            for (int x = 0; x < WB; ++x)
#pragma unroll
                for (int y = 0; y < WB; ++y)
#pragma unroll
                    for (int v = 0; v < 4; ++v) {
                        const int li = wm * (TT / 2) + x * 16 + Mfma16<double>::row(lane, v);
                        const int lj = y * 16 + (lane & 15);  // within the half
                        Tm[lj][li] = acc[x][y][v];
                    }
        }
        __syncthreads();
        for (int e = tid; e < (TT / 2) * TT; e += 256) {
            const int lr = e / TT, lc = e % TT;
            const int64_t gj = c0 + h * (TT / 2) + lr, gi = r0 + lc;  // mirror element (gj, gi)
            if (gj < n_new && gi < gj) Sn[gj * ldsn + gi] = Tm[lr][lc];
        }
    }
}

// ---------------------------------------------------------------------------
// Small Grams (n <= SMALL_N): the whole factorisation in one workgroup, so a
// pivot costs two block barriers instead of a kernel launch.  Same algorithm
// and pivot rule: S (a copy of M, positions = original indices, both
// triangles) takes a rank-SNB update after every SNB pivots; within a panel
// the pivot row is S[p][a] - sum_{t' < t} P[t'][p] P[t'][a] from the panel
// rows kept in LDS.  Writes R rows in original column order (Rorig), piv
// (accepted pivots), state[ST_RANK] and the pivot statistics.
// ---------------------------------------------------------------------------
constexpr int SMALL_N = 512;
constexpr int SNB = 16;
constexpr int SPT = 1024;

__device__ __forceinline__ void pchol_small_body(int n, const double* __restrict__ M, int64_t ldm,
                                        double* __restrict__ S, double tau, int32_t* __restrict__ piv,
                                        double* __restrict__ Rorig, int64_t ldr, int* state,
                                        double* pstats) {
    // No global store happens between the barriers of a pivot step (a
    // barrier waits for the block's outstanding stores): R rows, pivots and
    // statistics are written out per panel or at the end.
    __shared__ double P[SNB][SMALL_N];
    __shared__ double d[SMALL_N];
    __shared__ int chosen[SMALL_N];
    __shared__ int pivl[SMALL_N];
    __shared__ double wv[SPT / 64];
    __shared__ int wi[SPT / 64];
    __shared__ double s_v, st_last, st_reject, st_max;
    __shared__ int s_p, s_stop;
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    bool bad = false;
    for (int a = tid; a < n; a += SPT) {
        d[a] = M[(int64_t)a * ldm + a];
        chosen[a] = 0;
        if (!isfinite(d[a])) bad = true;
    }
    if (bad) state[ST_BAD] = 1;
    if (tid == 0) {
        st_last = INFINITY;
        st_reject = -INFINITY;
        st_max = 0.0;
        s_stop = 0;
    }
    __syncthreads();
    int k = 0;
    while (k < n) {
        const int k0 = k;
        const int nb = n - k < SNB ? n - k : SNB;
        // the first panel reads M itself; later panels the updated copy
        const double* Sc = k0 == 0 ? M : S;
        const int64_t lsc = k0 == 0 ? ldm : n;
        int t = 0;
        for (; t < nb; ++t) {
            // largest remaining Schur diagonal, lowest index on ties
            double bv = -INFINITY;
            int bi = INT_MAX;
            for (int a = tid; a < n; a += SPT)
                if (!chosen[a] && better(d[a], a, bv, bi)) { bv = d[a]; bi = a; }
            for (int off = 32; off > 0; off >>= 1) {
                const double v2 = __shfl_xor(bv, off);
                const int i2 = __shfl_xor(bi, off);
                if (better(v2, i2, bv, bi)) { bv = v2; bi = i2; }
            }
            if (lane == 0) { wv[wave] = bv; wi[wave] = bi; }
            __syncthreads();
            if (tid == 0) {
                for (int w = 1; w < SPT / 64; ++w)
                    if (better(wv[w], wi[w], bv, bi)) { bv = wv[w]; bi = wi[w]; }
                if (k == 0) st_max = bv;
                if (!(bv > tau)) {
                    s_stop = 1;
                    st_reject = bv;
                } else {
                    chosen[bi] = 1;
                    pivl[k] = bi;
                    st_last = bv;
                }
                s_v = bv;
                s_p = bi;
            }
            __syncthreads();
            if (s_stop) break;
            const int p = s_p;
            const double rpp = sqrt(s_v);
            for (int a = tid; a < n; a += SPT) {
                double val;
                if (a == p) {
                    val = rpp;
                } else if (chosen[a]) {
                    val = 0.0;
                } else {
                    double acc = Sc[(int64_t)p * lsc + a];
                    for (int q = 0; q < t; ++q) acc -= P[q][p] * P[q][a];
                    val = acc / rpp;
                    d[a] -= val * val;
                }
                P[t][a] = val;
            }
            ++k;
            __syncthreads();
        }
        // this panel's rows of R (original column order)
        for (int64_t e = tid; e < (int64_t)t * n; e += SPT) {
            const int q = (int)(e / n), a = (int)(e % n);
            Rorig[(int64_t)(k0 + q) * ldr + a] = P[q][a];
        }
        if (s_stop || k >= n) break;
        // S[a][b] -= sum_t P[t][a] P[t][b], in 4 x 4 blocks per thread (two
        // LDS reads per four products).  Entries of chosen positions are
        // updated too and never read again.
        const int n4 = (n + 3) >> 2;
        for (int blk = tid; blk < n4 * n4; blk += SPT) {
            const int a0 = (blk / n4) * 4, b0 = (blk % n4) * 4;
            double acc[4][4];
#pragma unroll
            for (int i = 0; i < 4; ++i)
#pragma unroll
                for (int j = 0; j < 4; ++j)
                    acc[i][j] = (a0 + i < n && b0 + j < n) ? Sc[(int64_t)(a0 + i) * lsc + b0 + j] : 0.0;
            for (int q = 0; q < t; ++q) {
                double pa[4], pb[4];
#pragma unroll
                for (int i = 0; i < 4; ++i) {
                    pa[i] = P[q][a0 + i];
                    pb[i] = P[q][b0 + i];
                }
#pragma unroll
                for (int i = 0; i < 4; ++i)
#pragma unroll
                    for (int j = 0; j < 4; ++j) acc[i][j] -= pa[i] * pb[j];
            }
#pragma unroll
            for (int i = 0; i < 4; ++i)
#pragma unroll
                for (int j = 0; j < 4; ++j)
                    if (a0 + i < n && b0 + j < n) S[(int64_t)(a0 + i) * n + b0 + j] = acc[i][j];
        }
        __syncthreads();
    }
    __syncthreads();
    for (int q = tid; q < k; q += SPT) piv[q] = pivl[q];
    if (tid == 0) {
        state[ST_RANK] = k;
        pstats[PS_LAST] = st_last;
        pstats[PS_REJECT] = st_reject;
        pstats[PS_MAX] = st_max;
        // the rejected positions follow the accepted pivots, in index order
        int j = k;
        for (int a = 0; a < n; ++a)
            if (!chosen[a]) piv[j++] = a;
    }
}

// ---------------------------------------------------------------------------
// One factorisation per launch
// ---------------------------------------------------------------------------
__global__ void init_kernel(int64_t n, int* rem0, int* state, double* pstats) {
    init_body((int64_t)blockIdx.x * blockDim.x + threadIdx.x, n, rem0, state, pstats);
}

__global__ __launch_bounds__(PT) void panel_start_kernel(int64_t n_rem, const double* __restrict__ S,
                                                         int64_t lds, double* __restrict__ d,
                                                         int* __restrict__ chosen, const int* rem0,
                                                         const int* rem1, Part* __restrict__ out,
                                                         int* state) {
    panel_start_body(blockIdx.x, n_rem, S, lds, d, chosen, rem0, rem1, out, state);
}

template <int G, int R>
__global__ __launch_bounds__(PT) void step_kernel(int64_t k, int t, int64_t n_rem,
                                                  const double* __restrict__ S, int64_t lds,
                                                  double* __restrict__ P, int64_t ldp,
                                                  double* __restrict__ d, int* __restrict__ chosen,
                                                  const int* rem0, const int* rem1,
                                                  const Part* __restrict__ in, int nparts,
                                                  Part* __restrict__ out, int* state, double tau,
                                                  int* __restrict__ piv, double* __restrict__ pstats) {
    step_body<G, R>(blockIdx.x, k, t, n_rem, S, lds, P, ldp, d, chosen, rem0, rem1, in, nparts, out,
                    state, tau, piv, pstats);
}

__global__ __launch_bounds__(PT) void scatter_kernel(int64_t ps, int nbp, int64_t n_rem,
                                                     const double* __restrict__ P, int64_t ldp,
                                                     const int* rem0, const int* rem1,
                                                     double* __restrict__ Rorig, int64_t ldr,
                                                     const int* state) {
    scatter_body(blockIdx.x, blockIdx.y, ps, nbp, n_rem, P, ldp, rem0, rem1, Rorig, ldr, state);
}

__global__ __launch_bounds__(1024) void compact_kernel(int64_t n_rem, const int* __restrict__ chosen,
                                                       int* rem0, int* rem1, int* __restrict__ map,
                                                       int* state) {
    compact_body(n_rem, chosen, rem0, rem1, map, state);
}

__global__ __launch_bounds__(1024) void finalize_kernel(int64_t n, const int* __restrict__ chosen,
                                                        const int* rem0, const int* rem1,
                                                        int* __restrict__ piv, int* state) {
    finalize_body(n, chosen, rem0, rem1, piv, state);
}

__global__ __launch_bounds__(256, 2) void trailing_kernel(int64_t n_new, const double* __restrict__ S,
                                                          int64_t lds, double* __restrict__ Sn,
                                                          int64_t ldsn, const double* __restrict__ P,
                                                          int64_t ldp, int nbp,
                                                          const int* __restrict__ map,
                                                          const int* state) {
    trailing_body(blockIdx.x, n_new, S, lds, Sn, ldsn, P, ldp, nbp, map, state);
}

__global__ __launch_bounds__(SPT) void pchol_small_kernel(int n, const double* __restrict__ M,
                                                          int64_t ldm, double* __restrict__ S,
                                                          double tau, int32_t* __restrict__ piv,
                                                          double* __restrict__ Rorig, int64_t ldr,
                                                          int* state, double* pstats) {
    pchol_small_body(n, M, ldm, S, tau, piv, Rorig, ldr, state, pstats);
}

// ---------------------------------------------------------------------------
// A group of independent factorisations per launch (blockIdx.y, or z for the
// two-dimensional scatter grid, selects the problem).  All problems follow
// the same panel schedule: panel j starts at position ps = j nb of every
// problem, a problem with n <= ps has finished, and one with fewer than nb
// remaining positions runs a shorter panel.  Each problem's arithmetic is
// the one-problem path's, in the same order.
// ---------------------------------------------------------------------------
struct GProb {
    const double* M;
    int64_t ldm, n;
    double* S[2];  // trailing matrices of alternate panels (ld n)
    double* P;     // panel rows, nb x n
    double* d;
    int *chosen, *rem0, *rem1, *map;
    Part* part[2];
    double* Rorig;  // n x n
    int* state;
    double* pstats;
    int32_t* piv;
    double tau;
};

// the trailing matrix that panel j reads
__device__ inline const double* panel_source(const GProb& q, int j, int64_t& lds) {
    lds = j == 0 ? q.ldm : q.n;
    return j == 0 ? q.M : q.S[(j - 1) & 1];
}

__global__ void init_grouped(const GProb* __restrict__ g) {
    const GProb& q = g[blockIdx.y];
    // one-workgroup problems keep no index list
    init_body((int64_t)blockIdx.x * blockDim.x + threadIdx.x, q.rem0 ? q.n : 0, q.rem0, q.state,
              q.pstats);
}

__global__ __launch_bounds__(PT) void panel_start_grouped(const GProb* __restrict__ g, int j, int nb) {
    const GProb& q = g[blockIdx.y];
    const int64_t n_rem = q.n - (int64_t)j * nb;
    if (n_rem <= 0 || (int64_t)blockIdx.x >= cdiv(n_rem, PT)) return;
    int64_t lds;
    const double* S = panel_source(q, j, lds);
    panel_start_body(blockIdx.x, n_rem, S, lds, q.d, q.chosen, q.rem0, q.rem1, q.part[0], q.state);
}

// prev_cpb: positions per block of the launch that wrote this step's argmax
// partials (uniform over the group: it depends on t only)
template <int G, int R>
__global__ __launch_bounds__(PT) void step_grouped(const GProb* __restrict__ g, int j, int nb, int t,
                                                   int prev_cpb) {
    const GProb& q = g[blockIdx.y];
    const int64_t ps = (int64_t)j * nb, n_rem = q.n - ps;
    if (n_rem <= 0 || t >= (n_rem < nb ? n_rem : nb)) return;
    if ((int64_t)blockIdx.x >= cdiv(n_rem, PT / G)) return;
    const int64_t k = ps + t;
    int64_t lds;
    const double* S = panel_source(q, j, lds);
    step_body<G, R>(blockIdx.x, k, t, n_rem, S, lds, q.P, q.n, q.d, q.chosen, q.rem0, q.rem1,
                    q.part[k & 1], (int)cdiv(n_rem, prev_cpb), q.part[(k + 1) & 1], q.state, q.tau,
                    q.piv, q.pstats);
}

__global__ __launch_bounds__(PT) void scatter_grouped(const GProb* __restrict__ g, int j, int nb) {
    const GProb& q = g[blockIdx.z];
    const int64_t ps = (int64_t)j * nb, n_rem = q.n - ps;
    if (n_rem <= 0) return;
    const int nbp = (int)(n_rem < nb ? n_rem : nb);
    if ((int64_t)blockIdx.y >= nbp) return;
    scatter_body(blockIdx.x, blockIdx.y, ps, nbp, n_rem, q.P, q.n, q.rem0, q.rem1, q.Rorig, q.n,
                 q.state);
}

__global__ __launch_bounds__(1024) void compact_grouped(const GProb* __restrict__ g, int j, int nb) {
    const GProb& q = g[blockIdx.y];
    const int64_t n_rem = q.n - (int64_t)j * nb;
    if (n_rem <= nb) return;  // no trailing matrix after this panel
    compact_body(n_rem, q.chosen, q.rem0, q.rem1, q.map, q.state);
}

__global__ __launch_bounds__(256, 2) void trailing_grouped(const GProb* __restrict__ g, int j, int nb) {
    const GProb& q = g[blockIdx.y];
    const int64_t n_new = q.n - (int64_t)j * nb - nb;
    if (n_new <= 0) return;
    const int64_t nt = cdiv(n_new, TT);
    if ((int64_t)blockIdx.x >= nt * (nt + 1) / 2) return;
    int64_t lds;
    const double* S = panel_source(q, j, lds);
    trailing_body(blockIdx.x, n_new, S, lds, q.S[j & 1], q.n, q.P, q.n, nb, q.map, q.state);
}

__global__ __launch_bounds__(1024) void finalize_grouped(const GProb* __restrict__ g) {
    const GProb& q = g[blockIdx.y];
    finalize_body(q.n, q.chosen, q.rem0, q.rem1, q.piv, q.state);
}

__global__ __launch_bounds__(SPT) void small_grouped(const GProb* __restrict__ g) {
    const GProb& q = g[blockIdx.x];
    pchol_small_body((int)q.n, q.M, q.ldm, q.S[0], q.tau, q.piv, q.Rorig, q.n, q.state, q.pstats);
}

__global__ void gather_kernel(int64_t r, int64_t n, const double* __restrict__ Rorig, int64_t ldro,
                              const int* __restrict__ piv, double* __restrict__ R, int64_t ldr) {
    const int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t t = blockIdx.y;
    if (c < n && t < r) R[t * ldr + c] = Rorig[t * ldro + piv[c]];
}

}  // namespace

// read back the rank and statistics, then R's columns into pivot order
static int64_t finish_pivoted_cholesky(hipStream_t s, int64_t n, const int32_t* piv,
                                       const double* Rorig, const int* state, const double* pstats,
                                       double** R_out, double* stats_out, elm_factor* f) {
    int hstate[ST_N];
    ELM_HIP_TRY(hipMemcpyAsync(hstate, state, sizeof(hstate), hipMemcpyDeviceToHost, s));
    ELM_HIP_TRY(hipMemcpyAsync(stats_out, pstats, PS_N * sizeof(double), hipMemcpyDeviceToHost, s));
    ELM_HIP_TRY(hipStreamSynchronize(s));
    if (hstate[ST_BAD]) throw Error{ELM_ERR_NOT_PSD, "Gram has a non-finite diagonal entry"};
    const int64_t r = hstate[ST_RANK];
    double* R = nullptr;
    if (r > 0) {
        R = (double*)factor_alloc(f, "R", (size_t)r * n * sizeof(double));
        gather_kernel<<<dim3((unsigned)cdiv(n, 256), (unsigned)r), 256, 0, s>>>(r, n, Rorig, n, piv,
                                                                                R, n);
        ELM_LAUNCH_CHECK();
    }
    *R_out = R;
    return r;
}

// Panel width.  Every pivot step re-reads its panel's rows (t of them at step
// t), every panel ends with a pass over the trailing matrix: orders up to
// MID_MAX take narrow panels (the re-read rows of many factorisations sharing
// the launches stay in the caches), larger ones NB.  ELM_MID_PANEL (32, 64,
// 128 or 256) overrides the narrow width for tuning.
static int panel_width(int64_t n, const Workspace& ws) {
    static const int mid_env = [] {
        if (const char* e = std::getenv("ELM_MID_PANEL")) {
            const int v = std::atoi(e);
            if (v == 32 || v == 64 || v == 128 || v == 256) return v;
        }
        return 64;
    }();
    if (n > MID_MAX) return NB;
    const int t = ws.find_tune(ELM_TUNE_PANEL, -1, -1, -1);   // the autotuner's width
    return t > 0 ? t : mid_env;
}

int64_t pivoted_cholesky(hipStream_t s, int64_t n, const double* M, int64_t ldm, double tau,
                         int32_t* piv, double** R_out, double* stats_out, Workspace& ws,
                         elm_factor* f) {
    const int pw = panel_width(n, ws);
    const int64_t nparts_max = cdiv(n, PT / 8);  // most blocks of any step launch
    int* state = (int*)ws.get("pc_state", ST_N * sizeof(int));
    double* pstats = (double*)ws.get("pc_stats", PS_N * sizeof(double));
    int* rem0 = (int*)ws.get("pc_rem0", n * sizeof(int));
    int* rem1 = (int*)ws.get("pc_rem1", n * sizeof(int));
    int* map = (int*)ws.get("pc_map", n * sizeof(int));
    int* chosen = (int*)ws.get("pc_chosen", n * sizeof(int));
    double* d = (double*)ws.get("pc_d", n * sizeof(double));
    double* P = (double*)ws.get("pc_P", (size_t)pw * n * sizeof(double));
    Part* parts = (Part*)ws.get("pc_parts", 2 * nparts_max * sizeof(Part));
    double* Rorig = (double*)ws.get("pc_Rorig", (size_t)n * n * sizeof(double));
    double* Sbuf[2] = {nullptr, nullptr};
    if (n > pw) {
        Sbuf[0] = (double*)ws.get("pc_S0", (size_t)n * n * sizeof(double));
        Sbuf[1] = (double*)ws.get("pc_S1", (size_t)n * n * sizeof(double));
    }
    Part* part[2] = {parts, parts + nparts_max};

    init_kernel<<<(unsigned)cdiv(n > ST_N ? n : ST_N, 256), 256, 0, s>>>(n, rem0, state, pstats);
    ELM_LAUNCH_CHECK();
    fill_kernel<<<1024, 256, 0, s>>>(Rorig, n * n, 0.0);
    ELM_LAUNCH_CHECK();
    if (n <= SMALL_N) {
        double* Sw = (double*)ws.get("pc_S0", (size_t)n * n * sizeof(double));
        pchol_small_kernel<<<1, SPT, 0, s>>>((int)n, M, ldm, Sw, tau, piv, Rorig, n, state, pstats);
        ELM_LAUNCH_CHECK();
        return finish_pivoted_cholesky(s, n, piv, Rorig, state, pstats, R_out, stats_out, f);
    }

    const double* Scur = M;
    int64_t lds = ldm;
    int which = 0;
    int64_t ps = 0, n_rem = n;
    while (ps < n) {
        const int nbp = (int)(n_rem < pw ? n_rem : pw);
        const int nblk = (int)cdiv(n_rem, PT);
        panel_start_kernel<<<nblk, PT, 0, s>>>(n_rem, Scur, lds, d, chosen, rem0, rem1, part[ps & 1],
                                                 state);
        ELM_LAUNCH_CHECK();
        int nparts = nblk;
        for (int t = 0; t < nbp; ++t) {
            const int64_t k = ps + t;
            Part* pin = part[k & 1];
            Part* pout = part[(k + 1) & 1];
            // lanes per position: enough 16-row groups to cover the t panel rows,
            // at most 8 (then 32 rows per lane)
            int g = 1;
            while (g < 8 && 16 * g < t) g *= 2;
            const int nb = (int)cdiv(n_rem, PT / g);
#define ELM_STEP(G, R)                                                                            \
    step_kernel<G, R><<<nb, PT, 0, s>>>(k, t, n_rem, Scur, lds, P, n, d, chosen, rem0, rem1, pin, \
                                        nparts, pout, state, tau, piv, pstats)
            if (g == 1) ELM_STEP(1, 16);
            else if (g == 2) ELM_STEP(2, 16);
            else if (g == 4) ELM_STEP(4, 16);
            else if (t <= 128) ELM_STEP(8, 16);
            else ELM_STEP(8, 32);
#undef ELM_STEP
            ELM_LAUNCH_CHECK();
            nparts = nb;
        }
        scatter_kernel<<<dim3((unsigned)nblk, (unsigned)nbp), PT, 0, s>>>(
            ps, nbp, n_rem, P, n, rem0, rem1, Rorig, n, state);
        ELM_LAUNCH_CHECK();
        const int64_t n_new = n_rem - nbp;
        if (n_new > 0) {
            compact_kernel<<<1, 1024, 0, s>>>(n_rem, chosen, rem0, rem1, map, state);
            ELM_LAUNCH_CHECK();
            double* Snew = Sbuf[which];
            const int64_t nt = cdiv(n_new, TT);
            trailing_kernel<<<(unsigned)(nt * (nt + 1) / 2), 256, 0, s>>>(n_new, Scur, lds, Snew, n,
                                                                          P, n, nbp, map, state);
            ELM_LAUNCH_CHECK();
            Scur = Snew;
            lds = n;
            which ^= 1;
        }
        ps += nbp;
        n_rem = n_new;
    }
    finalize_kernel<<<1, 1024, 0, s>>>(n, chosen, rem0, rem1, piv, state);
    ELM_LAUNCH_CHECK();
    return finish_pivoted_cholesky(s, n, piv, Rorig, state, pstats, R_out, stats_out, f);
}

void pivoted_cholesky_grouped(hipStream_t s, std::vector<PcholProblem>& probs, Workspace& ws) {
    const int count = (int)probs.size();
    if (count == 0) return;
    if (count > 65535) throw Error{ELM_ERR_UNSUPPORTED, "at most 65535 factorisations per group"};
    // large problems first (multi-block panels), then the one-workgroup ones
    std::vector<int> order(count);
    for (int e = 0; e < count; ++e) order[e] = e;
    std::stable_sort(order.begin(), order.end(), [&](int a, int b) { return probs[a].n > probs[b].n; });
    int nbig = 0, nlarge = 0;
    while (nbig < count && probs[order[nbig]].n > MID_MAX) ++nbig;
    nlarge = nbig;
    while (nlarge < count && probs[order[nlarge]].n > SMALL_N) ++nlarge;
    const int nsmall = count - nlarge;

    // one arena for the per-problem scratch, one for R (cleared in one fill)
    auto al = [](size_t b) { return (b + 255) & ~(size_t)255; };
    size_t scratch = 0, rbytes = 0;
    std::vector<size_t> off(count), roff(count);
    for (int i = 0; i < count; ++i) {
        const int64_t n = probs[order[i]].n;
        if (n < 1) throw Error{ELM_ERR_INVALID_ARG, "a grouped factorisation has n < 1"};
        const size_t nn = (size_t)n * n * sizeof(double);
        off[i] = scratch;
        scratch += al(nn) + al(n * sizeof(int32_t));  // S0, piv
        if (n > SMALL_N)
            scratch += al(nn) + al((size_t)panel_width(n, ws) * n * sizeof(double)) + al(n * sizeof(double)) +
                       4 * al(n * sizeof(int)) + 2 * al(cdiv(n, PT / 8) * sizeof(Part));
        roff[i] = rbytes;
        rbytes += al(nn);
    }
    char* arena = (char*)ws.get("gp_arena", scratch);
    char* rarena = (char*)ws.get("gp_rorig", rbytes);
    int* states = (int*)ws.get("gp_state", (size_t)count * ST_N * sizeof(int));
    double* stats = (double*)ws.get("gp_stats", (size_t)count * PS_N * sizeof(double));
    GProb* dg = (GProb*)ws.get("gp_desc", (size_t)count * sizeof(GProb));
    std::vector<GProb> hg(count);
    int64_t nmax = 0;
    for (int i = 0; i < count; ++i) {
        const PcholProblem& pr = probs[order[i]];
        const int64_t n = pr.n;
        const size_t nn = (size_t)n * n * sizeof(double);
        char* c = arena + off[i];
        auto take = [&](size_t b) {
            char* r = c;
            c += al(b);
            return r;
        };
        GProb& q = hg[i];
        std::memset(&q, 0, sizeof(q));
        q.M = pr.M;
        q.ldm = pr.ldm;
        q.n = n;
        q.tau = pr.tau;
        q.S[0] = (double*)take(nn);
        q.piv = (int32_t*)take(n * sizeof(int32_t));
        if (n > SMALL_N) {
            q.S[1] = (double*)take(nn);
            q.P = (double*)take((size_t)panel_width(n, ws) * n * sizeof(double));
            q.d = (double*)take(n * sizeof(double));
            q.chosen = (int*)take(n * sizeof(int));
            q.rem0 = (int*)take(n * sizeof(int));
            q.rem1 = (int*)take(n * sizeof(int));
            q.map = (int*)take(n * sizeof(int));
            q.part[0] = (Part*)take(cdiv(n, PT / 8) * sizeof(Part));
            q.part[1] = (Part*)take(cdiv(n, PT / 8) * sizeof(Part));
        }
        q.Rorig = (double*)(rarena + roff[i]);
        q.state = states + (size_t)i * ST_N;
        q.pstats = stats + (size_t)i * PS_N;
        nmax = std::max(nmax, n);
    }
    ELM_HIP_TRY(hipMemcpyAsync(dg, hg.data(), (size_t)count * sizeof(GProb), hipMemcpyHostToDevice, s));
    init_grouped<<<dim3((unsigned)cdiv(std::max<int64_t>(nmax, ST_N), 256), (unsigned)count), 256, 0,
                   s>>>(dg);
    ELM_LAUNCH_CHECK();
    launch_fill(s, (double*)rarena, (int64_t)(rbytes / sizeof(double)), 0.0);
    if (nsmall > 0) {
        small_grouped<<<(unsigned)nsmall, SPT, 0, s>>>(dg + nlarge);
        ELM_LAUNCH_CHECK();
    }
    // one chain of launches per panel width: orders above MID_MAX, then the
    // mid-size ones
    auto chain = [&](const GProb* dgs, int np, int64_t nmax_c, int nb) {
        if (np <= 0) return;
        const unsigned ny = (unsigned)np;
        for (int j = 0; (int64_t)j * nb < nmax_c; ++j) {
            const int64_t n_rem = nmax_c - (int64_t)j * nb;  // largest of the chain
            const int nbp = (int)(n_rem < nb ? n_rem : nb);
            panel_start_grouped<<<dim3((unsigned)cdiv(n_rem, PT), ny), PT, 0, s>>>(dgs, j, nb);
            ELM_LAUNCH_CHECK();
            int prev_cpb = PT;
            for (int t = 0; t < nbp; ++t) {
                int g = 1;
                while (g < 8 && 16 * g < t) g *= 2;
                const dim3 grid((unsigned)cdiv(n_rem, PT / g), ny);
#define ELM_GSTEP(G, R) step_grouped<G, R><<<grid, PT, 0, s>>>(dgs, j, nb, t, prev_cpb)
                if (g == 1) ELM_GSTEP(1, 16);
                else if (g == 2) ELM_GSTEP(2, 16);
                else if (g == 4) ELM_GSTEP(4, 16);
                else if (t <= 128) ELM_GSTEP(8, 16);
                else ELM_GSTEP(8, 32);
#undef ELM_GSTEP
                ELM_LAUNCH_CHECK();
                prev_cpb = PT / g;
            }
            scatter_grouped<<<dim3((unsigned)cdiv(n_rem, PT), (unsigned)nbp, ny), PT, 0, s>>>(dgs, j,
                                                                                           nb);
            ELM_LAUNCH_CHECK();
            const int64_t n_new = n_rem - nbp;
            if (n_new > 0) {
                compact_grouped<<<dim3(1, ny), 1024, 0, s>>>(dgs, j, nb);
                ELM_LAUNCH_CHECK();
                const int64_t nt = cdiv(n_new, TT);
                trailing_grouped<<<dim3((unsigned)(nt * (nt + 1) / 2), ny), 256, 0, s>>>(dgs, j, nb);
                ELM_LAUNCH_CHECK();
            }
        }
        finalize_grouped<<<dim3(1, ny), 1024, 0, s>>>(dgs);
        ELM_LAUNCH_CHECK();
    };
    // A chain's launches depend only on (descriptor address, problem count,
    // largest order, panel width): they are captured once into a HIP graph and
    // replayed, which takes the host's per-launch cost off the pivot steps.
    // Streams that cannot be captured (the legacy default stream, or one that
    // is capturing already) launch directly.
    hipStreamCaptureStatus cap = hipStreamCaptureStatusNone;
    const bool can_graph = s != nullptr && hipStreamIsCapturing(s, &cap) == hipSuccess &&
                           cap == hipStreamCaptureStatusNone;
    auto run_chain = [&](const GProb* dgs, int np, int64_t nmax_c, int nb) {
        if (!can_graph) {
            chain(dgs, np, nmax_c, nb);
            return;
        }
        char key[128];
        std::snprintf(key, sizeof(key), "pchol_chain:%p:%d:%lld:%d", (const void*)dgs, np,
                      (long long)nmax_c, nb);
        hipGraphExec_t exec = ws.find_graph(key);
        if (!exec) {
            ELM_HIP_TRY(hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal));
            hipGraph_t graph = nullptr;
            try {
                chain(dgs, np, nmax_c, nb);
            } catch (...) {
                (void)hipStreamEndCapture(s, &graph);
                if (graph) (void)hipGraphDestroy(graph);
                throw;
            }
            ELM_HIP_TRY(hipStreamEndCapture(s, &graph));
            const hipError_t ie = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
            (void)hipGraphDestroy(graph);
            if (ie != hipSuccess) throw Error{ELM_ERR_HIP, "graph instantiation of the pivot steps failed"};
            ws.put_graph(key, exec);
            ++ws.graph_captures;
        }
        ELM_HIP_TRY(hipGraphLaunch(exec, s));
        ++ws.graph_launches;
    };
    if (nbig > 0) run_chain(dg, nbig, probs[order[0]].n, panel_width(probs[order[0]].n, ws));
    if (nlarge > nbig)
        run_chain(dg + nbig, nlarge - nbig, probs[order[nbig]].n, panel_width(probs[order[nbig]].n, ws));
    std::vector<int> hstate((size_t)count * ST_N);
    std::vector<double> hstats((size_t)count * PS_N);
    ELM_HIP_TRY(hipMemcpyAsync(hstate.data(), states, hstate.size() * sizeof(int),
                               hipMemcpyDeviceToHost, s));
    ELM_HIP_TRY(hipMemcpyAsync(hstats.data(), stats, hstats.size() * sizeof(double),
                               hipMemcpyDeviceToHost, s));
    ELM_HIP_TRY(hipStreamSynchronize(s));
    ++ws.host_syncs;
    for (int i = 0; i < count; ++i) {
        PcholProblem& pr = probs[order[i]];
        pr.rank = hstate[(size_t)i * ST_N + ST_RANK];
        pr.bad = hstate[(size_t)i * ST_N + ST_BAD] != 0;
        for (int u = 0; u < PS_N; ++u) pr.stats[u] = hstats[(size_t)i * PS_N + u];
        pr.piv = hg[i].piv;
        pr.Rorig = hg[i].Rorig;
    }
}

void launch_gather_rows(hipStream_t s, int64_t r, int64_t n, const double* Rorig, int64_t ldro,
                        const int32_t* piv, double* R, int64_t ldr) {
    if (r <= 0 || n <= 0) return;
    gather_kernel<<<dim3((unsigned)cdiv(n, 256), (unsigned)r), 256, 0, s>>>(r, n, Rorig, ldro, piv, R,
                                                                            ldr);
    ELM_LAUNCH_CHECK();
}

void launch_fill(hipStream_t s, double* p, int64_t count, double v) {
    if (count <= 0) return;
    fill_kernel<<<(unsigned)std::min<int64_t>(cdiv(count, 256), 4096), 256, 0, s>>>(p, count, v);
    ELM_LAUNCH_CHECK();
}

}  // namespace elm
