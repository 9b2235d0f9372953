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

#include <climits>
#include <cmath>

namespace elm {
namespace {

constexpr int PT = 256;     // threads per block, step kernels
constexpr int NB = 128;     // panel width
constexpr int TT = 64;      // trailing-update tile
enum { ST_DONE = 0, ST_RANK = 1, ST_BAD = 2, ST_CUR = 3, ST_NREM = 4, ST_N = 5 };

__device__ inline bool better(double v1, int o1, double v2, int o2) {
    return v1 > v2 || (v1 == v2 && o1 < o2);
}

// all lanes of the wave end with the wave-wide best (v, o, p)
__device__ inline void wave_argmax(double& v, int& o, int& p) {
    for (int off = 32; off > 0; off >>= 1) {
        double v2 = __shfl_xor(v, off);
        int o2 = __shfl_xor(o, off);
        int p2 = __shfl_xor(p, off);
        if (better(v2, o2, v, o)) { v = v2; o = o2; p = p2; }
    }
}

struct Parts {
    double* v;
    int* o;
    int* p;
};

__global__ void init_kernel(int64_t n, int* rem0, int* state) {
    const int64_t a = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (a < n) rem0[a] = (int)a;
    if (a < ST_N) state[a] = 0;
}

__global__ void fill_kernel(double* p, int64_t count, double v) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < count;
         i += (int64_t)gridDim.x * blockDim.x)
        p[i] = v;
}

// partials are per wave: slot blockIdx.x * WPB + wave
constexpr int WPB = PT / 64;

__global__ __launch_bounds__(PT) void panel_start_kernel(int64_t n_rem, const double* __restrict__ S,
                                                         int64_t lds, double* __restrict__ d,
                                                         int* __restrict__ chosen, const int* rem0,
                                                         const int* rem1, Parts out, int* state) {
    if (state[ST_DONE]) return;
    const int* rem = state[ST_CUR] ? rem1 : rem0;
    const int64_t a = (int64_t)blockIdx.x * PT + threadIdx.x;
    double v = -INFINITY;
    int o = INT_MAX, p = -1;
    if (a < n_rem) {
        const double x = S[a * lds + a];
        d[a] = x;
        chosen[a] = 0;
        if (!isfinite(x)) state[ST_BAD] = 1;
        v = x; o = rem[a]; p = (int)a;
    }
    wave_argmax(v, o, p);
    if ((threadIdx.x & 63) == 0) {
        const int slot = blockIdx.x * WPB + (threadIdx.x >> 6);
        out.v[slot] = v; out.o[slot] = o; out.p[slot] = p;
    }
}

__global__ __launch_bounds__(PT) void step_kernel(int64_t k, int t, int64_t n_rem,
                                                  const double* __restrict__ S, int64_t lds,
                                                  double* __restrict__ P, int64_t ldp,
                                                  double* __restrict__ d, int* __restrict__ chosen,
                                                  const int* rem0, const int* rem1, Parts in,
                                                  int nparts, Parts out, int* state, double tau,
                                                  int* __restrict__ piv) {
    // The kernel is a chain of dependent memory round trips, so loads that do
    // not depend on each other are issued together: (flags, all partials),
    // then (S row entry, d, chosen, rem, the panel column).
    const int lane = threadIdx.x & 63;
    const int done = state[ST_DONE];
    const int cur = state[ST_CUR];
    // every wave reduces all of the previous launch's per-wave partials itself
    double pv[4];
    int po[4], pq[4];
#pragma unroll
    for (int j = 0; j < 4; ++j) {
        const int i = lane + 64 * j;
        const bool ok = i < nparts;
        pv[j] = ok ? in.v[i] : -INFINITY;
        po[j] = ok ? in.o[i] : INT_MAX;
        pq[j] = ok ? in.p[i] : -1;
    }
    double bv = -INFINITY;
    int bo = INT_MAX, bp = -1;
#pragma unroll
    for (int j = 0; j < 4; ++j)
        if (better(pv[j], po[j], bv, bo)) { bv = pv[j]; bo = po[j]; bp = pq[j]; }
    for (int i = lane + 256; i < nparts; i += 64)
        if (better(in.v[i], in.o[i], bv, bo)) { bv = in.v[i]; bo = in.o[i]; bp = in.p[i]; }
    if (done) return;
    wave_argmax(bv, bo, bp);
    bp = __builtin_amdgcn_readfirstlane(bp);
    bo = __builtin_amdgcn_readfirstlane(bo);
    if (!(bv > tau)) {  // largest remaining Schur diagonal at or below tau: rank = k
        if (blockIdx.x == 0 && threadIdx.x == 0) {
            state[ST_RANK] = (int)k;
            state[ST_NREM] = (int)n_rem;
            state[ST_DONE] = 1;
        }
        return;
    }
    const double rpp = sqrt(bv);
    const int64_t a = (int64_t)blockIdx.x * PT + threadIdx.x;
    const int64_t ac = a < n_rem ? a : n_rem - 1;  // in-bounds twin for the batched loads
    double s = S[(int64_t)bp * lds + ac];
    const double d_a = d[ac];
    const int ch = chosen[ac];
    const int ra = cur ? rem1[ac] : rem0[ac];
    // S[p][a] - sum_{q < t} P[q][p] P[q][a]; P[q][p] is the same for the whole
    // wave.  Chunks of 16 keep 32 loads in flight.
    const double* __restrict__ pa = P + ac;
    const double* __restrict__ pp = P + bp;
    int q = 0;
    for (; q + 16 <= t; q += 16) {
        double x[16], y[16];
#pragma unroll
        for (int u = 0; u < 16; ++u) {
            x[u] = pp[(int64_t)(q + u) * ldp];
            y[u] = pa[(int64_t)(q + u) * ldp];
        }
#pragma unroll
        for (int u = 0; u < 16; ++u) s -= x[u] * y[u];
    }
    for (; q < t; ++q) s -= pp[(int64_t)q * ldp] * pa[(int64_t)q * ldp];
    double v = -INFINITY;
    int o = INT_MAX, p = -1;
    if (a < n_rem) {
        if (a == bp) {
            P[(int64_t)t * ldp + a] = rpp;
            chosen[a] = 1;
        } else if (ch) {
            P[(int64_t)t * ldp + a] = 0.0;
        } else {
            const double val = s / rpp;
            P[(int64_t)t * ldp + a] = val;
            const double da = d_a - val * val;
            d[a] = da;
            v = da; o = ra; p = (int)a;
        }
    }
    wave_argmax(v, o, p);
    if (lane == 0) {
        const int slot = blockIdx.x * WPB + (threadIdx.x >> 6);
        out.v[slot] = v; out.o[slot] = o; out.p[slot] = p;
    }
    if (blockIdx.x == 0 && threadIdx.x == 0) piv[k] = bo;
}

// panel rows -> R, columns by original index
__global__ void scatter_kernel(int64_t ps, int nbp, int64_t n_rem, const double* __restrict__ P,
                               int64_t ldp, const int* rem0, const int* rem1, double* __restrict__ Rorig,
                               int64_t ldr, const int* state) {
    const int* rem = state[ST_CUR] ? rem1 : rem0;
    int64_t t_act = nbp;
    if (state[ST_DONE]) {
        t_act = (int64_t)state[ST_RANK] - ps;
        if (t_act < 0) t_act = 0;
        if (t_act > nbp) t_act = nbp;
    }
    const int64_t t = blockIdx.y;
    if (t >= t_act) return;
    const int64_t a = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
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

__global__ __launch_bounds__(1024) void compact_kernel(int64_t n_rem, const int* __restrict__ chosen,
                                                       int* rem0, int* rem1, int* __restrict__ map,
                                                       int* state) {
    if (state[ST_DONE]) return;
    const int cur = state[ST_CUR];
    const int* in = cur ? rem1 : rem0;
    int* out = cur ? rem0 : rem1;
    block_compact(n_rem, chosen, in, out, map);
    __syncthreads();
    if (threadIdx.x == 0) state[ST_CUR] = cur ^ 1;
}

// tail of the pivot order: the rejected indices, in their current order
__global__ __launch_bounds__(1024) void finalize_kernel(int64_t n,
                                                        const int* __restrict__ chosen,
                                                        const int* rem0, const int* rem1,
                                                        int* __restrict__ piv, int* state) {
    if (!state[ST_DONE]) {
        if (threadIdx.x == 0) state[ST_RANK] = (int)n;
        return;
    }
    // chosen[] and the live index list still describe the panel that stopped
    const int* rem = state[ST_CUR] ? rem1 : rem0;
    const int64_t r = state[ST_RANK];
    block_compact(state[ST_NREM], chosen, rem, piv + r, nullptr);
}

// S'[a][b] = S[q(a)][q(b)] - sum_t P[t][q(a)] P[t][q(b)], upper tiles, mirrored
__global__ __launch_bounds__(256) void trailing_kernel(int64_t n_new, const double* __restrict__ S,
                                                       int64_t lds, double* __restrict__ Sn,
                                                       int64_t ldsn, const double* __restrict__ P,
                                                       int64_t ldp, int nbp,
                                                       const int* __restrict__ map, const int* state) {
    if (state[ST_DONE]) return;
    constexpr int BK = 16;
    __shared__ double As[BK][TT + 1];
    __shared__ double Bs[BK][TT + 1];
    __shared__ int qa[TT], qb[TT];

    // tile index -> (bi <= bj)
    const int64_t tix = blockIdx.x;
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

    d4v acc[2][2];
    for (int x = 0; x < 2; ++x)
        for (int y = 0; y < 2; ++y) acc[x][y] = d4v{};

    for (int k0 = 0; k0 < nbp; k0 += BK) {
        for (int e = tid; e < BK * TT; e += 256) {
            const int k = e / TT, i = e % TT;
            const bool kin = (k0 + k) < nbp;
            As[k][i] = (kin && r0 + i < n_new) ? P[(int64_t)(k0 + k) * ldp + qa[i]] : 0.0;
            Bs[k][i] = (kin && c0 + i < n_new) ? P[(int64_t)(k0 + k) * ldp + qb[i]] : 0.0;
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
                const int li = wm * 32 + x * 16 + Mfma16<double>::row(lane, v);
                const int lj = wn * 32 + y * 16 + (lane & 15);
                const int64_t gi = r0 + li, gj = c0 + lj;
                if (gi >= n_new || gj >= n_new || gi > gj) continue;
                const double val = S[(int64_t)qa[li] * lds + qb[lj]] - acc[x][y][v];
                Sn[gi * ldsn + gj] = val;
                Sn[gj * ldsn + gi] = val;
            }
}

__global__ void gather_kernel(int64_t r, int64_t n, const double* __restrict__ Rorig, int64_t ldro,
                              const int* __restrict__ piv, double* __restrict__ R, int64_t ldr) {
    const int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t t = blockIdx.y;
    if (c < n && t < r) R[t * ldr + c] = Rorig[t * ldro + piv[c]];
}

}  // namespace

int64_t pivoted_cholesky(hipStream_t s, int64_t n, const double* M, int64_t ldm, double tau,
                         int32_t* piv, double** R_out, Workspace& ws) {
    const int64_t nparts_max = cdiv(n, PT) * WPB;
    int* state = (int*)ws.get("pc_state", ST_N * sizeof(int));
    int* rem0 = (int*)ws.get("pc_rem0", n * sizeof(int));
    int* rem1 = (int*)ws.get("pc_rem1", n * sizeof(int));
    int* map = (int*)ws.get("pc_map", n * sizeof(int));
    int* chosen = (int*)ws.get("pc_chosen", n * sizeof(int));
    double* d = (double*)ws.get("pc_d", n * sizeof(double));
    double* P = (double*)ws.get("pc_P", (size_t)NB * n * sizeof(double));
    double* pv = (double*)ws.get("pc_pv", 2 * nparts_max * sizeof(double));
    int* po = (int*)ws.get("pc_po", 2 * nparts_max * sizeof(int));
    int* pp = (int*)ws.get("pc_pp", 2 * nparts_max * sizeof(int));
    double* Rorig = (double*)ws.get("pc_Rorig", (size_t)n * n * sizeof(double));
    double* Sbuf[2] = {nullptr, nullptr};
    if (n > NB) {
        Sbuf[0] = (double*)ws.get("pc_S0", (size_t)n * n * sizeof(double));
        Sbuf[1] = (double*)ws.get("pc_S1", (size_t)n * n * sizeof(double));
    }
    Parts part[2] = {{pv, po, pp}, {pv + nparts_max, po + nparts_max, pp + nparts_max}};

    init_kernel<<<(unsigned)cdiv(n > ST_N ? n : ST_N, 256), 256, 0, s>>>(n, rem0, state);
    ELM_LAUNCH_CHECK();
    fill_kernel<<<1024, 256, 0, s>>>(Rorig, n * n, 0.0);
    ELM_LAUNCH_CHECK();

    const double* Scur = M;
    int64_t lds = ldm;
    int which = 0;
    int64_t ps = 0, n_rem = n;
    while (ps < n) {
        const int nbp = (int)(n_rem < NB ? n_rem : NB);
        const int nblk = (int)cdiv(n_rem, PT);
        const int nparts = nblk * WPB;
        panel_start_kernel<<<nblk, PT, 0, s>>>(n_rem, Scur, lds, d, chosen, rem0, rem1,
                                                 part[ps & 1], state);
        ELM_LAUNCH_CHECK();
        for (int t = 0; t < nbp; ++t) {
            const int64_t k = ps + t;
            step_kernel<<<nblk, PT, 0, s>>>(k, t, n_rem, Scur, lds, P, n, d, chosen, rem0, rem1,
                                              part[k & 1], nparts, part[(k + 1) & 1], state, tau,
                                              piv);
            ELM_LAUNCH_CHECK();
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

    int hstate[ST_N];
    ELM_HIP_TRY(hipMemcpyAsync(hstate, state, sizeof(hstate), hipMemcpyDeviceToHost, s));
    ELM_HIP_TRY(hipStreamSynchronize(s));
    if (hstate[ST_BAD]) throw Error{ELM_ERR_NOT_PSD, "Gram has a non-finite diagonal entry"};
    const int64_t r = hstate[ST_RANK];
    double* R = nullptr;
    if (r > 0) {
        ELM_HIP_TRY(hipMalloc(&R, (size_t)r * n * sizeof(double)));
        gather_kernel<<<dim3((unsigned)cdiv(n, 256), (unsigned)r), 256, 0, s>>>(r, n, Rorig, n, piv,
                                                                                R, n);
        ELM_LAUNCH_CHECK();
    }
    *R_out = R;
    return r;
}

void launch_fill(hipStream_t s, double* p, int64_t count, double v) {
    if (count <= 0) return;
    fill_kernel<<<(unsigned)std::min<int64_t>(cdiv(count, 256), 4096), 256, 0, s>>>(p, count, v);
    ELM_LAUNCH_CHECK();
}

}  // namespace elm
