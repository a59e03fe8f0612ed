// TOPSIS scoring and selection (section V-C) over a batch of decision
// matrices that are already in device memory: T tiles of C integer criteria
// by N servers, criterion-major.  Per tile: exact column statistics (sum of
// squares, maximum, minimum), the closeness of every server with the same
// FP32 arithmetic as the fused container step, and the feasible server of
// highest closeness, lowest index on ties.  This is the scoring stage of the
// step on its own: a streaming pass bound by HBM bandwidth.
#pragma once
#include "dc_step.hpp"

namespace dcs {

struct TileArgs {
    const int *x;                 // [T][C][N] criteria, 0 <= value < 2^22
    const unsigned char *feas;    // [T][N] feasibility (nonzero = feasible), or null: all feasible
    float *scores;                // [T][N] closeness, or null
    int *best;                    // [T] chosen server, -1 when none is feasible
    float *best_score;            // [T] its closeness (0 when none), or null
    int C, N;
    float w[kMaxCrit];
    int cost[kMaxCrit];
};

constexpr int kTileBlock = 256;
constexpr int kTileWaves = kTileBlock / kWave;

// Block totals of per-thread column statistics; every thread receives them.
// The 64-bit sums of squares travel as three 17-bit chunks (as in the fused
// step), so no partial sum can overflow.
__device__ __forceinline__ void tile_stats(int C, unsigned long long *s2, int *mx, int *mn, int *wst) {
    const int lane = threadIdx.x & (kWave - 1), wid = threadIdx.x / kWave;
#pragma unroll
    for (int c = 0; c < kMaxCrit; ++c) {
        if (c >= C) break;
        const int c0 = wave_sum(static_cast<int>(s2[c] & 0x1ffffu));
        const int c1 = wave_sum(static_cast<int>((s2[c] >> 17) & 0x1ffffu));
        const int c2 = wave_sum(static_cast<int>(s2[c] >> 34));
        const int hi = wave_max(mx[c]), lo = wave_min(mn[c]);
        if (lane < 5) wst[(5 * c + lane) * kTileWaves + wid] = lane == 0 ? c0 : lane == 1 ? c1 : lane == 2 ? c2
                                                                 : lane == 3 ? hi : -lo;
    }
    __syncthreads();
#pragma unroll
    for (int c = 0; c < kMaxCrit; ++c) {
        if (c >= C) break;
        int a0 = 0, a1 = 0, a2 = 0, hi = -kBig - 1, nlo = -kBig - 1;
#pragma unroll
        for (int x = 0; x < kTileWaves; ++x) {
            a0 += wst[(5 * c) * kTileWaves + x];
            a1 += wst[(5 * c + 1) * kTileWaves + x];
            a2 += wst[(5 * c + 2) * kTileWaves + x];
            hi = max(hi, wst[(5 * c + 3) * kTileWaves + x]);
            nlo = max(nlo, wst[(5 * c + 4) * kTileWaves + x]);
        }
        s2[c] = static_cast<unsigned long long>(static_cast<unsigned>(a0)) +
                (static_cast<unsigned long long>(static_cast<unsigned>(a1)) << 17) +
                (static_cast<unsigned long long>(static_cast<unsigned>(a2)) << 34);
        mx[c] = hi;
        mn[c] = -nlo;
    }
}

// Weighted normalisation folded into one factor per criterion, q = w^2 / S2,
// and the ideal / anti-ideal values (swapped for a cost criterion).
__device__ __forceinline__ void tile_factors(const TileArgs &a, const unsigned long long *s2, const int *mx,
                                             const int *mn, float *q, float *ap, float *am) {
#pragma unroll
    for (int c = 0; c < kMaxCrit; ++c) {
        q[c] = ap[c] = am[c] = 0.f;
        if (c >= a.C) continue;
        q[c] = s2[c] ? (a.w[c] * a.w[c]) / static_cast<float>(s2[c]) : 0.0f;
        ap[c] = static_cast<float>(a.cost[c] ? mn[c] : mx[c]);
        am[c] = static_cast<float>(a.cost[c] ? mx[c] : mn[c]);
    }
}

// Block argmax of the per-thread best keys; thread 0 writes the result.
__device__ __forceinline__ void tile_select(const TileArgs &a, long long t, unsigned long long kb,
                                            unsigned long long *wkey) {
    const int lane = threadIdx.x & (kWave - 1), wid = threadIdx.x / kWave;
    const unsigned hiw = wave_umax(static_cast<unsigned>(kb >> 32));
    const unsigned low = wave_umax(static_cast<unsigned>(kb >> 32) == hiw ? static_cast<unsigned>(kb) : 0u);
    if (lane == 0) wkey[wid] = (static_cast<unsigned long long>(hiw) << 32) | low;
    __syncthreads();
    if (threadIdx.x == 0) {
        unsigned long long best = 0;
#pragma unroll
        for (int x = 0; x < kTileWaves; ++x) best = wkey[x] > best ? wkey[x] : best;
        a.best[t] = best ? static_cast<int>(~static_cast<unsigned>(best)) : -1;
        if (a.best_score) a.best_score[t] = best ? __uint_as_float(static_cast<unsigned>(best >> 32) - 1u) : 0.f;
    }
}

__device__ __forceinline__ float tile_close(int nc, const int *v, const float *q, const float *ap, const float *am) {
    return topsis_close(nc, [&](int c) { return v[c]; }, q, ap, am);
}

// N % 4 == 0 and N <= 256 * V: one wavefront per tile, four per workgroup,
// walking tiles with a grid stride.  Lane l holds the 4-server groups
// l, l + 64, ..., l + 64 (V - 1) of every criterion in registers (16-byte
// loads, coalesced along the servers), so a tile crosses HBM exactly once;
// all reductions are wave DPP reductions, with no LDS and no barrier.
typedef int dcs_v4i __attribute__((ext_vector_type(4)));

template <int C, int V>
__global__ __launch_bounds__(kTileBlock) void k_topsis_tiles_wave(TileArgs a, long long T) {
    const int lane = threadIdx.x & (kWave - 1);
    const long long W = static_cast<long long>(gridDim.x) * kTileWaves;
    const int N = a.N;
    const size_t tile = static_cast<size_t>(C) * N;
    for (long long t = static_cast<long long>(blockIdx.x) * kTileWaves + threadIdx.x / kWave; t < T; t += W) {
        const int *x = a.x + t * tile;
        int4 v[C][V];
#pragma unroll
        for (int q = 0; q < V; ++q) {
            const int g = 4 * (q * kWave + lane);
#pragma unroll
            for (int c = 0; c < C; ++c) {
                int4 e = make_int4(0, 0, 0, 0);
                if (g < N) {
                    const dcs_v4i r = __builtin_nontemporal_load(
                        reinterpret_cast<const dcs_v4i *>(x + static_cast<size_t>(c) * N + g));
                    e = make_int4(r.x, r.y, r.z, r.w);
                }
                v[c][q] = e;
            }
        }
        // exact column statistics: per-lane 64-bit sums of squares (values
        // below 2^22, at most 4V <= 32 of them, so below 2^49), reduced as a
        // low 26-bit chunk (64 lanes sum below 2^32) and the rest
        unsigned long long s2[kMaxCrit];
        int mx[kMaxCrit], mn[kMaxCrit];
#pragma unroll
        for (int c = 0; c < kMaxCrit; ++c) { s2[c] = 0; mx[c] = -kBig - 1; mn[c] = kBig; }
#pragma unroll
        for (int q = 0; q < V; ++q) {
            if (4 * (q * kWave + lane) >= N) break;
#pragma unroll
            for (int c = 0; c < C; ++c) {
                const int4 e = v[c][q];
                const unsigned ex = e.x, ey = e.y, ez = e.z, ew = e.w;
                s2[c] += static_cast<unsigned long long>(ex) * ex;
                s2[c] += static_cast<unsigned long long>(ey) * ey;
                s2[c] += static_cast<unsigned long long>(ez) * ez;
                s2[c] += static_cast<unsigned long long>(ew) * ew;
                mx[c] = max(mx[c], max(max(e.x, e.y), max(e.z, e.w)));
                mn[c] = min(mn[c], min(min(e.x, e.y), min(e.z, e.w)));
            }
        }
#pragma unroll
        for (int c = 0; c < C; ++c) {
            const unsigned lo = static_cast<unsigned>(wave_sum(static_cast<int>(s2[c] & 0x3ffffffu)));
            const unsigned hi = static_cast<unsigned>(wave_sum(static_cast<int>(s2[c] >> 26)));
            s2[c] = static_cast<unsigned long long>(lo) + (static_cast<unsigned long long>(hi) << 26);
            mx[c] = wave_max(mx[c]);
            mn[c] = wave_min(mn[c]);
        }
        float q[kMaxCrit], ap[kMaxCrit], am[kMaxCrit];
        tile_factors(a, s2, mx, mn, q, ap, am);
        unsigned long long kb = 0;
#pragma unroll
        for (int qq = 0; qq < V; ++qq) {
            const int g = 4 * (qq * kWave + lane);
            if (g >= N) break;
            unsigned fm = 0x01010101u;
            if (a.feas) fm = *reinterpret_cast<const unsigned *>(a.feas + static_cast<size_t>(t) * N + g);
            float sc[4];
#pragma unroll
            for (int j = 0; j < 4; ++j) {
                int vv[C];
#pragma unroll
                for (int c = 0; c < C; ++c)
                    vv[c] = j == 0 ? v[c][qq].x : j == 1 ? v[c][qq].y : j == 2 ? v[c][qq].z : v[c][qq].w;
                sc[j] = tile_close(C, vv, q, ap, am);
                if ((fm >> (8 * j)) & 0xffu) {
                    const unsigned long long k = score_key(sc[j], g + j);
                    kb = k > kb ? k : kb;
                }
            }
            if (a.scores)
                *reinterpret_cast<float4 *>(a.scores + static_cast<size_t>(t) * N + g) =
                    make_float4(sc[0], sc[1], sc[2], sc[3]);
        }
        const unsigned hiw = wave_umax(static_cast<unsigned>(kb >> 32));
        const unsigned low = wave_umax(static_cast<unsigned>(kb >> 32) == hiw ? static_cast<unsigned>(kb) : 0u);
        if (lane == 0) {
            const unsigned long long best = (static_cast<unsigned long long>(hiw) << 32) | low;
            a.best[t] = best ? static_cast<int>(~low) : -1;
            if (a.best_score) a.best_score[t] = best ? __uint_as_float(hiw - 1u) : 0.f;
        }
    }
}

// Any shape: one workgroup per tile, two passes over the tile in global
// memory (the second pass mostly hits the caches).
__global__ __launch_bounds__(kTileBlock) void k_topsis_tiles_gen(TileArgs a) {
    __shared__ int wst[5 * kMaxCrit * kTileWaves];
    __shared__ unsigned long long wkey[kTileWaves];
    const long long t = blockIdx.x;
    const int N = a.N, C = a.C;
    const int *x = a.x + static_cast<size_t>(t) * C * N;
    unsigned long long s2[kMaxCrit];
    int mx[kMaxCrit], mn[kMaxCrit];
#pragma unroll
    for (int c = 0; c < kMaxCrit; ++c) { s2[c] = 0; mx[c] = -kBig - 1; mn[c] = kBig; }
    for (int u = threadIdx.x; u < N; u += kTileBlock) {
#pragma unroll
        for (int c = 0; c < kMaxCrit; ++c) {
            if (c >= C) break;
            const int e = x[static_cast<size_t>(c) * N + u];
            s2[c] += static_cast<unsigned long long>(static_cast<long long>(e) * e);
            mx[c] = max(mx[c], e);
            mn[c] = min(mn[c], e);
        }
    }
    tile_stats(C, s2, mx, mn, wst);
    float q[kMaxCrit], ap[kMaxCrit], am[kMaxCrit];
    tile_factors(a, s2, mx, mn, q, ap, am);
    unsigned long long kb = 0;
    for (int u = threadIdx.x; u < N; u += kTileBlock) {
        int vv[kMaxCrit];
#pragma unroll
        for (int c = 0; c < kMaxCrit; ++c) vv[c] = c < C ? x[static_cast<size_t>(c) * N + u] : 0;
        const float sc = tile_close(C, vv, q, ap, am);
        if (!a.feas || a.feas[static_cast<size_t>(t) * N + u]) {
            const unsigned long long k = score_key(sc, u);
            kb = k > kb ? k : kb;
        }
        if (a.scores) a.scores[static_cast<size_t>(t) * N + u] = sc;
    }
    tile_select(a, t, kb, wkey);
}

// ---------------------------------------------------------------- large tiles
// A few tiles of many servers (a large data center's matrix) would leave
// most of the device idle at one workgroup per tile, so each tile is split
// into slices of kSplitSlice servers, one workgroup each, and the
// reductions go through partials in scratch memory:
//   1. per slice, the exact column statistics -> sp.s2, sp.mx, sp.mn;
//   2. per slice, the tile's totals from all slices (in slice order), the
//      closeness of the slice's servers and the slice's best key -> sp.key;
//   3. per tile, the best key over its slices.
// The totals are exact integers, so the scores are bit-identical to the
// other paths.
constexpr int kSplitSlice = 2048;
constexpr long long kSplitMaxTiles = 1024;   // more tiles fill the device at one workgroup each

struct TileSplit {
    unsigned long long *s2;   // [T][S][C] slice sums of squares
    int *mx, *mn;             // [T][S][C] slice maxima / minima
    unsigned long long *key;  // [T][S] slice best keys
    int S;                    // slices per tile
};

// Scratch bytes of the split path for T tiles of N servers and C criteria
// (each region 256-byte aligned).
__host__ __device__ inline size_t split_scratch_bytes(long long T, int N, int C) {
    const long long S = (N + kSplitSlice - 1) / kSplitSlice;
    auto al = [](long long b) { return static_cast<size_t>((b + 255) & ~255LL); };
    return al(T * S * C * 8) + 2 * al(T * S * C * 4) + al(T * S * 8);
}

__host__ __device__ inline TileSplit split_carve(void *base, long long T, int N, int C) {
    const long long S = (N + kSplitSlice - 1) / kSplitSlice;
    auto al = [](long long b) { return static_cast<size_t>((b + 255) & ~255LL); };
    char *p = static_cast<char *>(base);
    TileSplit sp;
    sp.S = static_cast<int>(S);
    sp.s2 = reinterpret_cast<unsigned long long *>(p); p += al(T * S * C * 8);
    sp.mx = reinterpret_cast<int *>(p); p += al(T * S * C * 4);
    sp.mn = reinterpret_cast<int *>(p); p += al(T * S * C * 4);
    sp.key = reinterpret_cast<unsigned long long *>(p);
    return sp;
}

// grid (S, T): column statistics of slice blockIdx.x of tile blockIdx.y.
__global__ __launch_bounds__(kTileBlock) void k_tiles_split_stats(TileArgs a, TileSplit sp) {
    __shared__ int wst[5 * kMaxCrit * kTileWaves];
    const int s = blockIdx.x;
    const long long t = blockIdx.y;
    const int N = a.N, C = a.C, u0 = s * kSplitSlice, u1 = min(N, u0 + kSplitSlice);
    const int *x = a.x + static_cast<size_t>(t) * C * N;
    unsigned long long s2[kMaxCrit];
    int mx[kMaxCrit], mn[kMaxCrit];
#pragma unroll
    for (int c = 0; c < kMaxCrit; ++c) { s2[c] = 0; mx[c] = -kBig - 1; mn[c] = kBig; }
    for (int u = u0 + threadIdx.x; u < u1; u += kTileBlock) {
#pragma unroll
        for (int c = 0; c < kMaxCrit; ++c) {
            if (c >= C) break;
            const int e = x[static_cast<size_t>(c) * N + u];
            s2[c] += static_cast<unsigned long long>(static_cast<long long>(e) * e);
            mx[c] = max(mx[c], e);
            mn[c] = min(mn[c], e);
        }
    }
    tile_stats(C, s2, mx, mn, wst);
    if (threadIdx.x < C) {
        const int c = threadIdx.x;
        const size_t o = (static_cast<size_t>(t) * sp.S + s) * C + c;
#pragma unroll
        for (int cc = 0; cc < kMaxCrit; ++cc)
            if (cc == c) { sp.s2[o] = s2[cc]; sp.mx[o] = mx[cc]; sp.mn[o] = mn[cc]; }
    }
}

// grid (S, T): closeness of the slice's servers from the tile's totals, and
// the slice's best feasible key.
__global__ __launch_bounds__(kTileBlock) void k_tiles_split_score(TileArgs a, TileSplit sp) {
    __shared__ unsigned long long ts2[kMaxCrit];
    __shared__ int tmx[kMaxCrit], tmn[kMaxCrit];
    __shared__ unsigned long long wkey[kTileWaves];
    const int s = blockIdx.x;
    const long long t = blockIdx.y;
    const int N = a.N, C = a.C, u0 = s * kSplitSlice, u1 = min(N, u0 + kSplitSlice);
    if (threadIdx.x < C) {
        // tile totals over the slices in slice order (exact integers)
        const int c = threadIdx.x;
        unsigned long long v = 0;
        int hi = -kBig - 1, lo = kBig;
        for (int x = 0; x < sp.S; ++x) {
            const size_t o = (static_cast<size_t>(t) * sp.S + x) * C + c;
            v += sp.s2[o];
            hi = max(hi, sp.mx[o]);
            lo = min(lo, sp.mn[o]);
        }
        ts2[c] = v;
        tmx[c] = hi;
        tmn[c] = lo;
    }
    __syncthreads();
    unsigned long long s2[kMaxCrit];
    int mx[kMaxCrit], mn[kMaxCrit];
#pragma unroll
    for (int c = 0; c < kMaxCrit; ++c) {
        s2[c] = c < C ? ts2[c] : 0;
        mx[c] = c < C ? tmx[c] : 0;
        mn[c] = c < C ? tmn[c] : 0;
    }
    float q[kMaxCrit], ap[kMaxCrit], am[kMaxCrit];
    tile_factors(a, s2, mx, mn, q, ap, am);
    const int *x = a.x + static_cast<size_t>(t) * C * N;
    unsigned long long kb = 0;
    for (int u = u0 + threadIdx.x; u < u1; u += kTileBlock) {
        int vv[kMaxCrit];
#pragma unroll
        for (int c = 0; c < kMaxCrit; ++c) vv[c] = c < C ? x[static_cast<size_t>(c) * N + u] : 0;
        const float sc = tile_close(C, vv, q, ap, am);
        if (!a.feas || a.feas[static_cast<size_t>(t) * N + u]) {
            const unsigned long long k = score_key(sc, u);
            kb = k > kb ? k : kb;
        }
        if (a.scores) a.scores[static_cast<size_t>(t) * N + u] = sc;
    }
    const int lane = threadIdx.x & (kWave - 1), wid = threadIdx.x / kWave;
    const unsigned hiw = wave_umax(static_cast<unsigned>(kb >> 32));
    const unsigned low = wave_umax(static_cast<unsigned>(kb >> 32) == hiw ? static_cast<unsigned>(kb) : 0u);
    if (lane == 0) wkey[wid] = (static_cast<unsigned long long>(hiw) << 32) | low;
    __syncthreads();
    if (threadIdx.x == 0) {
        unsigned long long best = 0;
#pragma unroll
        for (int w = 0; w < kTileWaves; ++w) best = wkey[w] > best ? wkey[w] : best;
        sp.key[static_cast<size_t>(t) * sp.S + s] = best;
    }
}

// grid T, one wave: the tile's best key over its slices.
__global__ __launch_bounds__(kWave) void k_tiles_split_select(TileArgs a, TileSplit sp) {
    const long long t = blockIdx.x;
    unsigned long long kb = 0;
    for (int x = threadIdx.x; x < sp.S; x += kWave) {
        const unsigned long long k = sp.key[static_cast<size_t>(t) * sp.S + x];
        kb = k > kb ? k : kb;
    }
    const unsigned hiw = wave_umax(static_cast<unsigned>(kb >> 32));
    const unsigned low = wave_umax(static_cast<unsigned>(kb >> 32) == hiw ? static_cast<unsigned>(kb) : 0u);
    if (threadIdx.x == 0) {
        const unsigned long long best = (static_cast<unsigned long long>(hiw) << 32) | low;
        a.best[t] = best ? static_cast<int>(~low) : -1;
        if (a.best_score) a.best_score[t] = best ? __uint_as_float(hiw - 1u) : 0.f;
    }
}

}  // namespace dcs
