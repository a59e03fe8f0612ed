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
    float dp2 = 0.f, dm2 = 0.f;
#pragma unroll
    for (int c = 0; c < kMaxCrit; ++c) {
        if (c >= nc) break;
        const float f = static_cast<float>(v[c]);
        const float a = f - ap[c], z = f - am[c];
        dp2 = fmaf(q[c] * a, a, dp2);
        dm2 = fmaf(q[c] * z, z, dm2);
    }
    const float dp = sqrtf(dp2), dm = sqrtf(dm2), den = dp + dm;
    return den > 0.f ? dm / den : 0.f;
}

// One workgroup per tile, N % 4 == 0 and N <= 4 * kTileBlock * IT: each
// thread loads its 4-server groups of every criterion once (16-byte loads,
// coalesced along the servers) and keeps them in registers for both passes,
// so the tile crosses HBM exactly once.
template <int C, int IT>
__global__ __launch_bounds__(kTileBlock) void k_topsis_tiles_reg(TileArgs a) {
    __shared__ int wst[5 * C * kTileWaves];
    __shared__ unsigned long long wkey[kTileWaves];
    const long long t = blockIdx.x;
    const int N = a.N;
    const int *x = a.x + static_cast<size_t>(t) * C * N;
    int4 v[C][IT];
#pragma unroll
    for (int it = 0; it < IT; ++it) {
        const int g = 4 * (it * kTileBlock + static_cast<int>(threadIdx.x));
#pragma unroll
        for (int c = 0; c < C; ++c)
            v[c][it] = g < N ? *reinterpret_cast<const int4 *>(x + static_cast<size_t>(c) * N + g) : make_int4(0, 0, 0, 0);
    }
    unsigned long long s2[kMaxCrit];
    int mx[kMaxCrit], mn[kMaxCrit];
#pragma unroll
    for (int c = 0; c < kMaxCrit; ++c) { s2[c] = 0; mx[c] = -kBig - 1; mn[c] = kBig; }
#pragma unroll
    for (int it = 0; it < IT; ++it) {
        if (4 * (it * kTileBlock + static_cast<int>(threadIdx.x)) >= N) break;
#pragma unroll
        for (int c = 0; c < C; ++c) {
            const int4 e = v[c][it];
            s2[c] += static_cast<unsigned long long>(static_cast<long long>(e.x) * e.x) +
                     static_cast<unsigned long long>(static_cast<long long>(e.y) * e.y) +
                     static_cast<unsigned long long>(static_cast<long long>(e.z) * e.z) +
                     static_cast<unsigned long long>(static_cast<long long>(e.w) * e.w);
            mx[c] = max(mx[c], max(max(e.x, e.y), max(e.z, e.w)));
            mn[c] = min(mn[c], min(min(e.x, e.y), min(e.z, e.w)));
        }
    }
    tile_stats(C, s2, mx, mn, wst);
    float q[kMaxCrit], ap[kMaxCrit], am[kMaxCrit];
    tile_factors(a, s2, mx, mn, q, ap, am);
    unsigned long long kb = 0;
#pragma unroll
    for (int it = 0; it < IT; ++it) {
        const int g = 4 * (it * kTileBlock + static_cast<int>(threadIdx.x));
        if (g >= N) break;
        unsigned fm = 0x01010101u;
        if (a.feas) fm = *reinterpret_cast<const unsigned *>(a.feas + static_cast<size_t>(t) * N + g);
        float sc[4];
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            int vv[C];
#pragma unroll
            for (int c = 0; c < C; ++c) vv[c] = j == 0 ? v[c][it].x : j == 1 ? v[c][it].y : j == 2 ? v[c][it].z : v[c][it].w;
            sc[j] = tile_close(C, vv, q, ap, am);
            if ((fm >> (8 * j)) & 0xffu) {
                const unsigned long long k = score_key(sc[j], g + j);
                kb = k > kb ? k : kb;
            }
        }
        if (a.scores)
            *reinterpret_cast<float4 *>(a.scores + static_cast<size_t>(t) * N + g) = make_float4(sc[0], sc[1], sc[2], sc[3]);
    }
    tile_select(a, t, kb, wkey);
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

}  // namespace dcs
