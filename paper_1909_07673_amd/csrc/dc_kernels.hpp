// Kernels of libdcsched (gfx950).  The per-step device code they share is in
// dc_step.hpp; this header is included by the single library translation
// unit (dc_lib.hip).
#pragma once
#include "dc_step.hpp"

namespace dcs {

struct Params {
    Topo t;
    State st;        // state of the instance the kernel works on (plain, release)
    Method m;
    Batch b;
    Trace tr;
    int *xs;         // global host scratch [(nc+4)][N] of that instance
    int pc_cap;      // peers per path-table chunk
    int inst;
    // batched form: state of instance i at state_base + i * state_stride
    int *state_base;
    long long state_stride;
    // AHP
    int *colpart;    // [nc][nI][N]
    float *rowpart;  // [nc][nJ][N]
    int ti, tj, nI, nJ;
    int r, i;        // request and container of a plain step
};

constexpr int kAhpBlock = 256;
constexpr int kAhpTile = 1024;   // values staged per LDS tile in the AHP passes
constexpr int kAhpAcc = 8;       // independent partial sums per row in pass B

// Dynamic LDS of the single-workgroup step.
inline size_t step_lds_bytes(int pc_cap, int nsw, size_t xs_ints, size_t state_ints) {
    return smem_fixed_bytes() + sizeof(int) * (2 * (size_t)pc_cap * nsw + xs_ints + state_ints);
}

__device__ __forceinline__ State state_at(int *base, long long stride, int inst, int N) {
    int *s = base + stride * inst;
    return State{s, s + N, s + 2 * N, s + 3 * N, s + 4 * N, s + 5 * N};
}

// ---------------------------------------------------------------- plain form
// One launch per container step, one workgroup; xs in LDS when XL.
template <int BS, bool XL>
__global__ __launch_bounds__(BS) void k_topsis_plain(Params p) {
    extern __shared__ __align__(16) char dsm[];
    Smem sm = carve(dsm, p.pc_cap, p.t.nsw);
    int *xs = XL ? reinterpret_cast<int *>(dsm + smem_fixed_bytes() + sizeof(int) * 2 * p.pc_cap * p.t.nsw) : p.xs;
    topsis_step<BS>(p.t, p.st, p.m, p.b, sm, xs, p.pc_cap, p.tr, p.inst, p.r, p.i);
}

// AHP step, stage 1: criteria of every server into the global xs rows.
template <int BS>
__global__ __launch_bounds__(BS) void k_criteria_plain(Params p) {
    extern __shared__ __align__(16) char dsm[];
    if (p.b.status[p.r] == 0) return;
    if (p.i == 0 && threadIdx.x == 0) p.b.tsb[p.r] = dev_clock();
    Smem sm = carve(dsm, p.pc_cap, p.t.nsw);
    const int g0 = p.b.coff[p.r], g = g0 + p.i;
    const int P = load_peers<BS>(p.st, p.b, sm, g0, g);
    criteria_stage<BS, false>(p.t, p.st, p.m, sm, p.xs, p.b.cpu[g], p.b.ram[g], P, p.pc_cap,
                              nullptr, nullptr, nullptr);
}

// ---------------------------------------------------------------- AHP (section V-B)
// Pairwise comparison on Saaty's 1-9 scale.  For values p (row server) and
// q (column server): equal -> 1; p > q -> s = ratio p/q rounded half up,
// clamped to 9 (q = 0 -> 9); p < q -> 1/s(q, p).  Returned scaled by 2520
// (the lcm of 1..9), so every entry and every column sum is an exact
// integer.  s = floor((2 hi + lo) / (2 lo)) is estimated with a reciprocal
// (r_hi_lo = 1/(2 lo)) and corrected by the exact remainder.
__device__ __forceinline__ float rcp2(float v) { return v > 0.f ? __builtin_amdgcn_rcpf(2.f * v) : __builtin_inff(); }

__device__ __forceinline__ float saaty2520(float p, float q, float rp, float rq) {
    const bool ge = p >= q;
    const float hi = ge ? p : q, lo = ge ? q : p, rl = ge ? rq : rp;
    const float num = fmaf(2.f, hi, lo);
    const float two_lo = lo + lo;
    float s = floorf(num * rl);
    const float rem = fmaf(-s, two_lo, num);
    s = rem < 0.f ? s - 1.f : s;
    s = rem >= two_lo ? s + 1.f : s;
    s = fminf(s, 9.f);
    s = lo == 0.f ? (hi == 0.f ? 1.f : 9.f) : s;
    return ge ? 2520.f * s : rintf(2520.f * __builtin_amdgcn_rcpf(s));
}

// Pass A: column sums colsum_c[j] = sum_i a_c(i, j), never storing the
// N x N matrix.  Grid (ceil(N/256), nI, nc): thread = column j, block y =
// chunk of ti rows.  Saaty sums are exact integers (x2520); the ratio scale
// sums floats.  Partials per row chunk, reduced in pass B in fixed order.
__global__ __launch_bounds__(kAhpBlock) void k_ahp_colsum(Params p) {
    if (p.b.status[p.r] == 0) return;
    __shared__ float sx[kAhpTile], sr[kAhpTile];
    const int N = p.t.N, c = blockIdx.z, ib = blockIdx.y;
    const int j = blockIdx.x * kAhpBlock + threadIdx.x;
    const int *x = p.xs + (size_t)c * N;
    const bool cost = p.m.cost[c] != 0, ratio = p.m.scale == 1;
    const float q = j < N ? static_cast<float>(x[j]) : 0.f;
    const float rq = rcp2(q);
    int acci = 0;
    float accf = 0.f;
    const int i0 = ib * p.ti, i1 = min(N, i0 + p.ti);
    for (int base = i0; base < i1; base += kAhpTile) {
        const int cnt = min(kAhpTile, i1 - base);
        __syncthreads();
        for (int t = threadIdx.x; t < cnt; t += kAhpBlock) {
            const float v = static_cast<float>(x[base + t]);
            sx[t] = v;
            sr[t] = rcp2(v);
        }
        __syncthreads();
        if (ratio) {
            if (cost) for (int t = 0; t < cnt; ++t) accf += q / sx[t];
            else for (int t = 0; t < cnt; ++t) accf += sx[t] / q;
        } else if (cost) {
            for (int t = 0; t < cnt; ++t) acci += static_cast<int>(saaty2520(q, sx[t], rq, sr[t]));
        } else {
            for (int t = 0; t < cnt; ++t) acci += static_cast<int>(saaty2520(sx[t], q, sr[t], rq));
        }
    }
    if (j < N) p.colpart[((size_t)c * p.nI + ib) * N + j] = ratio ? __float_as_int(accf) : acci;
}

// Pass B: row sums of the column-normalised matrix,
// L2_c[i] * N = sum_j a_c(i, j) / colsum_c[j].  Grid (ceil(N/256), nJ, nc):
// thread = row i, block y = chunk of tj columns; kAhpAcc interleaved partial
// sums keep the FP32 error small.  Partials per column chunk.
__global__ __launch_bounds__(kAhpBlock) void k_ahp_rowsum(Params p) {
    if (p.b.status[p.r] == 0) return;
    __shared__ float sx[kAhpTile], sr[kAhpTile], sinv[kAhpTile];
    const int N = p.t.N, c = blockIdx.z, jb = blockIdx.y;
    const int i = blockIdx.x * kAhpBlock + threadIdx.x;
    const int *x = p.xs + (size_t)c * N;
    const bool cost = p.m.cost[c] != 0, ratio = p.m.scale == 1;
    const float pv = i < N ? static_cast<float>(x[i]) : 0.f;
    const float rp = rcp2(pv);
    float acc[kAhpAcc];
#pragma unroll
    for (int a = 0; a < kAhpAcc; ++a) acc[a] = 0.f;
    const int j0 = jb * p.tj, j1 = min(N, j0 + p.tj);
    for (int base = j0; base < j1; base += kAhpTile) {
        const int cnt = min(kAhpTile, j1 - base);
        __syncthreads();
        for (int t = threadIdx.x; t < cnt; t += kAhpBlock) {
            const int j = base + t;
            const float v = static_cast<float>(x[j]);
            sx[t] = v;
            sr[t] = rcp2(v);
            if (ratio) {
                float s = 0.f;
                for (int ib = 0; ib < p.nI; ++ib) s += __int_as_float(p.colpart[((size_t)c * p.nI + ib) * N + j]);
                sinv[t] = 1.f / s;
            } else {
                long long s = 0;
                for (int ib = 0; ib < p.nI; ++ib) s += p.colpart[((size_t)c * p.nI + ib) * N + j];
                sinv[t] = static_cast<float>(1.0 / static_cast<double>(s));
            }
        }
        __syncthreads();
        int t = 0;
        if (ratio) {
            for (; t + kAhpAcc <= cnt; t += kAhpAcc)
#pragma unroll
                for (int a = 0; a < kAhpAcc; ++a)
                    acc[a] = fmaf(cost ? sx[t + a] / pv : pv / sx[t + a], sinv[t + a], acc[a]);
            for (; t < cnt; ++t) acc[0] = fmaf(cost ? sx[t] / pv : pv / sx[t], sinv[t], acc[0]);
        } else if (cost) {
            for (; t + kAhpAcc <= cnt; t += kAhpAcc)
#pragma unroll
                for (int a = 0; a < kAhpAcc; ++a)
                    acc[a] = fmaf(saaty2520(sx[t + a], pv, sr[t + a], rp), sinv[t + a], acc[a]);
            for (; t < cnt; ++t) acc[0] = fmaf(saaty2520(sx[t], pv, sr[t], rp), sinv[t], acc[0]);
        } else {
            for (; t + kAhpAcc <= cnt; t += kAhpAcc)
#pragma unroll
                for (int a = 0; a < kAhpAcc; ++a)
                    acc[a] = fmaf(saaty2520(pv, sx[t + a], rp, sr[t + a]), sinv[t + a], acc[a]);
            for (; t < cnt; ++t) acc[0] = fmaf(saaty2520(pv, sx[t], rp, sr[t]), sinv[t], acc[0]);
        }
    }
    float s = 0.f;
#pragma unroll
    for (int a = 0; a < kAhpAcc; ++a) s += acc[a];
    if (i < N) p.rowpart[((size_t)c * p.nJ + jb) * N + i] = s;
}

// AHP step, last stage: global priority PG[u] = sum_c P1[c] * L2_c[u], with
// P1 the local rank of the criteria-level ratio matrix W[a]/W[b] (equal to
// W when the weights sum to 1), then selection and commit.
template <int BS>
__global__ __launch_bounds__(BS) void k_ahp_select(Params p) {
    extern __shared__ __align__(16) char dsm[];
    if (p.b.status[p.r] == 0) return;
    Smem sm = carve(dsm, 0, p.t.nsw);
    const Topo &t = p.t;
    const int N = t.N, nc = p.m.nc;
    const int g0 = p.b.coff[p.r], g = g0 + p.i, n = p.b.coff[p.r + 1] - g0;
    const int P = load_peers<BS>(p.st, p.b, sm, g0, g);
    if (threadIdx.x == 0) {
        double colsum[kMaxCrit];
        for (int b = 0; b < nc; ++b) {
            colsum[b] = 0.0;
            for (int a = 0; a < nc; ++a) colsum[b] += static_cast<double>(p.m.w[a]) / p.m.w[b];
        }
        for (int a = 0; a < nc; ++a) {
            double s = 0.0;
            for (int b = 0; b < nc; ++b) s += (static_cast<double>(p.m.w[a]) / p.m.w[b]) / colsum[b];
            sm.q[a] = static_cast<float>(s / nc);
        }
        sm.misc[1] = trace_slot(p.tr, p.inst, p.r, p.i);
    }
    __syncthreads();
    double p1[kMaxCrit];
#pragma unroll
    for (int c = 0; c < kMaxCrit; ++c) p1[c] = c < nc ? sm.q[c] : 0.0;
    const double invN = 1.0 / N;
    auto pg = [&](int u) -> float {
        double s = 0.0;
#pragma unroll
        for (int c = 0; c < kMaxCrit; ++c) {
            if (c >= nc) break;
            double l = 0.0;
            for (int jb = 0; jb < p.nJ; ++jb) l += p.rowpart[((size_t)c * p.nJ + jb) * N + u];
            s += p1[c] * (l * invN);
        }
        return static_cast<float>(s);
    };
    const int slot = sm.misc[1];
    if (slot >= 0)
        for (int u = threadIdx.x; u < N; u += BS) p.tr.scores[(size_t)slot * N + u] = pg(u);
    select_commit<BS>(t, p.st, p.b, sm, p.xs + (size_t)nc * N, p.r, p.i, n, g, P, p.b.cpu[g], p.b.ram[g],
                      [&](int u) { return score_key(pg(u), u); });
}

// ---------------------------------------------------------------- batched form
// One persistent workgroup per data-center instance: the instance's state
// and scratch live in LDS for the whole launch; the workgroup walks its
// requests in FCFS order and their containers in index order.
template <int BS>
__global__ __launch_bounds__(BS) void k_topsis_batched(Params p) {
    extern __shared__ __align__(16) char dsm[];
    const int inst = blockIdx.x;
    const int N = p.t.N;
    Smem sm = carve(dsm, p.pc_cap, p.t.nsw);
    int *xs = reinterpret_cast<int *>(dsm + smem_fixed_bytes() + sizeof(int) * 2 * p.pc_cap * p.t.nsw);
    int *ls = xs + (size_t)(p.m.nc + 4) * N;
    const State gs = state_at(p.state_base, p.state_stride, inst, N);
    for (int x = threadIdx.x; x < 6 * N; x += BS) ls[x] = gs.cpu[x];
    __syncthreads();
    const State st{ls, ls + N, ls + 2 * N, ls + 3 * N, ls + 4 * N, ls + 5 * N};
    const int r0 = p.b.iroff[inst], r1 = p.b.iroff[inst + 1];
    for (int r = r0; r < r1; ++r) {
        const int n = p.b.coff[r + 1] - p.b.coff[r];
        for (int i = 0; i < n; ++i) {
            topsis_step<BS>(p.t, st, p.m, p.b, sm, xs, p.pc_cap, p.tr, inst, r, i);
            __syncthreads();
            if (p.b.status[r] == 0) break;
        }
    }
    __syncthreads();
    for (int x = threadIdx.x; x < 6 * N; x += BS) gs.cpu[x] = ls[x];
}

// ---------------------------------------------------------------- release
// Departure of accepted request p.r: CPU, RAM, placed count and every path
// demand go back to the state (integer, exact).
template <int BS>
__global__ __launch_bounds__(BS) void k_release(Params p) {
    const int n = p.b.coff[p.r + 1] - p.b.coff[p.r];
    give_back<BS>(p.t, p.st, p.b, p.r, n);
}

__global__ void k_fill_i32(int *dst, int value, long long n) {
    for (long long x = blockIdx.x * (long long)blockDim.x + threadIdx.x; x < n; x += (long long)gridDim.x * blockDim.x)
        dst[x] = value;
}

}  // namespace dcs
