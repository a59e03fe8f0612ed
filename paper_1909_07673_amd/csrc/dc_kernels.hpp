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
    int *xs;         // global per-server scratch [nc+6][N] of that instance
    int pc_cap;      // peers per path-table chunk
    int inst;
    // batched form: state of instance i at state_base + i * state_stride
    int *state_base;
    long long state_stride;
    // AHP
    int *colpart;    // [nc][nI][N] (doubles on the difference scale)
    float *rowpart;  // [nc][nJ][N]
    int ti, tj, nI, nJ;
    int *ysort;      // AHP on the 1-9 scale: [nc][N] criterion values in ascending order
    double *wsort;   // and 1 / column sum at each sorted position
    double p1[kMaxCrit];  // criteria-level priorities P1 (ahp_p1), computed once per context
    StepIn s;        // the container step of a plain launch
    int pj[kMaxN], pbw[kMaxN];   // its placed peers (container index, minimum demand)
    int pbmax[kMaxN];            // and their maximum demands
};

constexpr int kAhpBlock = 256;
constexpr int kAhpTile = 1024;   // values staged per LDS tile in the AHP passes
constexpr int kAhpAcc = 8;       // independent partial sums per row in pass B
constexpr int kAhpSortMax = 8192; // servers up to which the 1-9 scale uses the sorted passes

// Dynamic LDS of the single-workgroup step: fixed part, capacity sums and
// peer tables, then optionally the criteria scratch xs and the state.
inline size_t step_lds_bytes(int pc_cap, int nsw, size_t xs_ints, size_t state_ints) {
    return smem_fixed_bytes() + sizeof(int) * (smem_var_ints(pc_cap, nsw) + xs_ints + state_ints);
}

// Rows of the per-server scratch: the criteria, the feasibility flag and
// five accumulators kept across peer chunks.
__host__ __device__ inline int xs_rows(int nc) { return nc + 6; }

__device__ __forceinline__ int *lds_after_tables(char *dsm, int pc_cap, int nsw) {
    return reinterpret_cast<int *>(dsm + smem_fixed_bytes() + sizeof(int) * smem_var_ints(pc_cap, nsw));
}

__device__ __forceinline__ State state_at(int *base, long long stride, int inst, int N) {
    int *s = base + stride * inst;
    return State{s, s + N, s + 2 * N, s + 3 * N, s + 4 * N, s + 5 * N};
}

// Copies n int32 (n % 4 == 0, 16-byte aligned) between global memory and
// LDS in int4 pieces, four loads in flight per thread.
template <int BS>
__device__ __forceinline__ void stage_in(int *lds, const int *g, int n) {
    const int4 *src = reinterpret_cast<const int4 *>(g);
    int4 *dst = reinterpret_cast<int4 *>(lds);
    const int n4 = n >> 2;
    int x = threadIdx.x;
    for (; x + 3 * BS < n4; x += 4 * BS) {
        const int4 a = src[x], b = src[x + BS], c = src[x + 2 * BS], d = src[x + 3 * BS];
        dst[x] = a; dst[x + BS] = b; dst[x + 2 * BS] = c; dst[x + 3 * BS] = d;
    }
    for (; x < n4; x += BS) dst[x] = src[x];
}

template <int BS>
__device__ __forceinline__ void stage_out(int *g, const int *lds, int n) {
    const int4 *src = reinterpret_cast<const int4 *>(lds);
    int4 *dst = reinterpret_cast<int4 *>(g);
    for (int x = threadIdx.x; x < (n >> 2); x += BS) dst[x] = src[x];
}

// ---------------------------------------------------------------- plain form
// The plain form passes the container's peer list in the kernel arguments,
// so only the peers' servers are read from memory.
//
// The persistent kernels (batched, serving) read the Batch pointers from an
// LDS copy: fields are then loaded when used, after each barrier, instead of
// holding some forty scalar registers across their request loops, which
// pushes the compiler into spilling scalars through vector lanes.  A plain
// launch runs one step, and keeps them in registers.
__device__ __forceinline__ ReqView plain_view(const Params &p) {
    return ReqView{p.pj, p.pbw, p.b.host + p.s.g0, nullptr, p.pbmax};
}

// One launch per container step, one workgroup.  With RES the instance's
// state (6N int32) is staged into LDS for the step and written back, and
// the criteria scratch lives in LDS too; otherwise both stay in HBM/L2.
// K > 0: compiled for k = K fat-trees on the four default criteria (as the
// batched kernel); K = 0: any.
template <int BS, bool RES, int K = 0>
__global__ __launch_bounds__(BS) void k_topsis_plain(Params p) {
    extern __shared__ __align__(16) char dsm[];
    if (p.b.status[p.s.r] == 0) return;        // request already rejected
    constexpr int CS = K ? 4 : 0;
    const Topo t = topo_of<K>(p.t);
    Smem sm = carve(dsm, p.pc_cap, t.nsw);
    const ReqView rv = plain_view(p);
    if (!RES) {
        topsis_step<BS, host_group(BS), false, CS>(t, p.st, p.m, p.b, sm, p.xs, p.pc_cap, p.tr, p.inst, p.s, rv);
        return;
    }
    const int N = t.N;
    int *xs = lds_after_tables(dsm, p.pc_cap, t.nsw);
    int *ls = xs + (size_t)xs_rows(crit_count<CS>(p.m)) * N;
    stage_in<BS>(ls, p.st.cpu, 6 * N);        // the six arrays are contiguous
    // (the barrier at the end of load_peers orders these writes before any read)
    const State st{ls, ls + N, ls + 2 * N, ls + 3 * N, ls + 4 * N, ls + 5 * N};
    topsis_step<BS, host_group(BS), true, CS>(t, st, p.m, p.b, sm, xs, p.pc_cap, p.tr, p.inst, p.s, rv);
    __syncthreads();
    stage_out<BS>(p.st.cpu, ls, 6 * N);
}

// AHP step, stage 1: criteria of every server into the global xs rows,
// spread over ceil(N / (G * BS)) workgroups.  K > 0: compiled for k = K
// fat-trees and the criteria list CS (as the TOPSIS kernels are); K = 0:
// any.
template <int BS, int K = 0, int CS = 0>
__global__ __launch_bounds__(BS) void k_criteria_plain(Params p) {
    extern __shared__ __align__(16) char dsm[];
    if (p.b.status[p.s.r] == 0) return;
    if (p.s.i == 0 && blockIdx.x == 0 && threadIdx.x == 0) p.b.tsb[p.s.r] = dev_clock();
    const Topo t = topo_of<K>(p.t);
    Smem sm = carve(dsm, p.pc_cap, t.nsw);
    load_peers<BS, true>(t, p.st, plain_view(p), sm, p.s.P);
    criteria_stage<BS, false, host_group(BS), CS>(t, p.st, p.m, sm, p.xs, p.s.cpu, p.s.ram, p.s.P, p.pc_cap,
                                                  blockIdx.x, gridDim.x);
}

// ---------------------------------------------------------------- AHP (section V-B)
// Pairwise comparison on Saaty's 1-9 scale.  For values p (row server) and
// q (column server): equal -> 1; p > q -> s = ratio p/q rounded half up,
// clamped to 9 (q = 0 -> 9); p < q -> 1/s(q, p).  Returned scaled by 2520
// (the lcm of 1..9), so every entry and every column sum is an exact
// integer.
//
// With hi = max(p, q), lo = min(p, q), num = 2 hi + lo: s = min(9,
// floor(num / (2 lo))).  rcp2 gives 1/(2 lo) from the hardware reciprocal
// (within 1 ulp) scaled down by 2^-21, so num * rl lies strictly below the
// exact quotient; its floor is then at most one below s wherever s < 11,
// and one test of the exact remainder num - s * 2 lo (all integers below
// 2^24) corrects it; larger quotients are clamped to 9 anyway.  lo = 0
// makes rl = 2^100: hi > 0 gives a quotient far above 9, clamped to 9;
// hi = 0 gives 0, which the remainder test (0 >= 0) turns into 1.  hi and
// lo are selected by the comparison already made, not by fmax / fmin.
__device__ __forceinline__ float rcp2(float v) {
    return v > 0.f ? __builtin_amdgcn_rcpf(2.f * v) * (1.0f - 0x1p-21f) : 0x1p100f;
}

__device__ __forceinline__ float saaty2520(float p, float q, float rp, float rq) {
    const bool ge = p >= q;
    const float hi = ge ? p : q, lo = ge ? q : p, rl = ge ? rq : rp;
    const float num = fmaf(2.f, hi, lo), two_lo = lo + lo;
    float s = floorf(num * rl);
    const float rem = fmaf(-s, two_lo, num);
    s = rem >= two_lo ? s + 1.f : s;
    s = fminf(s, 9.f);
    return rintf(2520.f * (ge ? s : __builtin_amdgcn_rcpf(s)));
}

// Difference scale (section V-B's rule on differences): the larger value's
// entry is p - q, equal values 1, the smaller value's 1 / (q - p).  Values
// are integers below 2^22, so |p - q| is exact in FP32 and at least 1 when
// they differ; the reciprocal of max(|p - q|, 1) is then 1 / (q - p), or
// exactly 1 for equal values (hardware reciprocal, within 1 ulp), with no
// branch.
__device__ __forceinline__ float diff_scale(float p, float q) {
    const float d = fabsf(p - q);
    return p > q ? d : __builtin_amdgcn_rcpf(fmaxf(d, 1.f));
}

// Pass A: column sums colsum_c[j] = sum_i a_c(i, j), never storing the
// N x N matrix.  Grid (ceil(N/256), nI, nc): thread = column j, block y =
// chunk of ti rows.  Saaty sums are exact integers (x2520); the ratio scale
// sums floats; the difference scale sums in FP64 (its integer entries,
// up to 2^22 each, stay exact).  Partials per row chunk (one int each, two
// on the difference scale), reduced in pass B in fixed order.
__global__ __launch_bounds__(kAhpBlock) void k_ahp_colsum(Params p) {
    if (p.b.status[p.s.r] == 0) return;
    __shared__ float sx[kAhpTile], sr[kAhpTile];
    const int N = p.t.N, c = blockIdx.z, ib = blockIdx.y;
    const int j = blockIdx.x * kAhpBlock + threadIdx.x;
    const int *x = p.xs + (size_t)c * N;
    const bool cost = p.m.cost[c] != 0, ratio = p.m.scale == 1, diff = p.m.scale == 2;
    const float q = j < N ? static_cast<float>(x[j]) : 0.f;
    const float rq = rcp2(q);
    int acci = 0;
    float accf = 0.f;
    double accd = 0.0;
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
        } else if (diff) {
            if (cost) for (int t = 0; t < cnt; ++t) accd += static_cast<double>(diff_scale(q, sx[t]));
            else for (int t = 0; t < cnt; ++t) accd += static_cast<double>(diff_scale(sx[t], q));
        } else if (cost) {
            for (int t = 0; t < cnt; ++t) acci += static_cast<int>(saaty2520(q, sx[t], rq, sr[t]));
        } else {
            for (int t = 0; t < cnt; ++t) acci += static_cast<int>(saaty2520(sx[t], q, sr[t], rq));
        }
    }
    if (j < N) {
        const size_t at = ((size_t)c * p.nI + ib) * N + j;
        if (diff) reinterpret_cast<double *>(p.colpart)[at] = accd;
        else p.colpart[at] = ratio ? __float_as_int(accf) : acci;
    }
}

// Pass B: row sums of the column-normalised matrix,
// L2_c[i] * N = sum_j a_c(i, j) / colsum_c[j].  Grid (ceil(N/256), nJ, nc):
// thread = row i, block y = chunk of tj columns; kAhpAcc interleaved partial
// sums keep the FP32 error small.  Partials per column chunk.
__global__ __launch_bounds__(kAhpBlock) void k_ahp_rowsum(Params p) {
    if (p.b.status[p.s.r] == 0) return;
    __shared__ float sx[kAhpTile], sr[kAhpTile], sinv[kAhpTile];
    const int N = p.t.N, c = blockIdx.z, jb = blockIdx.y;
    const int i = blockIdx.x * kAhpBlock + threadIdx.x;
    const int *x = p.xs + (size_t)c * N;
    const bool cost = p.m.cost[c] != 0, ratio = p.m.scale == 1, diff = p.m.scale == 2;
    const float pv = i < N ? static_cast<float>(x[i]) : 0.f;
    const float rp = rcp2(pv);
    const int *cp = p.colpart + (size_t)c * p.nI * N;
    const double *cpd = reinterpret_cast<const double *>(p.colpart) + (size_t)c * p.nI * N;
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
                for (int ib = 0; ib < p.nI; ++ib) s += __int_as_float(cp[(size_t)ib * N + j]);
                sinv[t] = 1.f / s;
            } else if (diff) {
                double s = 0.0;
                for (int ib = 0; ib < p.nI; ++ib) s += cpd[(size_t)ib * N + j];
                sinv[t] = static_cast<float>(1.0 / s);
            } else {
                long long s = 0;
                for (int ib = 0; ib < p.nI; ++ib) s += cp[(size_t)ib * N + j];
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
        } else if (diff) {
            for (; t + kAhpAcc <= cnt; t += kAhpAcc)
#pragma unroll
                for (int a = 0; a < kAhpAcc; ++a)
                    acc[a] = fmaf(cost ? diff_scale(sx[t + a], pv) : diff_scale(pv, sx[t + a]), sinv[t + a], acc[a]);
            for (; t < cnt; ++t) acc[0] = fmaf(cost ? diff_scale(sx[t], pv) : diff_scale(pv, sx[t]), sinv[t], acc[0]);
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

// ---------------------------------------------------------------- AHP, 1-9 scale, sorted form
// On the 1-9 scale an entry takes one of 17 values, and which one is fixed
// by integer thresholds: for p > q > 0 the rounded ratio s = min(9,
// floor((2p + q) / 2q)) is at least k exactly when 2p >= (2k - 1) q, and a
// value of 0 against a larger one scores 9.  With a criterion's values
// sorted, the sum of a(v, y_m) w_m over all servers m (or of a(y_m, v) w_m)
// is therefore a weighted count over 17 buckets, whose bounds are 18 binary
// searches: unit weights give the exact column sums, weights 1 / column sum
// (prefix-summed in FP64) give the row sums of the column-normalised matrix
// (section V-B, Eqs. (9)-(10)).  The result equals the pairwise passes up to
// the row sums' rounding; the work is O(C N log N) after an O(C N^2) rank
// count of two instructions per pair.

// Bucket bounds of value v (>= 0) against the ascending y[0, n): [lv, uv)
// holds the values equal to v; positions [ai[k], n) hold the larger values
// whose rounded ratio to v is at least k, and [0, bi[k]) the smaller values
// whose ratio from v is at least k (k = 1..9; index 10 closes the sums).
// The 18 lower bounds advance together, one LDS load each per halving.
struct SaatyBuckets {
    int lv, uv, ai[11], bi[11];
};

__device__ __forceinline__ SaatyBuckets saaty_buckets(const int *y, int n, int v) {
    int t[18], pos[18];
    t[0] = v;
    t[1] = v + 1;
#pragma unroll
    for (int k = 2; k <= 9; ++k) {
        t[2 * k - 2] = max(((2 * k - 1) * v + 1) >> 1, v + 1);   // y >= this: ratio y / v rounds to >= k
        t[2 * k - 1] = (2 * v) / (2 * k - 1) + 1;                 // y < this: ratio v / y rounds to >= k
    }
#pragma unroll
    for (int q = 0; q < 18; ++q) pos[q] = 0;
    for (int step = 1 << (31 - __builtin_clz(n | 1)); step > 0; step >>= 1) {
        int val[18];
#pragma unroll
        for (int q = 0; q < 18; ++q) val[q] = y[min(pos[q] + step, n) - 1];
#pragma unroll
        for (int q = 0; q < 18; ++q) pos[q] = (pos[q] + step <= n && val[q] < t[q]) ? pos[q] + step : pos[q];
    }
    SaatyBuckets b;
    b.lv = pos[0];
    b.uv = pos[1];
    b.ai[1] = b.uv;
    b.bi[1] = b.lv;
#pragma unroll
    for (int k = 2; k <= 9; ++k) {
        b.ai[k] = pos[2 * k - 2];
        b.bi[k] = min(pos[2 * k - 1], b.lv);
    }
    b.ai[10] = n;
    b.bi[10] = 0;
    return b;
}

// Sum over m of 2520 a(v, y_m) w_m (first) or 2520 a(y_m, v) w_m, with
// W(a, b) the weight of the sorted positions [a, b): the side whose ratio
// is s contributes 2520 s per position, the other side 2520 / s.
template <class T, class WFn>
__device__ __forceinline__ T saaty_sum(const SaatyBuckets &b, int n, bool first, WFn W) {
    T big = 0, small = 0;
#pragma unroll
    for (int k = 1; k <= 9; ++k) {
        const T a = W(b.ai[k], n), bb = W(0, b.bi[k]);
        const T da = W(b.ai[k], b.ai[k + 1]), db = W(b.bi[k + 1], b.bi[k]);
        big += first ? bb : a;
        small += static_cast<T>(2520 / k) * (first ? da : db);
    }
    return static_cast<T>(2520) * (W(b.lv, b.uv) + big) + small;
}

// Exclusive scan of one value per thread over the BS threads of the block.
template <int BS, class T, class Op>
__device__ __forceinline__ T block_excl_scan(T v, T id, T *sh, Op op) {
    const int tid = threadIdx.x;
    sh[tid] = v;
    __syncthreads();
    for (int off = 1; off < BS; off <<= 1) {
        const T o = tid >= off ? sh[tid - off] : id;
        __syncthreads();
        sh[tid] = op(sh[tid], o);
        __syncthreads();
    }
    const T r = tid ? sh[tid - 1] : id;
    __syncthreads();
    return r;
}

// n int32 from global memory into LDS (16-byte aligned), four 16-byte loads
// in flight per thread when the source allows it.
template <int BS>
__device__ __forceinline__ void lds_load_i32(int *lds, const int *g, int n) {
    if ((reinterpret_cast<uintptr_t>(g) & 15) == 0 && (n & 3) == 0) {
        stage_in<BS>(lds, g, n);
    } else {
        for (int x = threadIdx.x; x < n; x += BS) lds[x] = g[x];
    }
}

// Pass S: the values of criterion c in ascending order, duplicates kept
// (what the column and row sums search), in two launches spread over
// R = ceil(N / 1024) workgroups per criterion.
//
// S1 sorts each run of 1,024 values (the last padded with INT_MAX, which
// sorts last) by a bitonic network, one value per thread: compare-exchanges
// at distances below 64 go between the lanes of a wave (lane xor j), longer
// ones through LDS, one barrier each; every trip count is a compile-time
// constant, so the network unrolls.  With one run its output is the sorted
// array itself, and S2 is not launched.  Grid (R, 1, nc).
constexpr int kAhpSortBlock = 1024;

__global__ __launch_bounds__(kAhpSortBlock) void k_ahp_sort_runs(Params p, int *runs) {
    if (p.b.status[p.s.r] == 0) return;
    constexpr int L = kAhpSortBlock;
    __shared__ int y[L];
    const int N = p.t.N, c = blockIdx.z, tid = threadIdx.x, i = tid;
    const int g = blockIdx.x * L + i;
    int v = g < N ? p.xs[(size_t)c * N + g] : INT_MAX;
#pragma unroll
    for (int k = 2; k <= L; k <<= 1) {
        const bool desc_k = (i & k) != 0;                  // ascending where bit k of the slot is clear
        if ((k >> 1) >= kWave) {
            y[i] = v;
            __syncthreads();
#pragma unroll
            for (int j = k >> 1; j >= kWave; j >>= 1) {
                if (tid < L / 2) {
                    const int a = 2 * tid - (tid & (j - 1));   // pair (a, a + j)
                    const int x0 = y[a], x1 = y[a + j];
                    const bool asc = (a & k) == 0;
                    y[a] = asc ? min(x0, x1) : max(x0, x1);
                    y[a + j] = asc ? max(x0, x1) : min(x0, x1);
                }
                __syncthreads();
            }
            v = y[i];
            __syncthreads();                                   // y is written again at the next k
        }
#pragma unroll
        for (int j = min(k >> 1, kWave / 2); j >= 1; j >>= 1) {
            const int o = __shfl_xor(v, j);
            v = desc_k == ((i & j) != 0) ? min(v, o) : max(v, o);
        }
    }
    const int R = gridDim.x;
    if (R == 1) {
        if (g < N) p.ysort[(size_t)c * N + g] = v;
    } else {
        runs[((size_t)c * R + blockIdx.x) * L + i] = v;
    }
}

// S2 merges the R sorted runs: the value at index a of run r goes to
// a + (values below it in every other run), counting a run's equal values
// when the run comes first, so that the positions are distinct.  Each
// workgroup takes one run's values against all runs staged in LDS, the
// binary searches into the other runs advanced together.  Grid (R, 1, nc).
__global__ __launch_bounds__(kAhpSortBlock) void k_ahp_merge_runs(Params p, const int *runs) {
    if (p.b.status[p.s.r] == 0) return;
    constexpr int L = kAhpSortBlock, RMAX = kAhpSortMax / L;
    __shared__ __align__(16) int y[kAhpSortMax];
    const int N = p.t.N, c = blockIdx.z, R = gridDim.x, r = blockIdx.x, a = threadIdx.x;
    lds_load_i32<kAhpSortBlock>(y, runs + (size_t)c * R * L, R * L);
    __syncthreads();
    const int x = y[r * L + a];
    if (x == INT_MAX) return;                                  // padding of the last run
    // per other run q: how many of its values come before x (< x for q
    // after r, <= x for q before r), by a branch-free search that halves a
    // window of the run, so that each halving issues its loads for all runs
    // together (runs past R and run r itself are searched too, and not
    // counted)
    // (x < INT_MAX here, so y <= x is y < x + 1)
    int base[RMAX], xq[RMAX];
#pragma unroll
    for (int q = 0; q < RMAX; ++q) {
        base[q] = min(q, R - 1) * L;
        xq[q] = q < r ? x + 1 : x;
    }
    auto before = [&](int q, int yv) { return yv < xq[q]; };
#pragma unroll
    for (int len = L; len > 1; len -= len >> 1) {
        const int half = len >> 1;
#pragma unroll
        for (int q = 0; q < RMAX; ++q) base[q] = before(q, y[base[q] + half]) ? base[q] + half : base[q];
    }
    int pos = a;
#pragma unroll
    for (int q = 0; q < RMAX; ++q)
        if (q < R && q != r) pos += base[q] - q * L + (before(q, y[base[q]]) ? 1 : 0);
    p.ysort[(size_t)c * N + pos] = x;
}

// Pass C: exact column sums at every sorted position, stored as 1 / sum
// (FP64).  Grid (ceil(N/256), 1, nc).
__global__ __launch_bounds__(kAhpBlock) void k_ahp_sort_col(Params p) {
    if (p.b.status[p.s.r] == 0) return;
    __shared__ __align__(16) int y[kAhpSortMax];
    const int N = p.t.N, c = blockIdx.z;
    lds_load_i32<kAhpBlock>(y, p.ysort + (size_t)c * N, N);
    __syncthreads();
    const int m = blockIdx.x * kAhpBlock + threadIdx.x;
    if (m < N) {
        // column j compares every row i against it: a(x_i, x_j), or
        // a(x_j, x_i) for a cost criterion
        const SaatyBuckets b = saaty_buckets(y, N, y[m]);
        const long long s = saaty_sum<long long>(b, N, p.m.cost[c] != 0,
                                                 [](int a, int e) { return static_cast<long long>(e - a); });
        p.wsort[(size_t)c * N + m] = 1.0 / static_cast<double>(s);
    }
}

// Pass D: row sums of the column-normalised matrix, L_c[i] * N =
// sum_j a(i, j) / colsum[j], from prefix sums of 1 / colsum in sorted
// order.  One partial per row (nJ = 1).  Grid (ceil(N/256), 1, nc).
__global__ __launch_bounds__(kAhpBlock) void k_ahp_sort_row(Params p) {
    if (p.b.status[p.s.r] == 0) return;
    // prefix sums P[0..N] in LDS with one pad slot after every E of them, E
    // the power-of-two chunk each thread scans, so the threads' chunks start
    // in different banks
    __shared__ __align__(16) int y[kAhpSortMax];
    __shared__ double P[kAhpSortMax + kAhpBlock + 2];
    __shared__ double sh[kAhpBlock];
    const int N = p.t.N, c = blockIdx.z, tid = threadIdx.x;
    const int e = max((N + kAhpBlock - 1) / kAhpBlock, 1), lgE = e > 1 ? 32 - __builtin_clz(e - 1) : 0, E = 1 << lgE;
    auto at = [lgE](int q) { return q + (q >> lgE); };
    lds_load_i32<kAhpBlock>(y, p.ysort + (size_t)c * N, N);
    const double *w = p.wsort + (size_t)c * N;
    if (N & 1) {
        for (int m = tid; m < N; m += kAhpBlock) P[at(m + 1)] = w[m];
    } else {
        // with N even every criterion's row is 16-byte aligned
        const int n2 = N >> 1;
        int x = tid;
        for (; x + 3 * kAhpBlock < n2; x += 4 * kAhpBlock) {
            double2 v[4];
#pragma unroll
            for (int u = 0; u < 4; ++u) v[u] = reinterpret_cast<const double2 *>(w)[x + u * kAhpBlock];
#pragma unroll
            for (int u = 0; u < 4; ++u) {
                P[at(2 * (x + u * kAhpBlock) + 1)] = v[u].x;
                P[at(2 * (x + u * kAhpBlock) + 2)] = v[u].y;
            }
        }
        for (; x < n2; x += kAhpBlock) {
            const double2 v = reinterpret_cast<const double2 *>(w)[x];
            P[at(2 * x + 1)] = v.x;
            P[at(2 * x + 2)] = v.y;
        }
    }
    if (tid == 0) P[0] = 0.0;
    __syncthreads();
    const int m0 = min(N, tid * E), m1 = min(N, m0 + E);
    double run = 0.0;
    for (int m = m0; m < m1; ++m) run += P[at(m + 1)];
    run = block_excl_scan<kAhpBlock>(run, 0.0, sh, [](double a, double b) { return a + b; });
    for (int m = m0; m < m1; ++m) {
        run += P[at(m + 1)];
        P[at(m + 1)] = run;
    }
    __syncthreads();
    const int i = blockIdx.x * kAhpBlock + tid;
    if (i < N) {
        // row i compares against every column j: a(x_i, x_j), or a(x_j, x_i)
        // for a cost criterion
        const SaatyBuckets b = saaty_buckets(y, N, p.xs[(size_t)c * N + i]);
        const double r =
            saaty_sum<double>(b, N, p.m.cost[c] == 0, [&](int a, int e) { return P[at(e)] - P[at(a)]; });
        p.rowpart[(size_t)c * N + i] = static_cast<float>(r);
    }
}

// Local rank of the criteria-level ratio matrix W[a] / W[b] (column sums,
// then row means of the normalised matrix); equal to W when the weights sum
// to 1.  Kept as FP32 values, widened to FP64 for the sums that use them.
// Depends on the weights only: computed on the host once per context and
// passed in the launch parameters (the same FP64 operations in the same
// order, each rounded as IEEE specifies on both sides).
__host__ __device__ inline void ahp_p1(const Method &m, double *p1) {
    const int nc = m.nc;
    double colsum[kMaxCrit];
    for (int b = 0; b < kMaxCrit; ++b) {
        colsum[b] = 1.0;
        if (b >= nc) continue;
        colsum[b] = 0.0;
        for (int a = 0; a < nc; ++a) colsum[b] += static_cast<double>(m.w[a]) / m.w[b];
    }
    for (int a = 0; a < kMaxCrit; ++a) {
        p1[a] = 0.0;
        if (a >= nc) continue;
        double s = 0.0;
        for (int b = 0; b < nc; ++b) s += (static_cast<double>(m.w[a]) / m.w[b]) / colsum[b];
        p1[a] = static_cast<double>(static_cast<float>(s / nc));
    }
}

// AHP step, stage 4: global priority of every server, PG[u] = sum_c P1[c] *
// L2_c[u], summing the row partials in fixed order.  Written as FP32 into
// xs row nc + 1 (free once the criteria stage is done), and into the trace
// when this step is recorded.
__global__ __launch_bounds__(kAhpBlock) void k_ahp_pg(Params p) {
    if (p.b.status[p.s.r] == 0) return;
    const int N = p.t.N, nc = p.m.nc;
    const int u = blockIdx.x * kAhpBlock + threadIdx.x;
    if (u >= N) return;
    const double invN = 1.0 / N;
    double s = 0.0;
    for (int c = 0; c < nc; ++c) {
        double l = 0.0;
        for (int jb = 0; jb < p.nJ; ++jb) l += p.rowpart[((size_t)c * p.nJ + jb) * N + u];
        s += p.p1[c] * (l * invN);
    }
    const float v = static_cast<float>(s);
    reinterpret_cast<float *>(p.xs + (size_t)(nc + 1) * N)[u] = v;
    if (p.tr.stride > 0) {
        // the slot k_ahp_select claims for this step (it advances the counter)
        const int cnt = p.tr.counter[p.inst];
        if (cnt % p.tr.stride == 0 && cnt / p.tr.stride < p.tr.cap)
            p.tr.scores[static_cast<size_t>(cnt / p.tr.stride) * N + u] = v;
    }
}

// AHP step, last stage: selection and commit on the global priorities.
template <int BS>
__global__ __launch_bounds__(BS) void k_ahp_select(Params p) {
    extern __shared__ __align__(16) char dsm[];
    if (p.b.status[p.s.r] == 0) return;
    Smem sm = carve(dsm, 0, p.t.nsw);
    const Topo &t = p.t;
    const int N = t.N, nc = p.m.nc;
    const ReqView rv = plain_view(p);
    if (threadIdx.x == 0) trace_slot(p.tr, p.inst, p.b.rid[p.s.r], p.s.i);   // scores written by k_ahp_pg
    load_peers<BS, false>(t, p.st, rv, sm, p.s.P);
    const float *pg = reinterpret_cast<const float *>(p.xs + (size_t)(nc + 1) * N);
    select_commit<BS, 1>(t, p.st, p.b, sm, p.xs + (size_t)nc * N, p.s, rv, p.m.route_end,
                      [&](int u) { return score_key(pg[u], u); });
}

// ---------------------------------------------------------------- batched form
// LDS ints of the request prefetch of the batched form: hosts, cpu, ram
// (kMaxN each), relative peer offsets (kMaxN + 4), peers, minimum and
// maximum demands (kMaxPairs each), maximum cpu and ram (kMaxN each).
__host__ __device__ inline size_t req_lds_ints() { return 6 * (size_t)kMaxN + 4 + 3 * (size_t)kMaxPairs; }

// One persistent workgroup per data-center instance: the instance's state,
// the per-server scratch and the request being scheduled live in LDS for
// the whole launch; the workgroup walks its requests in FCFS order and
// their containers in index order.  Each thread scores G servers together
// (the autotuner picks BS and G, and the peer chunk p.pc_cap).
// K > 0: the data centers are k = K fat-trees scored on the four default
// criteria (CPU, RAM, active, path bandwidth; all benefits), so the
// topology and the criterion list are compile-time constants: index
// arithmetic becomes shifts and the per-criterion selection folds away.
// Same arithmetic as K = 0 (any k and criteria), bit-identical results.
template <int BS, int G, int K>
__global__ __launch_bounds__(BS) void k_topsis_batched(Params p) {
    extern __shared__ __align__(16) char dsm[];
    const int inst = blockIdx.x;
    const Topo t = topo_of<K>(p.t);
    const Method &m = p.m;
    constexpr int CS = K ? 4 : 0;
    const int N = t.N;
    Smem sm = carve(dsm, p.pc_cap, t.nsw);
    int *xs = lds_after_tables(dsm, p.pc_cap, t.nsw);
    int *ls = xs + (size_t)xs_rows(crit_count<CS>(m)) * N;
    int *rq_host = ls + 6 * (size_t)N;
    int *rq_cpu = rq_host + kMaxN, *rq_ram = rq_cpu + kMaxN, *rq_poff = rq_ram + kMaxN;
    int *rq_pj = rq_poff + kMaxN + 4, *rq_pbw = rq_pj + kMaxPairs, *rq_pbmax = rq_pbw + kMaxPairs;
    int *rq_cmax = rq_pbmax + kMaxPairs, *rq_rmax = rq_cmax + kMaxN;
    const State gs = state_at(p.state_base, p.state_stride, inst, N);
    stage_in<BS>(ls, gs.cpu, 6 * N);
    const State st{ls, ls + N, ls + 2 * N, ls + 3 * N, ls + 4 * N, ls + 5 * N};
    __shared__ Batch lb;
    if (threadIdx.x == 0) lb = p.b;
    __syncthreads();
    // per-request values are the same on every lane: moved to scalar
    // registers once loaded, so that no later wait for memory (which also
    // waits for the step's outstanding stores) is placed for them
    const int r0 = uniform(p.b.iroff[inst]), r1 = uniform(p.b.iroff[inst + 1]);
    for (int r = r0; r < r1; ++r) {
        const int g0 = uniform(p.b.coff[r]), n = uniform(p.b.coff[r + 1]) - g0;
        const int pb = uniform(p.b.poff[g0]), npair = uniform(p.b.poff[g0 + n]) - pb;
        for (int x = threadIdx.x; x <= n; x += BS) {
            rq_poff[x] = p.b.poff[g0 + x] - pb;
            if (x < n) {
                rq_cpu[x] = p.b.cpu[g0 + x];
                rq_ram[x] = p.b.ram[g0 + x];
                rq_cmax[x] = p.b.cmax[g0 + x];
                rq_rmax[x] = p.b.rmax[g0 + x];
                rq_host[x] = -1;
            }
        }
        for (int x = threadIdx.x; x < npair; x += BS) {
            rq_pj[x] = p.b.pj[pb + x];
            rq_pbw[x] = p.b.pbw[pb + x];
            rq_pbmax[x] = p.b.pbmax[pb + x];
        }
        __syncthreads();
        for (int i = 0; i < n; ++i) {
            const int q0 = rq_poff[i];
            const StepIn s{r, i, n, g0, g0 + i, pb + q0, rq_poff[i + 1] - q0, rq_cpu[i], rq_ram[i],
                           rq_cmax[i], rq_rmax[i]};
            const ReqView rv{rq_pj + q0, rq_pbw + q0, rq_host, rq_host, rq_pbmax + q0, rq_poff, rq_pj};
            if (!topsis_step<BS, G, true, CS>(t, st, m, lb, sm, xs, p.pc_cap, p.tr, inst, s, rv)) break;
        }
        __syncthreads();
    }
    __syncthreads();
    stage_out<BS>(gs.cpu, ls, 6 * N);
}

// ---------------------------------------------------------------- release
// Departure of accepted request p.r: CPU, RAM, placed count and every path
// demand go back to the state (integer, exact).
template <int BS>
__global__ __launch_bounds__(BS) void k_release(Params p) {
    const int n = p.b.coff[p.s.r + 1] - p.b.coff[p.s.r];
    give_back<BS>(p.t, p.st, p.b, p.s.r, n);
}

__global__ void k_fill_i32(int *dst, int value, long long n) {
    for (long long x = blockIdx.x * (long long)blockDim.x + threadIdx.x; x < n; x += (long long)gridDim.x * blockDim.x)
        dst[x] = value;
}

}  // namespace dcs
