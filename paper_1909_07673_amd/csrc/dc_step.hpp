// Device side of one container step: path stage, criteria, TOPSIS scoring,
// argmax selection, commit with widest shortest-path routing, and request
// rollback.  Everything here runs inside one workgroup; the plain, batched
// and serving kernels differ only in where the data-center state lives
// (HBM/L2 or LDS) and in how steps are fed.
//
// Paper references (arXiv 1909.07673):
//   section II-A / Table I  data-center graph, capacities, requests
//   section IV-A            k-ary fat-tree
//   section V               criteria c^s_u, bw^s_u, f_u
//   section V-C             TOPSIS
//   section V-D             widest shortest path, one residual per undirected link
//   Eqs. (4)-(5)            capacity and bandwidth constraints
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace dcs {

constexpr int kMaxCrit = 8;
constexpr int kMaxN = 64;          // containers per request
constexpr int kWave = 64;
constexpr int kBig = 0x7fffffff;

enum { CRIT_CPU = 0, CRIT_RAM = 1, CRIT_ACTIVE = 2, CRIT_PATHBW = 3, CRIT_UPLINK = 4, CRIT_HOPS = 5 };

// Fat-tree sizes.  h = k/2 hosts per edge switch and aggregation switches per
// pod; hh = h*h hosts per pod; nsw = k*k/2 edge (and aggregation) switches.
struct Topo {
    int k, h, hh, N, nsw;
};

// Residual state of one data center, structure-of-arrays, N entries each.
struct State {
    int *cpu, *ram, *npl, *up, *ea, *ac;
};

struct Method {
    int method, scale, nc, pad;
    int crit[kMaxCrit];
    int cost[kMaxCrit];
    float w[kMaxCrit];
};

// Requests of one schedule call, CSR layout.  Container g of request r is
// coff[r] + i; its placed peers are pj[poff[g]..poff[g+1]) (container index
// within the request, ascending) with demands pbw[].
struct Batch {
    const int *coff, *cpu, *ram, *poff, *pj, *pbw;
    int *host;      // [Ct] chosen server, -1 until placed
    float *score;   // [Ct] score of the chosen server
    int *code;      // [Pt] path choice per peer pair, -1 when co-located
    int *status;    // [R]  1 accepted (optimistic), 0 rejected
    int *failat;    // [R]  container without a server, -1
    const int *iroff;  // [I+1] first request of each instance (batched form)
    long long *tsb, *tse;  // [R] device clock (100 MHz) at the first step's start / the decision
};

// Constant-rate device clock (100 MHz), read without a memory access.
__device__ __forceinline__ long long dev_clock() { return static_cast<long long>(wall_clock64()); }

struct Trace {
    int *meta;        // [cap][4]
    float *scores;    // [cap][N]
    int *counter;     // per instance step counter
    int stride, cap;
};

// LDS scratch of a step, carved from dynamic shared memory.
struct Smem {
    int *ph, *pbw, *upv;              // [kMaxN] peer server, demand, its uplink residual
    int *tabT, *tabE;                 // [pc][nsw] per-peer aggregation / edge tables
    unsigned long long *wkey;         // [32] per-wave argmax partials
    unsigned long long *ws2;          // [32][kMaxCrit] per-wave sum of squares
    int *wmx, *wmn;                   // [32][kMaxCrit]
    float *q, *ap, *am;               // [kMaxCrit]
    int *misc;                        // [16]
};

__host__ __device__ inline size_t smem_fixed_bytes() {
    return sizeof(int) * 3 * kMaxN + sizeof(unsigned long long) * 32 +
           sizeof(unsigned long long) * 32 * kMaxCrit + sizeof(int) * 2 * 32 * kMaxCrit +
           sizeof(float) * 3 * kMaxCrit + sizeof(int) * 16;
}

__device__ inline Smem carve(char *base, int pc, int nsw) {
    Smem s;
    unsigned long long *p64 = reinterpret_cast<unsigned long long *>(base);
    s.wkey = p64; p64 += 32;
    s.ws2 = p64; p64 += 32 * kMaxCrit;
    int *p = reinterpret_cast<int *>(p64);
    s.wmx = p; p += 32 * kMaxCrit;
    s.wmn = p; p += 32 * kMaxCrit;
    s.ph = p; p += kMaxN;
    s.pbw = p; p += kMaxN;
    s.upv = p; p += kMaxN;
    s.misc = p; p += 16;
    float *f = reinterpret_cast<float *>(p);
    s.q = f; f += kMaxCrit;
    s.ap = f; f += kMaxCrit;
    s.am = f; f += kMaxCrit;
    p = reinterpret_cast<int *>(f);
    s.tabT = p; p += pc * nsw;
    s.tabE = p;
    return s;
}

// ---------------------------------------------------------------- wave / block reductions
__device__ __forceinline__ unsigned long long wave_max_u64(unsigned long long v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) {
        unsigned long long w = __shfl_xor(v, o, kWave);
        v = w > v ? w : v;
    }
    return v;
}
__device__ __forceinline__ unsigned long long wave_sum_u64(unsigned long long v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, kWave);
    return v;
}
__device__ __forceinline__ int wave_max_i(int v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v = max(v, __shfl_xor(v, o, kWave));
    return v;
}
__device__ __forceinline__ int wave_min_i(int v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v = min(v, __shfl_xor(v, o, kWave));
    return v;
}

// Block-wide maximum of a 64-bit key; every thread gets the result.
template <int BS>
__device__ __forceinline__ unsigned long long block_max_u64(unsigned long long v, unsigned long long *wbuf) {
    v = wave_max_u64(v);
    const int lane = threadIdx.x & (kWave - 1), wid = threadIdx.x / kWave;
    if (lane == 0) wbuf[wid] = v;
    __syncthreads();
    unsigned long long r = 0;
#pragma unroll
    for (int w = 0; w < BS / kWave; ++w) r = wbuf[w] > r ? wbuf[w] : r;
    __syncthreads();
    return r;
}

// ---------------------------------------------------------------- topology helpers
// Applies delta to every link of the path between servers u != v chosen by
// candidate c: uplinks of u and v; with different edge switches the two
// edge-aggregation links through aggregation index a; with different pods
// the two aggregation-core links through core (a, j).  c = a (same pod) or
// a*h + j (different pods).
template <bool ATOMIC>
__device__ __forceinline__ void path_apply(const Topo &t, const State &st, int u, int v, int c, int delta) {
    const int eu = u / t.h, ev = v / t.h, pu = u / t.hh, pv = v / t.hh;
    int a = 0, j = 0;
    if (pu == pv) a = c; else { a = c / t.h; j = c - a * t.h; }
    int *l[6];
    int nl = 2;
    l[0] = st.up + u; l[1] = st.up + v;
    if (eu != ev) { l[2] = st.ea + eu * t.h + a; l[3] = st.ea + ev * t.h + a; nl = 4; }
    if (pu != pv) { l[4] = st.ac + (pu * t.h + a) * t.h + j; l[5] = st.ac + (pv * t.h + a) * t.h + j; nl = 6; }
    for (int x = 0; x < nl; ++x) {
        if (ATOMIC) atomicAdd(l[x], delta);
        else *l[x] += delta;
    }
}

// Widest minimum-hop path from u to v under the current residuals; ties go
// to the lowest aggregation then core index (candidate order).  Evaluated by
// one wave, candidates spread over lanes.  Returns key = bottleneck << 32 |
// ~candidate (bottlenecks are non-negative).
__device__ __forceinline__ unsigned long long widest_wave(const Topo &t, const State &st, int u, int v, int lane) {
    const int eu = u / t.h, ev = v / t.h, pu = u / t.hh, pv = v / t.hh;
    const int ncand = (eu == ev) ? 1 : (pu == pv ? t.h : t.hh);
    const int base = min(st.up[u], st.up[v]);
    unsigned long long best = 0;
    for (int c = lane; c < ncand; c += kWave) {
        int b = base;
        if (eu != ev) {
            const int a = (pu == pv) ? c : c / t.h;
            b = min(b, min(st.ea[eu * t.h + a], st.ea[ev * t.h + a]));
            if (pu != pv) {
                const int j = c - a * t.h;
                b = min(b, min(st.ac[(pu * t.h + a) * t.h + j], st.ac[(pv * t.h + a) * t.h + j]));
            }
        }
        const unsigned long long key = (static_cast<unsigned long long>(static_cast<unsigned>(b)) << 32) |
                                       static_cast<unsigned>(~c);
        best = key > best ? key : best;
    }
    return wave_max_u64(best);
}

// Commit container (cpu_i, ram_i) on server u with its P placed peers
// (servers ph[], demands pbw[], ascending container index): route each
// remote peer on its widest shortest path under the current residuals,
// failing when a bottleneck is below the demand (Eqs. (4)-(5)).  On failure
// every change is undone.  Run by one whole wave; lane 0 writes.
__device__ __forceinline__ bool commit_wave(const Topo &t, const State &st, int u, int cpu_i, int ram_i, int P,
                                            const int *ph, const int *pbw, int *code_out, int lane) {
    if (st.cpu[u] < cpu_i || st.ram[u] < ram_i) return false;
    int routed = 0;
    bool ok = true;
    for (int p = 0; p < P; ++p) {
        const int v = ph[p];
        if (v == u) {
            if (lane == 0) code_out[p] = -1;
            routed = p + 1;
            continue;
        }
        const unsigned long long best = widest_wave(t, st, u, v, lane);
        const int b = static_cast<int>(best >> 32);
        const int c = static_cast<int>(~static_cast<unsigned>(best & 0xffffffffu));
        if (b < pbw[p]) { ok = false; break; }
        if (lane == 0) {
            path_apply<false>(t, st, u, v, c, -pbw[p]);
            code_out[p] = c;
        }
        __threadfence_block();
        routed = p + 1;
    }
    if (!ok) {
        if (lane == 0)
            for (int p = routed - 1; p >= 0; --p)
                if (ph[p] != u) path_apply<false>(t, st, u, ph[p], code_out[p], pbw[p]);
        __threadfence_block();
        return false;
    }
    if (lane == 0) {
        st.cpu[u] -= cpu_i;
        st.ram[u] -= ram_i;
        st.npl[u] += 1;
    }
    __threadfence_block();
    return true;
}

// Gives back containers [0, upto) of request r: CPU, RAM, placed count and
// the demand of every routed peer pair.  Block-wide, with atomics.
template <int BS>
__device__ void give_back(const Topo &t, const State &st, const Batch &b, int r, int upto) {
    const int g0 = b.coff[r];
    const int p_beg = b.poff[g0], p_end = b.poff[g0 + upto];
    for (int q = p_beg + threadIdx.x; q < p_end; q += BS) {
        // container owning pair q: largest g with poff[g] <= q
        int lo = g0, hi = g0 + upto - 1;
        while (lo < hi) {
            const int mid = (lo + hi + 1) >> 1;
            if (b.poff[mid] <= q) lo = mid; else hi = mid - 1;
        }
        const int u = b.host[lo];
        const int v = b.host[g0 + b.pj[q]];
        const int c = b.code[q];
        if (u != v && c >= 0) path_apply<true>(t, st, u, v, c, b.pbw[q]);
    }
    for (int i = threadIdx.x; i < upto; i += BS) {
        const int u = b.host[g0 + i];
        atomicAdd(st.cpu + u, b.cpu[g0 + i]);
        atomicAdd(st.ram + u, b.ram[g0 + i]);
        atomicSub(st.npl + u, 1);
    }
}

// Request r found no server for container `upto`: undo containers
// [0, upto) (all or nothing) and mark the request rejected.  host[] keeps
// the servers the undone containers had been given (attempt record).
template <int BS>
__device__ void rollback_request(const Topo &t, const State &st, const Batch &b, int r, int upto) {
    give_back<BS>(t, st, b, r, upto);
    __syncthreads();
    if (threadIdx.x == 0) {
        b.status[r] = 0;
        b.failat[r] = upto;
        b.tse[r] = dev_clock();
    }
    __threadfence_block();
    __syncthreads();
}

// ---------------------------------------------------------------- path stage + criteria
// Peer tables for the peers [pbeg, pbeg+pn) (section V-D routing on a
// fat-tree, per destination server v in pod pv and edge switch ev):
//   T[ag] = max_j min(ac(ag, j), ac((pv, a), j))  for aggregation (p, a), p != pv
//   E[eg] = max_a min(ea(eg, a), ea(ev, a), T[(p, a)] or +inf in pod pv)   eg != ev
// so that the widest shortest path from u to v has bottleneck
// min(up[u], up[v], E[edge(u)]) (or min(up[u], up[v]) on the same edge).
template <int BS>
__device__ __forceinline__ void build_tables(const Topo &t, const State &st, const Smem &sm, int pbeg, int pn) {
    const int tot = pn * t.nsw;
    for (int it = threadIdx.x; it < tot; it += BS) {
        const int pc = it / t.nsw, ag = it - pc * t.nsw;
        const int v = sm.ph[pbeg + pc];
        const int pv = v / t.hh, pa = ag / t.h;
        int val = 0;
        if (pa != pv) {
            const int a = ag - pa * t.h;
            const int *x = st.ac + ag * t.h;
            const int *y = st.ac + (pv * t.h + a) * t.h;
            for (int j = 0; j < t.h; ++j) val = max(val, min(x[j], y[j]));
        }
        sm.tabT[it] = val;
    }
    __syncthreads();
    for (int it = threadIdx.x; it < tot; it += BS) {
        const int pc = it / t.nsw, eg = it - pc * t.nsw;
        const int v = sm.ph[pbeg + pc];
        const int ev = v / t.h, pv = v / t.hh, pe = eg / t.h;
        int val = 0;
        if (eg != ev) {
            const int *x = st.ea + eg * t.h;
            const int *y = st.ea + ev * t.h;
            const int *T = sm.tabT + pc * t.nsw + pe * t.h;
            for (int a = 0; a < t.h; ++a) {
                int w = min(x[a], y[a]);
                if (pe != pv) w = min(w, T[a]);
                val = max(val, w);
            }
        }
        sm.tabE[it] = val;
    }
    __syncthreads();
}

// Per-host criteria for one container.  xs rows (N ints each): [0, nc) the
// criteria values, nc the feasibility flag, nc+1..nc+3 partial accumulators
// kept across peer chunks.  Accumulates the TOPSIS column statistics
// (sum of squares, max, min) when STATS.
template <int BS, bool STATS>
__device__ void criteria_stage(const Topo &t, const State &st, const Method &m, const Smem &sm, int *xs,
                               int cpu_i, int ram_i, int P, int pc_cap, unsigned long long *s2, int *mx, int *mn) {
    const int N = t.N, nc = m.nc;
    const int nch = P == 0 ? 1 : (P + pc_cap - 1) / pc_cap;
    for (int ch = 0; ch < nch; ++ch) {
        const int pbeg = ch * pc_cap;
        const int pn = min(P, pbeg + pc_cap) - pbeg;
        if (pn > 0) build_tables<BS>(t, st, sm, pbeg, pn);
        for (int u = threadIdx.x; u < N; u += BS) {
            const int up_u = st.up[u];
            int pbw_acc, up_acc, hop_acc, feas;
            if (ch == 0) {
                pbw_acc = up_u; up_acc = 0; hop_acc = 0;
                feas = (st.cpu[u] >= cpu_i) & (st.ram[u] >= ram_i);
            } else {
                feas = xs[nc * N + u];
                pbw_acc = xs[(nc + 1) * N + u];
                up_acc = xs[(nc + 2) * N + u];
                hop_acc = xs[(nc + 3) * N + u];
            }
            const int eu = u / t.h, pu = u / t.hh;
            for (int pc = 0; pc < pn; ++pc) {
                const int v = sm.ph[pbeg + pc];
                if (v == u) continue;                 // co-located peer: no link
                const int bw = sm.pbw[pbeg + pc];
                int w = min(up_u, sm.upv[pbeg + pc]);
                int hop = 2;
                if (v / t.h != eu) {
                    w = min(w, sm.tabE[pc * t.nsw + eu]);
                    hop = (v / t.hh == pu) ? 4 : 6;
                }
                pbw_acc = min(pbw_acc, w);
                up_acc += bw;
                hop_acc += hop;
                feas &= (w >= bw);
            }
            if (ch + 1 < nch) {
                xs[nc * N + u] = feas;
                xs[(nc + 1) * N + u] = pbw_acc;
                xs[(nc + 2) * N + u] = up_acc;
                xs[(nc + 3) * N + u] = hop_acc;
                continue;
            }
            feas &= (up_u >= up_acc);
            xs[nc * N + u] = feas;
#pragma unroll
            for (int c = 0; c < kMaxCrit; ++c) {
                if (c >= nc) break;
                int x;
                switch (m.crit[c]) {
                case CRIT_CPU: x = st.cpu[u]; break;
                case CRIT_RAM: x = st.ram[u]; break;
                case CRIT_ACTIVE: x = st.npl[u] > 0 ? 1 : 0; break;
                case CRIT_PATHBW: x = pbw_acc; break;
                case CRIT_UPLINK: x = up_u; break;
                default: x = hop_acc; break;
                }
                xs[c * N + u] = x;
                if (STATS) {
                    s2[c] += static_cast<unsigned long long>(static_cast<long long>(x) * x);
                    mx[c] = max(mx[c], x);
                    mn[c] = min(mn[c], x);
                }
            }
        }
        if (ch + 1 < nch) __syncthreads();
    }
}

// Loads the peer list of container g into LDS.  Returns P.
template <int BS>
__device__ __forceinline__ int load_peers(const State &st, const Batch &b, const Smem &sm, int g0, int g) {
    const int p0 = b.poff[g], P = b.poff[g + 1] - p0;
    for (int p = threadIdx.x; p < P; p += BS) {
        const int v = b.host[g0 + b.pj[p0 + p]];
        sm.ph[p] = v;
        sm.pbw[p] = b.pbw[p0 + p];
        sm.upv[p] = st.up[v];
    }
    __syncthreads();
    return P;
}

__device__ __forceinline__ unsigned long long score_key(float s, int u) {
    return (static_cast<unsigned long long>(__float_as_uint(s)) << 32) | static_cast<unsigned>(~u);
}

// Trace slot of this step, or -1.  Called by thread 0 only.
__device__ __forceinline__ int trace_slot(const Trace &tr, int inst, int r, int i) {
    if (tr.stride <= 0) return -1;
    const int s = tr.counter[inst];
    tr.counter[inst] = s + 1;
    if (s % tr.stride) return -1;
    const int slot = s / tr.stride;
    if (slot >= tr.cap) return -1;
    tr.meta[4 * slot + 0] = inst;
    tr.meta[4 * slot + 1] = r;
    tr.meta[4 * slot + 2] = i;
    tr.meta[4 * slot + 3] = s;
    return slot;
}

// Select-and-commit loop shared by TOPSIS and AHP: keys come from
// key_of(u) (0 = infeasible).  Visits servers in decreasing key order by
// repeated block argmax; a server whose commit fails is masked in the
// feasibility row and the argmax repeats.  Rolls the request back when no
// server is left.  Returns true when the container was placed.
template <int BS, class KeyFn>
__device__ bool select_commit(const Topo &t, const State &st, const Batch &b, const Smem &sm, int *feas_row,
                              int r, int i, int n, int g, int P, int cpu_i, int ram_i, KeyFn key_of) {
    const int lane = threadIdx.x & (kWave - 1);
    for (;;) {
        unsigned long long kb = 0;
        for (int u = threadIdx.x; u < t.N; u += BS) {
            if (!feas_row[u]) continue;
            const unsigned long long k = key_of(u);
            kb = k > kb ? k : kb;
        }
        kb = block_max_u64<BS>(kb, sm.wkey);
        if (kb == 0) {
            rollback_request<BS>(t, st, b, r, i);
            return false;
        }
        const int u = static_cast<int>(~static_cast<unsigned>(kb & 0xffffffffu));
        if (threadIdx.x < kWave) {
            const int p0 = b.poff[g];
            const bool ok = commit_wave(t, st, u, cpu_i, ram_i, P, sm.ph, sm.pbw, b.code + p0, lane);
            if (lane == 0) {
                sm.misc[0] = ok;
                if (ok) {
                    b.host[g] = u;
                    b.score[g] = __uint_as_float(static_cast<unsigned>(kb >> 32));
                    if (i == n - 1) b.tse[r] = dev_clock();
                } else {
                    feas_row[u] = 0;
                }
            }
        }
        __threadfence_block();
        __syncthreads();
        const int ok = sm.misc[0];
        __syncthreads();
        if (ok) return true;
    }
}

// ---------------------------------------------------------------- TOPSIS step (section V-C)
// Scores every server by closeness to the ideal solution: column L2
// normalisation and weighting fold into q_c = w_c^2 / sum_u x_cu^2, so
// Ed+- = sqrt(sum_c q_c (x_cu - A+-_c)^2) with A+- the column max / min in
// raw units (swapped for cost criteria); Rank = Ed- / (Ed+ + Ed-), 0 when
// both are 0.  Column statistics are exact integer reductions.
template <int BS>
__device__ void topsis_step(const Topo &t, const State &st, const Method &m, const Batch &b, const Smem &sm,
                            int *xs, int pc_cap, const Trace &tr, int inst, int r, int i) {
    const int g0 = b.coff[r];
    const int n = b.coff[r + 1] - g0;
    const int g = g0 + i;
    if (b.status[r] == 0) return;
    if (i == 0 && threadIdx.x == 0) b.tsb[r] = dev_clock();
    const int cpu_i = b.cpu[g], ram_i = b.ram[g];
    const int P = load_peers<BS>(st, b, sm, g0, g);
    const int nc = m.nc, N = t.N;

    unsigned long long s2[kMaxCrit];
    int mx[kMaxCrit], mn[kMaxCrit];
#pragma unroll
    for (int c = 0; c < kMaxCrit; ++c) { s2[c] = 0; mx[c] = -kBig; mn[c] = kBig; }
    criteria_stage<BS, true>(t, st, m, sm, xs, cpu_i, ram_i, P, pc_cap, s2, mx, mn);

    // column statistics: wave then block reduction
    const int lane = threadIdx.x & (kWave - 1), wid = threadIdx.x / kWave;
#pragma unroll
    for (int c = 0; c < kMaxCrit; ++c) {
        if (c >= nc) break;
        const unsigned long long a = wave_sum_u64(s2[c]);
        const int hi = wave_max_i(mx[c]), lo = wave_min_i(mn[c]);
        if (lane == 0) { sm.ws2[wid * kMaxCrit + c] = a; sm.wmx[wid * kMaxCrit + c] = hi; sm.wmn[wid * kMaxCrit + c] = lo; }
    }
    __syncthreads();
    if (threadIdx.x < nc) {
        const int c = threadIdx.x;
        unsigned long long a = 0;
        int hi = -kBig, lo = kBig;
        for (int w = 0; w < BS / kWave; ++w) {
            a += sm.ws2[w * kMaxCrit + c];
            hi = max(hi, sm.wmx[w * kMaxCrit + c]);
            lo = min(lo, sm.wmn[w * kMaxCrit + c]);
        }
        const double wc = m.w[c];
        sm.q[c] = a ? static_cast<float>(wc * wc / static_cast<double>(a)) : 0.0f;
        sm.ap[c] = static_cast<float>(m.cost[c] ? lo : hi);
        sm.am[c] = static_cast<float>(m.cost[c] ? hi : lo);
    }
    if (threadIdx.x == 0) sm.misc[1] = trace_slot(tr, inst, r, i);
    __syncthreads();

    float q[kMaxCrit], ap[kMaxCrit], am[kMaxCrit];
#pragma unroll
    for (int c = 0; c < kMaxCrit; ++c) {
        q[c] = c < nc ? sm.q[c] : 0.f;
        ap[c] = c < nc ? sm.ap[c] : 0.f;
        am[c] = c < nc ? sm.am[c] : 0.f;
    }
    auto closeness = [&](int u) -> float {
        float dp2 = 0.f, dm2 = 0.f;
#pragma unroll
        for (int c = 0; c < kMaxCrit; ++c) {
            if (c >= nc) break;
            const float x = static_cast<float>(xs[c * N + u]);
            const float a = x - ap[c], z = x - am[c];
            dp2 = fmaf(q[c] * a, a, dp2);
            dm2 = fmaf(q[c] * z, z, dm2);
        }
        const float dp = sqrtf(dp2), dm = sqrtf(dm2);
        const float den = dp + dm;
        return den > 0.f ? dm / den : 0.f;
    };
    const int slot = sm.misc[1];
    if (slot >= 0)
        for (int u = threadIdx.x; u < N; u += BS) tr.scores[static_cast<size_t>(slot) * N + u] = closeness(u);
    select_commit<BS>(t, st, b, sm, xs + nc * N, r, i, n, g, P, cpu_i, ram_i,
                      [&](int u) { return score_key(closeness(u), u); });
}

}  // namespace dcs
