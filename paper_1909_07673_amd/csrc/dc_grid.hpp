// Cooperative container step for large data centers: one workgroup per pod
// (k workgroups, launched cooperatively so that all are resident).  Each
// workgroup builds the path tables for its own pod's aggregation and edge
// switches, scores its pod's servers; the column statistics and the
// capacity sums are exchanged through tagged per-workgroup records, the
// argmax and the commit's outcome through tagged slots (selection rounds),
// so that a step has no grid barrier; workgroup 0 commits.  Same arithmetic as the single-workgroup step, so
// results are bit-identical.  Used by the plain form (one cooperative launch
// per container step) and the serving form (one persistent cooperative
// kernel) when k is large.
#pragma once
#include "dc_serve.hpp"

namespace dcs {

// Threads per pod workgroup.  The step is bound by memory latency and the
// waits between workgroups, not by threads: 1024 threads measured no faster
// than 256.
constexpr int kGridBlock = 256;

// Cross-workgroup state, in device memory.
struct GridCtl {
    unsigned *count, *gen;        // grid barrier: arrivals, generation
    int *err;                     // set when a barrier wait timed out
    unsigned long long *kslot;    // [2][G] per-workgroup best key of a selection round, tagged
    unsigned long long *rflag;    // outcome of a selection round's commit, tagged
    unsigned long long *rec;      // [G][kRecWords] per-workgroup records of a step, tagged (below)
    unsigned *round;              // selection rounds so far (kept across launches)
    int *flag;                    // [kGridFlags]: command buffers
};

// Selection rounds.  Round r of the argmax and commit needs no grid barrier:
// each workgroup publishes its best key in its own slot of set r & 1 as one
// 64-bit word, tagged with r, which a wave of every workgroup polls until all
// slots carry r (the payload is the word itself, so no fence is needed);
// workgroup 0 then commits and publishes the outcome tagged with r (release),
// which the others poll for (acquire).  A workgroup publishes round r + 2 in
// the same slot only after the outcome of round r + 1, which workgroup 0
// gives only after reading every slot of round r + 1, so nothing is
// overwritten before every workgroup has read it.  Keys are packed as
// (score bits + 1) << 17 | (2^17 - 1 - server) (servers below 2^17), the tag
// in bits 47..63; tags never are 0, which the slots hold initially.
constexpr int kRoundTagShift = 47;
constexpr unsigned long long kRoundPayload = (1ull << kRoundTagShift) - 1;
__device__ __forceinline__ unsigned long long round_tag(unsigned r) {
    return static_cast<unsigned long long>((r & 0xffffu) | 0x10000u) << kRoundTagShift;
}
__device__ __forceinline__ unsigned long long round_key(unsigned long long kb) {
    if (!kb) return 0ull;
    const unsigned u = ~static_cast<unsigned>(kb);
    return ((kb >> 32) << 17) | (0x1ffffu - u);
}

// Wave: waits until the G slots of round r all carry its tag and returns the
// largest payload, or sets bad when the wait timed out or a workgroup
// reported an error.
__device__ __forceinline__ unsigned long long round_max(const GridCtl &g, unsigned r, long long timeout,
                                                        bool &bad) {
    const int lane = threadIdx.x & (kWave - 1), G = gridDim.x;
    const unsigned long long *sl = g.kslot + (r & 1) * G, tag = round_tag(r);
    const long long t0 = dev_clock();
    for (;;) {
        bool ok = true;
        unsigned long long m = 0;
        for (int x = lane; x < G; x += kWave) {
            const unsigned long long v = __hip_atomic_load(sl + x, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            ok &= (v & ~kRoundPayload) == tag;
            const unsigned long long pv = v & kRoundPayload;
            m = pv > m ? pv : m;
        }
        if (__all(ok)) {
            const unsigned hiw = wave_umax(static_cast<unsigned>(m >> 32));
            const unsigned low = wave_umax(static_cast<unsigned>(m >> 32) == hiw ? static_cast<unsigned>(m) : 0u);
            return (static_cast<unsigned long long>(hiw) << 32) | low;
        }
        if (__hip_atomic_load(g.err, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) || dev_clock() - t0 > timeout) {
            if (lane == 0) __hip_atomic_store(g.err, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            bad = true;
            return 0ull;
        }
    }
}

// Thread: waits for workgroup 0's outcome of round r; -1 when the wait
// timed out or a workgroup reported an error.
__device__ __forceinline__ int round_outcome(const GridCtl &g, unsigned r, long long timeout) {
    const unsigned long long tag = round_tag(r);
    const long long t0 = dev_clock();
    for (;;) {
        const unsigned long long v = __hip_atomic_load(g.rflag, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        if ((v & ~kRoundPayload) == tag) {
            __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
            return static_cast<int>(v & 3u);
        }
        if (__hip_atomic_load(g.err, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) || dev_clock() - t0 > timeout) {
            __hip_atomic_store(g.err, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            return -1;
        }
        __builtin_amdgcn_s_sleep(1);
    }
}

// flag[8 + 8 * (pos & 1) ...]: the command at ring position pos,
// double-buffered so that the leader can publish command pos + 1 while a
// slower workgroup still reads command pos.
constexpr int kGridFlags = 24;
enum { GF_GOT = 0, GF_TYPE, GF_N, GF_NPAIR, GF_SLOT, GF_RID };
__device__ __forceinline__ int *cmd_flags(const GridCtl &g, int pos) { return g.flag + 8 + 8 * (pos & 1); }

// Grid barrier over gridDim.x co-resident workgroups with agent-scope
// release / acquire.  A wait longer than `timeout` device ticks sets *err;
// every barrier returns false once *err is set, so all workgroups leave.
// Ordering: each arrival's fetch_add releases the workgroup's writes (after
// the block barrier) and acquires the earlier arrivals'; the last arrival
// publishes the next generation with a release store; the others poll it
// with relaxed loads and take one acquire fence once it has changed.  The
// generation is read before arriving, which the release of the fetch_add
// keeps in place.  No other fence is needed, and on a device of several
// XCDs each one costs a second-level cache writeback or invalidation.
__device__ __forceinline__ bool grid_sync(const GridCtl &g, int *lds_flag, long long timeout) {
    __syncthreads();
    if (threadIdx.x == 0) {
        int bad = __hip_atomic_load(g.err, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        if (!bad) {
            const unsigned gen = __hip_atomic_load(g.gen, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            const unsigned arrived = __hip_atomic_fetch_add(g.count, 1u, __ATOMIC_ACQ_REL, __HIP_MEMORY_SCOPE_AGENT);
            if (arrived == gridDim.x - 1) {
                __hip_atomic_store(g.count, 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                __hip_atomic_store(g.gen, gen + 1, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
            } else {
                const long long t0 = dev_clock();
                while (__hip_atomic_load(g.gen, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) == gen) {
                    if (__hip_atomic_load(g.err, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)) { bad = 1; break; }
                    if (dev_clock() - t0 > timeout) {
                        __hip_atomic_store(g.err, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                        bad = 1;
                        break;
                    }
                    __builtin_amdgcn_s_sleep(1);
                }
                __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
            }
        }
        *lds_flag = bad;
    }
    __syncthreads();
    return !*lds_flag;
}

// Records of a step: instead of a grid barrier, each workgroup publishes
// its column-statistics partials, its edge switches' and its pod's summed
// residuals (and workgroup 0 the trace slot) as 64-bit words, the value in
// the low half and in the high half a tag made of the number of the step's
// first selection round with the top bit set (never 0, which the words hold
// initially); a reader polls a word until it carries that tag, so no fence
// is needed.  Every word is written at every step, a step has fewer than
// 2^31 rounds, so a word read with the current tag was written in this step.
// A workgroup writes the next step's record only after this step's last
// selection round, whose outcome needs every workgroup's key, which each
// publishes after it has read the records.
__device__ __forceinline__ unsigned long long rec_tag(unsigned r) {
    return static_cast<unsigned long long>(r | 0x80000000u) << 32;
}
constexpr int kRecWords = 80;
constexpr int kRecCapE = 5 * kMaxCrit;            // then h edge switches (h <= 32)
constexpr int kRecCapP = kRecCapE + 32;
constexpr int kRecTrace = kRecCapP + 1;
static_assert(kRecTrace < kRecWords, "record layout");

__device__ __forceinline__ void rec_put(const GridCtl &g, int w, int x, unsigned long long tag, int v) {
    __hip_atomic_store(g.rec + static_cast<size_t>(w) * kRecWords + x, tag | static_cast<unsigned>(v),
                       __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

__device__ __forceinline__ unsigned long long rec_load(const GridCtl &g, int w, int x) {
    return __hip_atomic_load(g.rec + static_cast<size_t>(w) * kRecWords + x, __ATOMIC_RELAXED,
                             __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ bool rec_has(unsigned long long v, unsigned long long tag) { return (v >> 32) == (tag >> 32); }

// Thread: n words of the records (workgroup ws[j], word xs[j]) once all
// carry tag, every poll with all its loads in flight together; false when
// the wait timed out or a workgroup reported an error.
template <int NW>
__device__ __forceinline__ bool rec_get(const GridCtl &g, int n, const int (&ws)[NW], const int (&xs)[NW],
                                        unsigned long long tag, long long timeout, int (&v)[NW]) {
    const long long t0 = dev_clock();
    for (;;) {
        bool ok = true;
#pragma unroll
        for (int j = 0; j < NW; ++j)
            if (j < n) {
                const unsigned long long r = rec_load(g, ws[j], xs[j]);
                ok &= rec_has(r, tag);
                v[j] = static_cast<int>(static_cast<unsigned>(r));
            }
        if (ok) return true;
        if (__hip_atomic_load(g.err, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) || dev_clock() - t0 > timeout) {
            __hip_atomic_store(g.err, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            return false;
        }
        __builtin_amdgcn_s_sleep(1);
    }
}

// LDS of the cooperative step (per workgroup): peers, own-pod tables and
// capacities, per-server scratch of the pod, statistics slots.
struct GSmem {
    int4 *pk;                     // [kMaxN] packed peers (as in Smem)
    int *wst;                     // [kStatFields][kMaxWaves]
    int *misc;                    // [M_MISC]
    int *capE;                    // [h] own edge switches
    int *tabT, *tabE;             // [kMaxN][h]
    int *xs;                      // [nc+6][hh]
    int *pcap;                    // [2][kMaxN] peers' edge-switch and pod capacities
};

__host__ __device__ inline size_t gsmem_bytes(int h, int hh, int nc) {
    return sizeof(int4) * kMaxN + sizeof(int) * (kStatFields * kMaxWaves + M_MISC + align4(h) +
                                                 2 * align4((size_t)kMaxN * h) + (size_t)(nc + 6) * hh +
                                                 2 * kMaxN);
}

__device__ inline GSmem gcarve(char *base, int h, int hh, int nc) {
    GSmem s;
    s.pk = reinterpret_cast<int4 *>(base);
    int *p = reinterpret_cast<int *>(base + sizeof(int4) * kMaxN);
    s.wst = p; p += kStatFields * kMaxWaves;
    s.misc = p; p += M_MISC;
    s.capE = p; p += align4(h);
    s.tabT = p; p += align4((size_t)kMaxN * h);
    s.tabE = p; p += align4((size_t)kMaxN * h);
    s.xs = p; p += (size_t)(nc + 6) * hh;
    s.pcap = p;
    return s;
}

// Sum of v over the block; the result is valid in every thread after the
// call (uses misc[M_MISC-1] and one LDS barrier pair).
template <int BS>
__device__ __forceinline__ int block_sum(int v, int *slot) {
    v = wave_sum(v);
    if (threadIdx.x == 0) *slot = 0;
    __syncthreads();
    if ((threadIdx.x & (kWave - 1)) == 0) atomicAdd(slot, v);
    __syncthreads();
    const int r = *slot;
    __syncthreads();
    return r;
}

// One container step on the pod of this workgroup (w = blockIdx.x).
// rv.hosts_out, when given, is this workgroup's LDS copy of the request's
// servers.  Returns false when the request was rejected at this container.
template <int BS, int CS = 0>
__device__ __forceinline__ bool grid_topsis_step(const Topo &t, const State &st, const Method &m, const Batch &b,
                                                 const GSmem &sm, const GridCtl &g, long long timeout, const StepIn &s,
                                                 const ReqView &rv, const Trace &tr, unsigned &rnd) {
    const int w = blockIdx.x, G = gridDim.x, h = t.h, hh = t.hh, nc = crit_count<CS>(m);
    const int lane = threadIdx.x & (kWave - 1), wid = threadIdx.x / kWave;
    const int P = s.P, ubase = w * hh;
    int *xs = sm.xs;
    const unsigned long long stag = rec_tag(rnd);     // this step's records
    int my_slot = -1;                                   // trace slot (workgroup 0, thread 0)
    if (w == 0 && threadIdx.x == 0) {
        if (s.i == 0) b.tsb[s.r] = dev_clock();
        if (tr.stride > 0) my_slot = trace_slot(tr, 0, b.rid[s.r], s.i);
    }
    // ---- A: peers, own capacities
    for (int p = threadIdx.x; p < P; p += BS) {
        const int v = rv.hosts[rv.pj[p]];
        sm.pk[p] = make_int4(v, edge_of(t, v) | (pod_of(t, v) << 16), rv.pbw[p], st.up[v]);
    }
    for (int e = threadIdx.x; e < h; e += BS) {
        int se = 0;
        for (int a = 0; a < h; ++a) se += st.ea[(w * h + e) * h + a];
        sm.capE[e] = se;
    }
    int cp = 0;
    for (int x = threadIdx.x; x < hh; x += BS) cp += st.ac[w * hh + x];
    // the deficit slots and the error flag of phase D, reset here so that
    // the barriers below order them before their use
    if (threadIdx.x < 6) sm.misc[M_DH0 + threadIdx.x] = (threadIdx.x & 1) ? -1 : kBig;
    if (threadIdx.x == 6) sm.misc[M_OK] = 0;
    const int capP_own = block_sum<BS>(cp, sm.misc + M_MISC - 1);   // ends with barriers
    // ---- B: path tables for this pod (T: its aggregation switches, E: its edge switches)
    for (int it = threadIdx.x; it < P * h; it += BS) {
        const int pc = it / h, a = it - pc * h;
        const int pv = sm.pk[pc].y >> 16;
        int val = 0;
        if (pv != w) {
            const int *x = st.ac + (w * h + a) * h, *y = st.ac + (pv * h + a) * h;
            for (int j = 0; j < h; ++j) val = max(val, min(x[j], y[j]));
        }
        sm.tabT[pc * h + a] = val;
    }
    __syncthreads();
    for (int it = threadIdx.x; it < P * h; it += BS) {
        const int pc = it / h, e = it - pc * h;
        const int ed = sm.pk[pc].y, ev = ed & 0xffff, pv = ed >> 16, eg = w * h + e;
        int val = 0;
        if (eg != ev) {
            const int *x = st.ea + eg * h, *y = st.ea + ev * h, *T = sm.tabT + pc * h;
            const int lim = pv != w ? 0 : kBig;
            for (int a = 0; a < h; ++a) val = max(val, min(min(x[a], y[a]), max(T[a], lim)));
        }
        sm.tabE[pc * h + e] = val;
    }
    __syncthreads();
    // ---- C: criteria of the pod's servers, partial column statistics
    unsigned long long s2[kMaxCrit];
    int mx[kMaxCrit], mn[kMaxCrit];
#pragma unroll
    for (int c = 0; c < kMaxCrit; ++c) { s2[c] = 0; mx[c] = -kBig - 1; mn[c] = kBig; }
    for (int x = threadIdx.x; x < hh; x += BS) {
        const int u = ubase + x;
        const int up_u = st.up[u], el = edge_of(t, x), eu = w * h + el;
        int pbw_acc = up_u, up_acc = 0, hop_acc = 0, oute = 0, outp = 0;
        int feas = (st.cpu[u] >= s.cpu) & (st.ram[u] >= s.ram);
        for (int pc = 0; pc < P; ++pc) {
            const int4 pk = sm.pk[pc];
            const int v = pk.x, bw = pk.z, ev = pk.y & 0xffff, pv = pk.y >> 16;
            const bool rem = v != u, far = ev != eu;
            int wv = min(up_u, pk.w);
            wv = far ? min(wv, sm.tabE[pc * h + el]) : wv;
            pbw_acc = rem ? min(pbw_acc, wv) : pbw_acc;
            up_acc += rem ? bw : 0;
            hop_acc += !rem ? 0 : !far ? 2 : (pv == w ? 4 : 6);
            feas &= (!rem) | (wv >= bw);
            oute += (rem & far) ? bw : 0;
            outp += (rem & far & (pv != w)) ? bw : 0;
        }
        feas &= (up_u >= up_acc);
        if (P > 0 && !m.route_end) feas &= (sm.capE[el] >= oute) & (capP_own >= outp);
        xs[nc * hh + x] = feas;
#pragma unroll
        for (int c = 0; c < kMaxCrit; ++c) {
            if (c >= nc) break;
            int v;
            switch (crit_at<CS>(m, c)) {
            case CRIT_CPU: v = st.cpu[u]; break;
            case CRIT_RAM: v = st.ram[u]; break;
            case CRIT_ACTIVE: v = st.npl[u] > 0 ? 1 : 0; break;
            case CRIT_PATHBW: v = pbw_acc; break;
            case CRIT_UPLINK: v = up_u; break;
            default: v = hop_acc; break;
            }
            xs[c * hh + x] = v;
            s2[c] += static_cast<unsigned long long>(static_cast<long long>(v) * v);
            mx[c] = max(mx[c], v);
            mn[c] = min(mn[c], v);
        }
    }
#pragma unroll
    for (int c = 0; c < kMaxCrit; ++c) {
        if (c >= nc) break;
        const int c0 = wave_sum(static_cast<int>(s2[c] & 0x1ffffu));
        const int c1 = wave_sum(static_cast<int>((s2[c] >> 17) & 0x1ffffu));
        const int c2 = wave_sum(static_cast<int>(s2[c] >> 34));
        const int hi = wave_max(mx[c]), lo = wave_min(mn[c]);
        if (lane < 5) sm.wst[(5 * c + lane) * kMaxWaves + wid] =
            lane == 0 ? c0 : lane == 1 ? c1 : lane == 2 ? c2 : lane == 3 ? hi : -lo;
    }
    __syncthreads();
    // this workgroup's record: statistics partials, own capacities for the
    // other pods' checks, and (workgroup 0) the trace slot
    for (int f = threadIdx.x; f < 5 * nc; f += BS) {
        int v = (f % 5) < 3 ? 0 : -kBig - 1;
        for (int x = 0; x < BS / kWave; ++x) {
            const int pv = sm.wst[f * kMaxWaves + x];
            v = (f % 5) < 3 ? v + pv : max(v, pv);
        }
        rec_put(g, w, f, stag, v);
    }
    for (int e = threadIdx.x; e < h; e += BS) rec_put(g, w, kRecCapE + e, stag, sm.capE[e]);
    if (threadIdx.x == 0) {
        rec_put(g, w, kRecCapP, stag, capP_own);
        if (w == 0) rec_put(g, 0, kRecTrace, stag, my_slot);
    }
    // ---- D: block totals, peer-side deficits, scores, workgroup best
    // One poll per thread of all it needs from the records, waiting until
    // every word carries this step's tag: in every wave, lane x the
    // statistics words of workgroup x (G <= 64; the lanes past G read
    // workgroup 0's and count identities instead), and thread p < P (P <=
    // 63) the capacity words of peer p's edge switch and pod (the other
    // threads read their own pod's word in their place).
    constexpr int NF = 5 * (CS ? CS : kMaxCrit);
    const bool hp = static_cast<int>(threadIdx.x) < P;
    const int4 me = hp ? sm.pk[threadIdx.x] : make_int4(-1, 0, 0, 0);
    bool bad = false;
    int fv[NF];
    int cv[2];
    {
        int ww[NF + 2], wx[NF + 2], wv[NF + 2];
        const int e = me.y & 0xffff, d = me.y >> 16;
        ww[0] = hp ? e / h : w;
        wx[0] = hp ? kRecCapE + e % h : kRecCapP;
        ww[1] = hp ? d : w;
        wx[1] = kRecCapP;
#pragma unroll
        for (int f = 0; f < NF; ++f) {
            ww[2 + f] = lane < G ? lane : 0;
            wx[2 + f] = f;
        }
        bad = !rec_get(g, 2 + 5 * nc, ww, wx, stag, timeout, wv);
        cv[0] = wv[0];
        cv[1] = wv[1];
#pragma unroll
        for (int f = 0; f < NF; ++f) fv[f] = lane < G ? wv[2 + f] : ((f % 5) < 3 ? 0 : -kBig - 1);
    }
    unsigned long long S2[kMaxCrit];
    int MX[kMaxCrit], MN[kMaxCrit];
#pragma unroll
    for (int c = 0; c < kMaxCrit; ++c) {
        S2[c] = 0;
        MX[c] = MN[c] = 0;
        if (c >= nc || 5 * c >= NF) continue;
        int a0 = fv[5 * c], a1 = fv[5 * c + 1], a2 = fv[5 * c + 2], hi = fv[5 * c + 3], nlo = fv[5 * c + 4];
        a0 = wave_sum(a0);
        a1 = wave_sum(a1);
        a2 = wave_sum(a2);
        S2[c] = static_cast<unsigned long long>(static_cast<unsigned>(a0)) +
                (static_cast<unsigned long long>(static_cast<unsigned>(a1)) << 17) +
                (static_cast<unsigned long long>(static_cast<unsigned>(a2)) << 34);
        MX[c] = wave_max(hi);
        MN[c] = -wave_max(nlo);
    }
    // peer-side deficits (server uplink, edge switch, pod) as in the
    // single-workgroup step; they only narrow the candidates (slots reset
    // in phase A)
    if (hp) {
        const int v = me.x, e = me.y & 0xffff, d = me.y >> 16;
        int sh = 0, se = 0, sp = 0;
        for (int q = 0; q < P; ++q) {
            const int4 o = sm.pk[q];
            sh += o.x == v ? o.z : 0;
            se += (o.y & 0xffff) == e ? o.z : 0;
            sp += (o.y >> 16) == d ? o.z : 0;
        }
        if (me.w < sh) { atomicMin(sm.misc + M_DH0, v); atomicMax(sm.misc + M_DH1, v); }
        if (cv[0] < se) {
            atomicMin(sm.misc + M_DE0, e);
            atomicMax(sm.misc + M_DE1, e);
        }
        if (cv[1] < sp) {
            atomicMin(sm.misc + M_DP0, d);
            atomicMax(sm.misc + M_DP1, d);
        }
    }
    int slot = -1;
    if (tr.stride > 0) {
        const int zw[1] = {0}, zx[1] = {kRecTrace};
        int zv[1];
        bad |= !rec_get(g, 1, zw, zx, stag, timeout, zv);
        slot = zv[0];
    }
    if (bad) sm.misc[M_OK] = 1;
    __syncthreads();
    if (sm.misc[M_OK]) return false;
    const int dh0 = sm.misc[M_DH0], dh1 = sm.misc[M_DH1], de0 = sm.misc[M_DE0], de1 = sm.misc[M_DE1];
    const int dp0 = sm.misc[M_DP0], dp1 = sm.misc[M_DP1];
    float q[kMaxCrit], ap[kMaxCrit], am[kMaxCrit];
#pragma unroll
    for (int c = 0; c < kMaxCrit; ++c) {
        q[c] = ap[c] = am[c] = 0.f;
        if (c >= nc) continue;
        q[c] = S2[c] ? (m.w[c] * m.w[c]) / static_cast<float>(S2[c]) : 0.0f;
        ap[c] = static_cast<float>(crit_cost<CS>(m, c) ? MN[c] : MX[c]);
        am[c] = static_cast<float>(crit_cost<CS>(m, c) ? MX[c] : MN[c]);
    }
    auto key_of = [&](int x) -> unsigned long long {
        const int u = ubase + x;
        int f = xs[nc * hh + x];
        if (!m.route_end) {
            f &= (dh1 < 0) | ((dh0 == dh1) & (u == dh0));
            f &= (de1 < 0) | ((de0 == de1) & (w * h + edge_of(t, x) == de0));
            f &= (dp1 < 0) | ((dp0 == dp1) & (w == dp0));
        }
        if (!f) return 0ull;
        return score_key(topsis_close(nc, [&](int c) { return xs[c * hh + x]; }, q, ap, am), u);
    };
    // the workgroup's best key (largest packed key) into LDS slot 0..1
    auto wg_best = [&]() {
        unsigned long long kb = 0;
        for (int x = threadIdx.x; x < hh; x += BS) {
            const unsigned long long k = key_of(x);
            kb = k > kb ? k : kb;
        }
        unsigned hiw = wave_umax(static_cast<unsigned>(kb >> 32));
        unsigned low = wave_umax(static_cast<unsigned>(kb >> 32) == hiw ? static_cast<unsigned>(kb) : 0u);
        if (lane == 0) {
            sm.wst[wid] = static_cast<int>(hiw);
            sm.wst[kMaxWaves + wid] = static_cast<int>(low);
        }
        __syncthreads();
        if (threadIdx.x == 0) {
            unsigned long long best = 0;
            for (int x = 0; x < BS / kWave; ++x) {
                const unsigned long long k = (static_cast<unsigned long long>(static_cast<unsigned>(sm.wst[x])) << 32) |
                                             static_cast<unsigned>(sm.wst[kMaxWaves + x]);
                best = k > best ? k : best;
            }
            *reinterpret_cast<unsigned long long *>(sm.misc + M_KEY) = round_key(best);
        }
    };
    if (slot >= 0)
        for (int x = threadIdx.x; x < hh; x += BS)
            tr.scores[static_cast<size_t>(slot) * t.N + ubase + x] =
                topsis_close(nc, [&](int c) { return xs[c * hh + x]; }, q, ap, am);
    wg_best();
    // ---- E: selection rounds (global argmax, commit by workgroup 0, retries)
    for (;;) {
        const unsigned r = rnd++;
        if (threadIdx.x == 0)
            __hip_atomic_store(g.kslot + (r & 1) * G + w,
                               round_tag(r) | *reinterpret_cast<const unsigned long long *>(sm.misc + M_KEY),
                               __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        if (threadIdx.x < kWave) {
            bool bad = false;
            const unsigned long long kb = round_max(g, r, timeout, bad);
            if (lane == 0) {
                *reinterpret_cast<unsigned long long *>(sm.wst + 2 * kMaxWaves) = kb;
                sm.misc[M_OK] = bad;
            }
        }
        __syncthreads();
        if (sm.misc[M_OK]) return false;
        const unsigned long long kb = *reinterpret_cast<const unsigned long long *>(sm.wst + 2 * kMaxWaves);
        if (kb == 0) {                                                        // no server left
            if (w == 0) rollback_request<BS>(t, st, b, s.r, s.i);
            grid_sync(g, sm.misc + M_OK, timeout);
            return false;
        }
        const int u = static_cast<int>(0x1ffffu - static_cast<unsigned>(kb & 0x1ffffu));
        if (w == 0) {
            // workgroup 0 commits: 1 placed, 0 retry with the next server,
            // 2 request rejected when its links were routed at its end
            if (threadIdx.x < kWave) {
                // commit_wave reads the peer servers from LDS; its routing
                // uses the global state
                Smem cs;
                cs.pk = sm.pk;
                const bool ok = commit_wave(t, st, b, u, s, m.route_end ? 0 : P, cs, b.pbmax + s.p0, lane);
                if (lane == 0) {
                    sm.misc[M_ROUTE + 1] = ok;
                    if (ok) {
                        b.host[s.g] = u;
                        b.score[s.g] = __uint_as_float(static_cast<unsigned>(kb >> 17) - 1u);
                        if (s.i == s.n - 1) b.tse[s.r] = dev_clock();
                    }
                }
            }
            __syncthreads();
            int res = sm.misc[M_ROUTE + 1];
            if (res && m.route_end && s.i == s.n - 1)
                res = route_request_end<BS>(t, st, b, sm.misc + M_ROUTE, s,
                                            [&](int q) { return q == s.i ? u : rv.hosts[q]; }) ? 1 : 2;
            __syncthreads();
            if (threadIdx.x == 0) {
                __hip_atomic_store(g.rflag, round_tag(r) | static_cast<unsigned>(res), __ATOMIC_RELEASE,
                                   __HIP_MEMORY_SCOPE_AGENT);
                sm.misc[M_RES] = res;
            }
        } else if (threadIdx.x == 0) {
            sm.misc[M_RES] = round_outcome(g, r, timeout);
        }
        __syncthreads();
        const int ok = sm.misc[M_RES];
        if (ok < 0 || ok == 2) return false;
        if (ok) {
            if (rv.hosts_out && threadIdx.x == 0) rv.hosts_out[s.i] = u;
            __syncthreads();
            return true;
        }
        if (u / hh == w) {                                                    // owner masks it and rescans
            if (threadIdx.x == 0) xs[nc * hh + (u - ubase)] = 0;
            __syncthreads();
            wg_best();
        }
        __syncthreads();
    }
}

}  // namespace dcs

namespace dcs {

// LDS of the request prefetch after the cooperative step's region.
__device__ __forceinline__ int *grid_req_lds(char *dsm, int h, int hh, int nc) {
    return reinterpret_cast<int *>(dsm + align4(gsmem_bytes(h, hh, nc) / sizeof(int)) * sizeof(int));
}

// Plain form, large data centers: one cooperative launch per container step.
// K > 0: k = K fat-trees on the four default criteria, as compile-time
// constants (as in the batched kernel); K = 0: any.
template <int BS, int K>
__global__ __launch_bounds__(BS) void k_topsis_grid(Params p, GridCtl g, long long timeout) {
    extern __shared__ __align__(16) char dsm[];
    // every workgroup leaves before any wait: the request was rejected at an
    // earlier step, or a wait of an earlier launch timed out (the launches of
    // a batch's steps are queued together, and a step after a failed one
    // would read the missing peer's server as -1)
    if (p.b.status[p.s.r] == 0 || __hip_atomic_load(g.err, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)) return;
    constexpr int CS = K ? 4 : 0;
    const Topo t = topo_of<K>(p.t);
    const GSmem sm = gcarve(dsm, t.h, t.hh, crit_count<CS>(p.m));
    unsigned rnd = __hip_atomic_load(g.round, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    grid_topsis_step<BS, CS>(t, p.st, p.m, p.b, sm, g, timeout, p.s, plain_view(p), p.tr, rnd);
    if (blockIdx.x == 0 && threadIdx.x == 0) __hip_atomic_store(g.round, rnd, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Serving form, large data centers: the persistent loop of k_serve run by
// one cooperative workgroup per pod.  Workgroup 0 polls the command ring
// and publishes each command to the others through a grid barrier; every
// workgroup keeps its own LDS copy of the request.
template <int BS, int K>
__global__ __launch_bounds__(BS) void k_serve_grid(Params p, ServeArgs a, GridCtl g, long long timeout) {
    extern __shared__ __align__(16) char dsm[];
    constexpr int CS = K ? 4 : 0;
    const Topo t = topo_of<K>(p.t);
    const GSmem sm = gcarve(dsm, t.h, t.hh, crit_count<CS>(p.m));
    int *rq_host = grid_req_lds(dsm, t.h, t.hh, crit_count<CS>(p.m));
    int *rq_cpu = rq_host + kMaxN, *rq_ram = rq_cpu + kMaxN, *rq_poff = rq_ram + kMaxN;
    int *rq_pj = rq_poff + kMaxN + 4, *rq_pbw = rq_pj + kMaxPairs, *rq_pbmax = rq_pbw + kMaxPairs;
    int *rq_cmax = rq_pbmax + kMaxPairs, *rq_rmax = rq_cmax + kMaxN;
    const bool lead = blockIdx.x == 0;
    int pos = a.start;
    unsigned rnd = __hip_atomic_load(g.round, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);   // selection rounds
    long long idle0 = dev_clock();
    for (;;) {
        if (lead && threadIdx.x == 0) {
            Cmd *c = a.cmds + (pos % a.cap);
            int got = 0;
            for (;;) {        // bounded wait: the workgroups leave after idle_ticks without work
                if (__hip_atomic_load(&c->seq, __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_SYSTEM) == pos + 1) {
                    got = 1;
                    break;
                }
                if (dev_clock() - idle0 > a.idle_ticks) break;
                __builtin_amdgcn_s_sleep(8);
            }
            int *cf = cmd_flags(g, pos);
            int type = CMD_STOP;
            if (got) {
                type = __hip_atomic_load(&c->type, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
                cf[GF_N] = __hip_atomic_load(&c->n, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
                cf[GF_NPAIR] = __hip_atomic_load(&c->npair, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
                cf[GF_SLOT] = __hip_atomic_load(&c->slot_off, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
                cf[GF_RID] = __hip_atomic_load(&c->rid, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
            }
            cf[GF_GOT] = got;
            cf[GF_TYPE] = type;
        }
        if (!grid_sync(g, sm.misc + M_OK, a.idle_ticks + timeout)) break;      // command barrier
        const int *cf = cmd_flags(g, pos);
        const int got = cf[GF_GOT], type = cf[GF_TYPE], n = cf[GF_N], P = cf[GF_NPAIR], rid = cf[GF_RID];
        int *sb = a.arena + cf[GF_SLOT];
        if (type == CMD_STOP) {
            if (got) ++pos;
            break;
        }
        const SlotLayout L = slot_layout(n, P);
        const Batch b = slot_batch(sb, L);
        const long long t_admit = dev_clock();
        bool fault = false;
        if (type == CMD_SUBMIT) {
            const int *stg = a.staging + (size_t)(pos % a.cap) * a.stage_ints;
            if (lead)
                for (int x = threadIdx.x; x < L.in_end; x += BS) sb[x] = stg[x];
            for (int x = threadIdx.x; x <= n; x += BS) {
                rq_poff[x] = stg[L.poff + x];
                if (x < n) {
                    rq_cpu[x] = stg[L.cpu + x];
                    rq_ram[x] = stg[L.ram + x];
                    rq_cmax[x] = stg[L.cmax + x];
                    rq_rmax[x] = stg[L.rmax + x];
                    rq_host[x] = -1;
                    if (lead) {
                        sb[L.host + x] = -1;
                        sb[L.score + x] = 0;
                    }
                }
            }
            for (int x = threadIdx.x; x < P; x += BS) {
                rq_pj[x] = stg[L.pj + x];
                rq_pbw[x] = stg[L.pbw + x];
                rq_pbmax[x] = stg[L.pbmax + x];
                if (lead) sb[L.code + x] = -1;
            }
            if (lead && threadIdx.x == 0) {
                sb[L.failat] = -1;
                sb[L.status] = 1;
            }
            __syncthreads();
            for (int i = 0; i < n; ++i) {
                const int q0 = rq_poff[i];
                const StepIn s{0, i, n, 0, i, q0, rq_poff[i + 1] - q0, rq_cpu[i], rq_ram[i], rq_cmax[i], rq_rmax[i]};
                const ReqView rv{rq_pj + q0, rq_pbw + q0, rq_host, rq_host, rq_pbmax + q0, rq_poff, rq_pj};
                if (!grid_topsis_step<BS, CS>(t, p.st, p.m, b, sm, g, timeout, s, rv, p.tr, rnd)) {
                    fault = __hip_atomic_load(g.err, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != 0;
                    break;
                }
            }
        } else if (lead) {
            give_back<BS>(t, p.st, b, 0, n);         // departure of an accepted request
        }
        if (fault) break;
        if (lead) {
            __syncthreads();
            Comp *cp = a.comps + (pos % a.cap);
            if (type == CMD_SUBMIT)
                for (int x = threadIdx.x; x < n; x += BS) {
                    cp->host[x] = b.host[x];
                    cp->score[x] = b.score[x];
                }
            if (threadIdx.x == 0) {
                cp->type = type;
                cp->rid = rid;
                cp->n = n;
                cp->status = type == CMD_SUBMIT ? b.status[0] : 1;
                cp->failat = type == CMD_SUBMIT ? b.failat[0] : -1;
                cp->t_admit = t_admit;
                cp->t_decide = dev_clock();
            }
            __threadfence_system();
            __syncthreads();
            if (threadIdx.x == 0) {
                __hip_atomic_store(&cp->seq, pos + 1, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_SYSTEM);
                __hip_atomic_store(a.ctrl, pos + 1, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_SYSTEM);
            }
        }
        ++pos;
        idle0 = dev_clock();
    }
    if (lead && threadIdx.x == 0) {
        __hip_atomic_store(g.round, rnd, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        __hip_atomic_store(a.ctrl, pos, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_SYSTEM);
        __hip_atomic_store(a.ctrl + 1, 1, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_SYSTEM);
    }
}

}  // namespace dcs
