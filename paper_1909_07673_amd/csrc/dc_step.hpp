// Device side of one container step: path stage, criteria, TOPSIS scoring,
// argmax selection, commit with widest shortest-path routing, and request
// rollback.  Everything here runs inside one workgroup; the plain, batched
// and serving kernels differ only in where the data-center state and the
// request data live (HBM/L2 or LDS) and in how steps are fed.
//
// Paper references (arXiv 1909.07673):
//   section II-A / Table I  data-center graph, capacities, requests
//   section IV-B            k-ary fat-tree (DC configuration)
//   section V               criteria c^s_u, bw^s_u, f_u
//   section V-C             TOPSIS
//   section V-D             widest shortest path, one residual per undirected link
//   Eqs. (4)-(5)            capacity and bandwidth constraints
//   section II-A            demand intervals [min, max]
//   section II-B, Eqs. (1)-(2)  their utilities
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace dcs {

constexpr int kMaxCrit = 8;
constexpr int kMaxN = 64;          // containers per request
constexpr int kMaxPairs = kMaxN * (kMaxN - 1) / 2;
constexpr int kMaxPods = 64;
constexpr int kWave = 64;
constexpr int kBig = 0x7fffffff;

enum { CRIT_CPU = 0, CRIT_RAM = 1, CRIT_ACTIVE = 2, CRIT_PATHBW = 3, CRIT_UPLINK = 4, CRIT_HOPS = 5 };

// Fat-tree sizes.  h = k/2 hosts per edge switch and aggregation switches per
// pod; hh = h*h hosts per pod; nsw = k*k/2 edge (and aggregation) switches;
// rh, rhh, rnsw their reciprocals in FP32 for exact small-integer division.
struct Topo {
    int k, h, hh, N, nsw;
    float rh, rhh, rnsw;
};

// floor(x / d) for 0 <= x < 2^18 and 1 <= d <= 2048, via the FP32
// reciprocal r = fl(1/d): (x + 1/2) / d lies at least 1/(2d) from an
// integer, far more than the two roundings can move it.
__device__ __forceinline__ int fdiv(int x, float r) { return static_cast<int>((static_cast<float>(x) + 0.5f) * r); }

// floor(x / d) for 0 <= x < 2^18: an integer division where d is known at
// compile time (a shift for a power of two), the reciprocal form otherwise.
__device__ __forceinline__ int div_floor(int x, int d, float r) {
    if (__builtin_constant_p(d)) return static_cast<int>(static_cast<unsigned>(x) / static_cast<unsigned>(d));
    return fdiv(x, r);
}

// The topology of a k = K fat-tree as compile-time constants (K = 0: the
// run-time values in t).
template <int K>
__device__ __forceinline__ Topo topo_of(const Topo &t) {
    if (K == 0) return t;
    constexpr int h = K / 2, hh = h * h;
    return Topo{K, h, hh, K * hh, K * h, 1.0f / h, 1.0f / hh, 1.0f / (K * h)};
}

// Edge switch and pod of server u.
__device__ __forceinline__ int edge_of(const Topo &t, int u) { return div_floor(u, t.h, t.rh); }
__device__ __forceinline__ int pod_of(const Topo &t, int u) { return div_floor(u, t.hh, t.rhh); }

// Residual state of one data center, structure-of-arrays, N entries each.
struct State {
    int *cpu, *ram, *npl, *up, *ea, *ac;
};

struct Method {
    int method, scale, nc;
    int route_end;      // 1: links routed after a request's last unit is placed (section V-D)
    int crit[kMaxCrit];
    int cost[kMaxCrit];
    float w[kMaxCrit];
};

// Criteria of a step: CS = 0 takes them from the method; CS = 4 is the
// default list (CPU, RAM, active, path bandwidth; all benefits) and CS = 5
// the five of the large AHP case (CPU, RAM, uplink, path bandwidth and hops,
// the last a cost), fixed at compile time.
template <int CS> __device__ __forceinline__ int crit_count(const Method &m) { return CS ? CS : m.nc; }
template <int CS> __device__ __forceinline__ int crit_at(const Method &m, int c) {
    if (CS == 4) return c;
    if (CS == 5) return c < 2 ? c : c == 2 ? CRIT_UPLINK : c == 3 ? CRIT_PATHBW : CRIT_HOPS;
    return m.crit[c];
}
template <int CS> __device__ __forceinline__ int crit_cost(const Method &m, int c) {
    if (CS == 4) return 0;
    if (CS == 5) return c == 4;
    return m.cost[c];
}

// A pointer to an array in global memory.  Indexing goes through an
// address-space-1 pointer, so the access stays a global load or store even
// where the pointer itself was read back from LDS (a plain pointer would
// become a flat access there, and every later wait for an LDS result would
// also wait for the flat access's round trip to memory).
#define DCS_GLOBAL __attribute__((address_space(1)))
template <class T>
struct GPtr {
    T *p;
    __host__ __device__ GPtr &operator=(T *q) { p = q; return *this; }
    __host__ __device__ __forceinline__ operator T *() const { return p; }
    __device__ __forceinline__ DCS_GLOBAL T &operator[](long long i) const { return ((DCS_GLOBAL T *)p)[i]; }
};

// Requests of one schedule call, CSR layout.  Container g of request r is
// coff[r] + i; its placed peers are pj[poff[g]..poff[g+1]) (container index
// within the request, ascending) with demands pbw[].  Demands are intervals
// (section II-A): cpu, ram, pbw are the minima, cmax, rmax, pbmax the
// maxima (equal for fixed demands); cpua, rama, pbwa receive what each
// container and pair was given, which is what a release gives back.
struct Batch {
    GPtr<const int> coff, cpu, ram, poff, pj, pbw;
    GPtr<const int> cmax, rmax, pbmax;
    GPtr<int> cpua, rama;  // [Ct] allocated CPU and RAM
    GPtr<int> pbwa;        // [Pt] allocated bandwidth
    GPtr<int> host;        // [Ct] chosen server, -1 until placed
    GPtr<float> score;     // [Ct] score of the chosen server
    GPtr<int> code;        // [Pt] path choice per peer pair, -1 when co-located
    GPtr<int> status;      // [R]  1 accepted (optimistic), 0 rejected
    GPtr<int> failat;      // [R]  container without a server, -1
    GPtr<const int> iroff; // [I+1] first request of each instance (batched form)
    GPtr<const int> rid;   // [R]  request id (low 31 bits), for trace records
    GPtr<long long> tsb, tse;  // [R] device clock (100 MHz) at the first step's start / the decision
};

// One container step: where it sits in the batch, and its demand.
struct StepIn {
    int r, i, n;       // request (batch index), container index, containers of the request
    int g0, g;         // global index of the request's container 0 and of this container
    int p0, P;         // first peer pair of this container and number of placed peers
    int cpu, ram;      // demand (minimum)
    int cmax, rmax;    // demand maximum
};

// Where a step reads its request data: the container's peer list (P
// entries) and the servers of the request's containers (indexed by
// container).  Global memory in the plain form, LDS in the batched form.
struct ReqView {
    const int *pj, *pbw, *hosts;
    int *hosts_out;    // LDS copy of hosts to update (batched form), or nullptr
    const int *pbmax;  // the peers' maximum demands
    // the whole request in LDS (forms that stage it there), else nullptr:
    // rpoff[x] the first pair of container x relative to the request's
    // first pair (x <= n), rpj the pairs' peer containers
    const int *rpoff = nullptr, *rpj = nullptr;
};

// Waits for this wave's outstanding global loads and stores (s_waitcnt
// vmcnt(0) on gfx9).  Placed at the end of rarely taken paths that load from
// global memory, so that where they join the common path the compiler's
// per-register wait analysis finds no load outstanding; otherwise it
// places waits there, which on this architecture also wait for every
// store issued since (the results a step writes).
__device__ __forceinline__ void vm_drain() { __builtin_amdgcn_s_waitcnt(0x0F70); }

// A value that is the same on every lane, as a scalar.
__device__ __forceinline__ int uniform(int v) { return __builtin_amdgcn_readfirstlane(v); }

// Constant-rate device clock (100 MHz), read without a memory access.
__device__ __forceinline__ long long dev_clock() { return static_cast<long long>(wall_clock64()); }

struct Trace {
    int *meta;        // [cap][4]
    float *scores;    // [cap][N]
    int *counter;     // per instance step counter
    int stride, cap;
};

// Slots of the LDS misc block.
enum {
    M_OK = 0, M_TRACE = 1,
    M_DH0 = 2, M_DH1 = 3, M_DE0 = 4, M_DE1 = 5, M_DP0 = 6, M_DP1 = 7,   // deficits (min, max id)
    M_ALIVE = 8, M_ROUTE = 9,
    M_KEY = 12,                  // cooperative step: the workgroup's packed best key (two slots, 8-byte aligned)
    M_RES = 14,                  // cooperative step: outcome of the selection round
    M_MISC = 16
};

constexpr int kMaxWaves = 16;          // 1024-thread workgroups
// Servers a thread works on together: enough independent chains to hide
// LDS latency, few enough to stay in registers at 1024 threads.
__host__ __device__ constexpr int host_group(int bs) { return bs >= 1024 ? 2 : 4; }
constexpr int kStatFields = 5 * kMaxCrit;  // per criterion: 3 sum-of-squares chunks, max, -min

// LDS scratch of a step, carved from dynamic shared memory.  Every region
// starts on a 16-byte boundary.
struct Smem {
    int4 *pk;                         // [kMaxN] packed peer: server, edge | pod << 16, demand, uplink residual
    int *wst;                         // [kStatFields][kMaxWaves] per-wave column statistics
    unsigned *ahi, *alo;              // [2][kMaxWaves] per-wave argmax keys (alternating per retry)
    int *ph, *pbw;                    // [kMaxN] peer server, maximum demand
    int *capP;                        // [kMaxPods] summed aggregation-core residual per pod
    int *misc;                        // [M_MISC]
    int *capE;                        // [nsw] summed edge-aggregation residual per edge switch
    int *tabT, *tabE;                 // [pc][nsw] per-peer aggregation / edge tables
};

__host__ __device__ inline size_t align4(size_t ints) { return (ints + 3) & ~size_t(3); }

__host__ __device__ inline size_t smem_fixed_bytes() {
    return sizeof(int4) * kMaxN + sizeof(int) * (kStatFields * kMaxWaves + 4 * kMaxWaves + 2 * kMaxN + kMaxPods +
                                                 M_MISC);
}

// Variable part: capE, then the per-peer tables (rounded to 16 bytes).
__host__ __device__ inline size_t smem_var_ints(int pc, int nsw) {
    return align4((size_t)nsw) + 2 * align4((size_t)pc * nsw);
}

__device__ inline Smem carve(char *base, int pc, int nsw) {
    Smem s;
    s.pk = reinterpret_cast<int4 *>(base);
    int *p = reinterpret_cast<int *>(base + sizeof(int4) * kMaxN);
    s.wst = p; p += kStatFields * kMaxWaves;
    s.ahi = reinterpret_cast<unsigned *>(p); p += 2 * kMaxWaves;
    s.alo = reinterpret_cast<unsigned *>(p); p += 2 * kMaxWaves;
    s.ph = p; p += kMaxN;
    s.pbw = p; p += kMaxN;
    s.capP = p; p += kMaxPods;
    s.misc = p; p += M_MISC;
    s.capE = p; p += align4(nsw);
    s.tabT = p; p += align4((size_t)pc * nsw);
    s.tabE = p;
    return s;
}

// ---------------------------------------------------------------- wave reductions (DPP)
// Reductions across a 64-lane wave with DPP row shifts and row broadcasts;
// the result is returned uniformly (read from lane 63).
template <int CTRL, int ROWS>
__device__ __forceinline__ int dpp(int identity, int v) {
    return __builtin_amdgcn_update_dpp(identity, v, CTRL, ROWS, 0xf, false);
}

#define DCS_WAVE_REDUCE(v, OP, ID)                        \
    do {                                                  \
        v = OP(v, dpp<0x111, 0xf>(ID, v));                \
        v = OP(v, dpp<0x112, 0xf>(ID, v));                \
        v = OP(v, dpp<0x114, 0xf>(ID, v));                \
        v = OP(v, dpp<0x118, 0xf>(ID, v));                \
        v = OP(v, dpp<0x142, 0xa>(ID, v));                \
        v = OP(v, dpp<0x143, 0xc>(ID, v));                \
        v = __builtin_amdgcn_readlane(v, 63);             \
    } while (0)

__device__ __forceinline__ int op_add(int a, int b) { return a + b; }
__device__ __forceinline__ int op_max(int a, int b) { return a > b ? a : b; }
__device__ __forceinline__ int op_min(int a, int b) { return a < b ? a : b; }
__device__ __forceinline__ int op_umax(int a, int b) { return (unsigned)a > (unsigned)b ? a : b; }

// Reduction within each row of 16 lanes; lane 16*row + 15 holds the result.
#define DCS_ROW_REDUCE(v, OP, ID)                         \
    do {                                                  \
        v = OP(v, dpp<0x111, 0xf>(ID, v));                \
        v = OP(v, dpp<0x112, 0xf>(ID, v));                \
        v = OP(v, dpp<0x114, 0xf>(ID, v));                \
        v = OP(v, dpp<0x118, 0xf>(ID, v));                \
    } while (0)

__device__ __forceinline__ int wave_sum(int v) { DCS_WAVE_REDUCE(v, op_add, 0); return v; }
__device__ __forceinline__ int wave_max(int v) { DCS_WAVE_REDUCE(v, op_max, -kBig - 1); return v; }
__device__ __forceinline__ int wave_min(int v) { DCS_WAVE_REDUCE(v, op_min, kBig); return v; }
__device__ __forceinline__ unsigned wave_umax(unsigned v) {
    int x = static_cast<int>(v);
    DCS_WAVE_REDUCE(x, op_umax, 0);
    return static_cast<unsigned>(x);
}

// ---------------------------------------------------------------- topology helpers
// Applies delta to every link of the path between servers u != v chosen by
// candidate c: uplinks of u and v; with different edge switches the two
// edge-aggregation links through aggregation index a; with different pods
// the two aggregation-core links through core (a, j).  c = a (same pod) or
// a*h + j (different pods).
// Link x (0..5) of that path, or nullptr when the path is shorter.
__device__ __forceinline__ int *path_link(const Topo &t, const State &st, int u, int v, int c, int x) {
    const int eu = edge_of(t, u), ev = edge_of(t, v), pu = pod_of(t, u), pv = pod_of(t, v);
    int a = 0, j = 0;
    if (pu == pv) a = c; else { a = div_floor(c, t.h, t.rh); j = c - a * t.h; }
    switch (x) {
    case 0: return st.up + u;
    case 1: return st.up + v;
    case 2: return eu != ev ? st.ea + eu * t.h + a : nullptr;
    case 3: return eu != ev ? st.ea + ev * t.h + a : nullptr;
    case 4: return pu != pv ? st.ac + (pu * t.h + a) * t.h + j : nullptr;
    default: return pu != pv ? st.ac + (pv * t.h + a) * t.h + j : nullptr;
    }
}

// The same for a lane-dependent x (u, v and c the same on every lane): the
// link is chosen by selects rather than branches, so a wave whose lanes
// take different links runs no divergent code.
__device__ __forceinline__ int *path_link_lane(const Topo &t, const State &st, int u, int v, int c, int x) {
    const int eu = edge_of(t, u), ev = edge_of(t, v), pu = pod_of(t, u), pv = pod_of(t, v);
    const int a = pu == pv ? c : div_floor(c, t.h, t.rh);
    const int j = c - a * t.h;
    const bool vs = x & 1;
    const int kind = x >> 1;
    int *l0 = st.up + (vs ? v : u);
    int *l1 = st.ea + (vs ? ev : eu) * t.h + a;
    int *l2 = st.ac + ((vs ? pv : pu) * t.h + a) * t.h + j;
    int *l = kind == 0 ? l0 : (kind == 1 ? l1 : l2);
    const bool has = x < 6 && (kind == 0 || (kind == 1 ? eu != ev : pu != pv));
    return has ? l : nullptr;
}

template <bool ATOMIC>
__device__ __forceinline__ void path_apply(const Topo &t, const State &st, int u, int v, int c, int delta) {
    for (int x = 0; x < 6; ++x) {
        int *l = path_link(t, st, u, v, c, x);
        if (!l) continue;
        if (ATOMIC) atomicAdd(l, delta);
        else *l += delta;
    }
}

// Widest minimum-hop path from u to v under the current residuals; ties go
// to the lowest aggregation then core index (candidate order).  Evaluated by
// one wave, candidates spread over lanes.  Returns the 32-bit key
// bottleneck << 10 | (1023 - candidate): residuals stay below 2^22 and
// there are at most 1024 candidates.
// Candidate paths a lane takes between two pods: hh / 64 rounded up, at
// most 1024 / 64 (k <= 64).
constexpr int kMaxCandIters = 16;

// The widest path's key and the residuals of its links (in the roles of
// path_link: uplinks of u and v, edge-aggregation links on u's and v's side,
// aggregation-core links on u's and v's side; 0 where the path has none).
struct Widest {
    unsigned key;
    int link[6];
};

__device__ __forceinline__ Widest widest_wave_links(const Topo &t, const State &st, int u, int v, int eu, int pu,
                                                    int ev, int pv, int lane) {
    // every load of a candidate is made before any is used, so a peer costs
    // one round of memory latency (the loop trips are compile-time constants
    // where the topology is); each lane keeps the residuals of its best
    // candidate, and the lane holding the overall best hands them out
    const int upu = st.up[u], upv = st.up[v];
    unsigned best = 0;
    int b2 = 0, b3 = 0, b4 = 0, b5 = 0;
    if (eu == ev) {                                   // same edge switch: the two uplinks
        best = lane == 0 ? (static_cast<unsigned>(min(upu, upv)) << 10) | 1023u : 0u;
    } else if (pu == pv) {                            // same pod: candidates are aggregation switches
        const int iters = (t.h + kWave - 1) / kWave;
#pragma unroll
        for (int i = 0; i < iters; ++i) {
            const int c = lane + i * kWave;
            if (c >= t.h) break;
            const int x2 = st.ea[eu * t.h + c], x3 = st.ea[ev * t.h + c];
            const int b = min(min(upu, upv), min(x2, x3));
            const unsigned key = (static_cast<unsigned>(b) << 10) | static_cast<unsigned>(1023 - c);
            if (key > best) { best = key; b2 = x2; b3 = x3; }
        }
    } else if (!__builtin_constant_p(t.hh)) {         // candidates c = a * h + j: aggregation a, core (a, j)
        for (int c = lane; c < t.hh; c += kWave) {
            const int a = div_floor(c, t.h, t.rh);
            const int x2 = st.ea[eu * t.h + a], x3 = st.ea[ev * t.h + a];
            const int x4 = st.ac[pu * t.hh + c], x5 = st.ac[pv * t.hh + c];
            const int b = min(min(min(upu, upv), min(x2, x3)), min(x4, x5));
            const unsigned key = (static_cast<unsigned>(b) << 10) | static_cast<unsigned>(1023 - c);
            if (key > best) { best = key; b2 = x2; b3 = x3; b4 = x4; b5 = x5; }
        }
    } else {
        // the same where hh is a compile-time constant: a trip count the
        // compiler sees, so the loads of all of a lane's candidates are made
        // up front, in registers
        const int iters = (t.hh + kWave - 1) / kWave;
        int x2[kMaxCandIters], x3[kMaxCandIters], x4[kMaxCandIters], x5[kMaxCandIters];
#pragma unroll
        for (int i = 0; i < kMaxCandIters; ++i) {
            if (i >= iters) break;
            const int c = min(lane + i * kWave, t.hh - 1);
            const int a = div_floor(c, t.h, t.rh);
            x2[i] = st.ea[eu * t.h + a];
            x3[i] = st.ea[ev * t.h + a];
            x4[i] = st.ac[pu * t.hh + c];
            x5[i] = st.ac[pv * t.hh + c];
        }
        const int base = min(upu, upv);
#pragma unroll
        for (int i = 0; i < kMaxCandIters; ++i) {
            if (i >= iters) break;
            const int c = lane + i * kWave;
            if (c >= t.hh) break;
            const int b = min(min(base, min(x2[i], x3[i])), min(x4[i], x5[i]));
            const unsigned key = (static_cast<unsigned>(b) << 10) | static_cast<unsigned>(1023 - c);
            if (key > best) { best = key; b2 = x2[i]; b3 = x3[i]; b4 = x4[i]; b5 = x5[i]; }
        }
    }
    Widest w;
    w.key = wave_umax(best);
    const unsigned long long mask = __ballot(best == w.key);
    const int src = mask ? __builtin_ctzll(mask) : 0;
    w.link[0] = upu;
    w.link[1] = upv;
    w.link[2] = __builtin_amdgcn_readlane(b2, src);
    w.link[3] = __builtin_amdgcn_readlane(b3, src);
    w.link[4] = __builtin_amdgcn_readlane(b4, src);
    w.link[5] = __builtin_amdgcn_readlane(b5, src);
    return w;
}

__device__ __forceinline__ unsigned widest_wave(const Topo &t, const State &st, int u, int v, int eu, int pu,
                                                int ev, int pv, int lane) {
    return widest_wave_links(t, st, u, v, eu, pu, ev, pv, lane).key;
}

// Lanes 0..5 each update one link of the path (its links are distinct).
template <bool ATOMIC>
__device__ __forceinline__ void path_apply_lanes(const Topo &t, const State &st, int u, int v, int c, int delta,
                                                 int lane) {
    int *l = path_link_lane(t, st, u, v, c, lane);
    if (l) {
        if (ATOMIC) atomicAdd(l, delta);
        else *l += delta;
    }
}

// Commit of container s on server u with its P placed peers (servers and
// minimum demands in the LDS peer list, ascending container index): route
// each remote peer's minimum on its widest shortest path under the current
// residuals, failing when a bottleneck is below it (Eqs. (4)-(5)); on
// failure every change is undone.  A container runs with anything in its
// demand interval and its utility (Eqs. (1)-(2)) grows with what it gets,
// so once the minima fit, each routed path in peer order is topped up by
// what its most loaded link still has, to at most the pair's maximum, and
// CPU and RAM take min(max, residual) of the server; a peer on the same
// server needs no link and gets its maximum.  Run by one whole wave; lane 0
// writes the server's resources, lane p peer p's route code and
// allocation.  pbmax[p]: peer p's maximum demand (LDS or global).
__device__ __forceinline__ bool commit_wave(const Topo &t, const State &st, const Batch &b, int u, const StepIn &s,
                                            int P, const Smem &sm, const int *pbmax, int lane) {
    const int pmax = lane < P ? pbmax[lane] : 0;
    // the result arrays' addresses, read now: the Batch may sit in LDS, and
    // read after the fences below they would add an LDS round trip to the
    // end of the chain
    const GPtr<int> o_code = b.code, o_pbwa = b.pbwa, o_cpua = b.cpua, o_rama = b.rama;
    // the server's resources, read once: only this wave writes them until
    // the commit ends
    const int cpu_u = st.cpu[u], ram_u = st.ram[u], npl_u = st.npl[u];
    if (cpu_u < s.cpu || ram_u < s.ram) return false;
    const int eu = edge_of(t, u), pu = pod_of(t, u);
    int routed = 0, mycode = -1, mine = pmax;   // lane p keeps peer p's path choice and allocation
    // lane p holds peer p's record (P <= 64), handed out per peer below
    const int4 mypk = lane < P ? sm.pk[lane] : make_int4(u, 0, 0, 0);
    bool ok = true;
    for (int p = 0; p < P; ++p) {
        const int4 pk = make_int4(__builtin_amdgcn_readlane(mypk.x, p), __builtin_amdgcn_readlane(mypk.y, p),
                                  __builtin_amdgcn_readlane(mypk.z, p), 0);
        const int v = pk.x;
        if (v == u) {
            routed = p + 1;
            continue;
        }
        const Widest wd = widest_wave_links(t, st, u, v, eu, pu, pk.y & 0xffff, pk.y >> 16, lane);
        const int bn = static_cast<int>(wd.key >> 10);
        const int c = 1023 - static_cast<int>(wd.key & 1023u);
        if (bn < pk.z) { ok = false; break; }
        // lane x writes link x of the path with its residual less the demand
        // (the residuals were just read; no other wave writes them meanwhile)
        {
            int *l = path_link_lane(t, st, u, v, c, lane);
            int cur = wd.link[0];
#pragma unroll
            for (int x = 1; x < 6; ++x) cur = lane == x ? wd.link[x] : cur;
            if (l) *l = cur - pk.z;
        }
        mycode = lane == p ? c : mycode;
        mine = lane == p ? pk.z : mine;
        __threadfence_block();
        routed = p + 1;
    }
    if (!ok) {
        for (int p = routed - 1; p >= 0; --p) {
            const int v = __builtin_amdgcn_readlane(mypk.x, p);
            if (v != u)
                path_apply_lanes<false>(t, st, u, v, __builtin_amdgcn_readlane(mycode, p),
                                        __builtin_amdgcn_readlane(mypk.z, p), lane);
            __threadfence_block();
        }
        return false;
    }
    // top-ups, only over the routed peers with room (none for fixed
    // demands); a lane always reads the links it alone writes (slot x of
    // every path from u is a link in the same role)
    for (unsigned long long todo = __ballot(mypk.x != u && pmax > mypk.z); todo; todo &= todo - 1) {
        const int p = __builtin_ctzll(todo);
        const int v = __builtin_amdgcn_readlane(mypk.x, p);
        const int room = __builtin_amdgcn_readlane(pmax, p) - __builtin_amdgcn_readlane(mypk.z, p);
        const int c = __builtin_amdgcn_readlane(mycode, p);
        const int *l = path_link_lane(t, st, u, v, c, lane);
        const int add = min(room, wave_min(l ? *l : kBig));
        if (add <= 0) continue;
        path_apply_lanes<false>(t, st, u, v, c, -add, lane);
        mine = lane == p ? mine + add : mine;
        __threadfence_block();
    }
    if (lane < P) {
        o_code[s.p0 + lane] = mycode;
        o_pbwa[s.p0 + lane] = mine;
    }
    if (lane == 0) {
        const int ca = max(s.cpu, min(s.cmax, cpu_u)), ra = max(s.ram, min(s.rmax, ram_u));
        st.cpu[u] = cpu_u - ca;
        st.ram[u] = ram_u - ra;
        st.npl[u] = npl_u + 1;
        o_cpua[s.g] = ca;
        o_rama[s.g] = ra;
    }
    __threadfence_block();
    return true;
}

// Gives back containers [0, upto) of request r: the CPU and RAM they were
// given, the placed count and the allocation of every routed peer pair.
// Block-wide, with atomics.
template <int BS>
__device__ __forceinline__ void give_back(const Topo &t, const State &st, const Batch &b, int r, int upto) {
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
        if (u != v && c >= 0) path_apply<true>(t, st, u, v, c, b.pbwa[q]);
    }
    for (int i = threadIdx.x; i < upto; i += BS) {
        const int u = b.host[g0 + i];
        atomicAdd(st.cpu + u, b.cpua[g0 + i]);
        atomicAdd(st.ram + u, b.rama[g0 + i]);
        atomicSub(st.npl + u, 1);
    }
}

// Request r found no server for container `upto`: undo containers
// [0, upto) (all or nothing) and mark the request rejected.  host[] keeps
// the servers the undone containers had been given (attempt record).
// The same from the LDS copy of the request (ReqView::rpoff, rpj, hosts):
// the pair owners are found in LDS, not by a search through global memory.
// g0 and pb: the request's first container and first pair in the batch.
template <int BS>
__device__ __forceinline__ void give_back_lds(const Topo &t, const State &st, const Batch &b, int g0, int pb,
                                              int upto, const ReqView &rv) {
    const int q_end = rv.rpoff[upto];
    for (int q = threadIdx.x; q < q_end; q += BS) {
        int lo = 0, hi = upto - 1;                       // container owning pair q
        while (lo < hi) {
            const int mid = (lo + hi + 1) >> 1;
            if (rv.rpoff[mid] <= q) lo = mid; else hi = mid - 1;
        }
        const int u = rv.hosts[lo], v = rv.hosts[rv.rpj[q]];
        const int c = b.code[pb + q];
        if (u != v && c >= 0) path_apply<true>(t, st, u, v, c, b.pbwa[pb + q]);
    }
    for (int i = threadIdx.x; i < upto; i += BS) {
        const int u = rv.hosts[i];
        atomicAdd(st.cpu + u, b.cpua[g0 + i]);
        atomicAdd(st.ram + u, b.rama[g0 + i]);
        atomicSub(st.npl + u, 1);
    }
}

template <int BS>
__device__ __forceinline__ void rollback_request(const Topo &t, const State &st, const Batch &b, int r, int upto,
                                                 const ReqView *rv = nullptr, const StepIn *s = nullptr) {
    if (rv && rv->rpoff)
        give_back_lds<BS>(t, st, b, s->g0, s->p0 - rv->rpoff[s->i], upto, *rv);
    else
        give_back<BS>(t, st, b, r, upto);
    __syncthreads();
    if (threadIdx.x == 0) {
        b.status[r] = 0;
        b.failat[r] = upto;
        b.tse[r] = dev_clock();
    }
    __threadfence_block();
    vm_drain();
    __syncthreads();
}

// ---------------------------------------------------------------- peers and path tables
// Peer tables for the peers [pbeg, pbeg+pn) (section V-D routing on a
// fat-tree, per destination server v in pod pv and edge switch ev):
//   T[ag] = max_j min(ac(ag, j), ac((pv, a), j))  for aggregation (p, a), p != pv
//   E[eg] = max_a min(ea(eg, a), ea(ev, a), T[(p, a)] or +inf in pod pv)   eg != ev
// so that the widest shortest path from u to v has bottleneck
// min(up[u], up[v], E[edge(u)]) (or min(up[u], up[v]) on the same edge).
// peer_pod(pc): the pod of peer pbeg + pc.
template <int BS, class PeerPod>
__device__ __forceinline__ void table_T(const Topo &t, const State &st, const Smem &sm, int pbeg, int pn,
                                        PeerPod peer_pod) {
    const int tot = pn * t.nsw;
    for (int it = threadIdx.x; it < tot; it += BS) {
        const int pc = div_floor(it, t.nsw, t.rnsw), ag = it - pc * t.nsw;
        const int pv = peer_pod(pc), pa = edge_of(t, ag);
        int val = 0;
        if (pa != pv) {
            const int a = ag - pa * t.h;
            const int *x = st.ac + ag * t.h;
            const int *y = st.ac + (pv * t.h + a) * t.h;
            if ((t.h & 3) == 0) {
                for (int j = 0; j < t.h; j += 4) {
                    const int4 a4 = *reinterpret_cast<const int4 *>(x + j);
                    const int4 b4 = *reinterpret_cast<const int4 *>(y + j);
                    val = max(val, max(max(min(a4.x, b4.x), min(a4.y, b4.y)), max(min(a4.z, b4.z), min(a4.w, b4.w))));
                }
            } else {
                for (int j = 0; j < t.h; ++j) val = max(val, min(x[j], y[j]));
            }
        }
        sm.tabT[it] = val;
    }
}

template <int BS>
__device__ __forceinline__ void table_E(const Topo &t, const State &st, const Smem &sm, int pbeg, int pn) {
    const int tot = pn * t.nsw;
    for (int it = threadIdx.x; it < tot; it += BS) {
        const int pc = div_floor(it, t.nsw, t.rnsw), eg = it - pc * t.nsw;
        const int ed = sm.pk[pbeg + pc].y;
        const int ev = ed & 0xffff, pv = ed >> 16, pe = edge_of(t, eg);
        int val = 0;
        if (eg != ev) {
            const int *x = st.ea + eg * t.h;
            const int *y = st.ea + ev * t.h;
            const int *T = sm.tabT + pc * t.nsw + pe * t.h;
            const int lim = pe != pv ? 0 : kBig;      // same pod: no aggregation-core leg
            if ((t.h & 3) == 0) {
                for (int a = 0; a < t.h; a += 4) {
                    const int4 a4 = *reinterpret_cast<const int4 *>(x + a);
                    const int4 b4 = *reinterpret_cast<const int4 *>(y + a);
                    const int4 t4 = *reinterpret_cast<const int4 *>(T + a);
                    val = max(val, max(max(min(min(a4.x, b4.x), max(t4.x, lim)), min(min(a4.y, b4.y), max(t4.y, lim))),
                                       max(min(min(a4.z, b4.z), max(t4.z, lim)), min(min(a4.w, b4.w), max(t4.w, lim)))));
                }
            } else {
                for (int a = 0; a < t.h; ++a) val = max(val, min(min(x[a], y[a]), max(T[a], lim)));
            }
        }
        sm.tabE[it] = val;
    }
}

// Phase A of a step (no barrier needed before it): the peer list of the
// container into LDS (server, demand, uplink residual, edge switch, pod),
// the summed residuals per edge switch and per pod when LIMITS, and the
// reset of the reduction slots.  With T0, also the aggregation table T of
// the first pc_cap peers, each peer's pod taken from the request itself,
// so that T needs no barrier of its own.  Ends with a barrier.
template <int BS, bool LIMITS, bool T0 = false>
__device__ __forceinline__ void load_peers(const Topo &t, const State &st, const ReqView &rv, const Smem &sm,
                                           int P, int pc_cap = 0) {
    for (int p = threadIdx.x; p < P; p += BS) {
        const int v = rv.hosts[rv.pj[p]];
        const int bw = rv.pbw[p];
        sm.ph[p] = v;
        sm.pbw[p] = rv.pbmax[p];
        sm.pk[p] = make_int4(v, edge_of(t, v) | (pod_of(t, v) << 16), bw, st.up[v]);
    }
    if (threadIdx.x < 6) sm.misc[M_DH0 + threadIdx.x] = (threadIdx.x & 1) ? -1 : kBig;
    if (LIMITS && P > 0) {
        for (int x = threadIdx.x; x < t.nsw; x += BS) {
            int se = 0;
            for (int a = 0; a < t.h; ++a) se += st.ea[x * t.h + a];
            sm.capE[x] = se;
        }
        // per pod: one wave sums the pod's h*h aggregation-core residuals
        const int lane = threadIdx.x & (kWave - 1), wid = threadIdx.x / kWave;
        for (int pod = wid; pod < t.k; pod += BS / kWave) {
            int s = 0;
            for (int x = lane; x < t.hh; x += kWave) s += st.ac[pod * t.hh + x];
            s = wave_sum(s);
            if (lane == 0) sm.capP[pod] = s;
        }
    }
    if (T0 && P > 0)
        table_T<BS>(t, st, sm, 0, min(P, pc_cap), [&](int pc) { return pod_of(t, rv.hosts[rv.pj[pc]]); });
    __syncthreads();
}

// Peer-side deficits: a peer server (edge switch, pod) whose uplink
// (uplinks) cannot carry the summed demand of the peers it holds can only
// be reached by a server inside it, so at most one such server (switch,
// pod) leaves any server feasible.  misc[M_DH0..M_DP1] = (min, max) id of
// the deficient servers, edge switches, pods; (kBig, -1) when none.  No
// barrier: the results are read after the next one.  Run by the last
// threads of the block, which the path tables that follow leave idle.
template <int BS>
__device__ __forceinline__ void peer_deficits(const Smem &sm, int P) {
    for (int p = BS - 1 - static_cast<int>(threadIdx.x); p < P; p += BS) {
        const int4 me = sm.pk[p];
        const int v = me.x, e = me.y & 0xffff, d = me.y >> 16;
        int sh = 0, se = 0, sp = 0;
#pragma unroll 4
        for (int q = 0; q < P; ++q) {
            const int4 o = sm.pk[q];
            sh += o.x == v ? o.z : 0;
            se += (o.y & 0xffff) == e ? o.z : 0;
            sp += (o.y >> 16) == d ? o.z : 0;
        }
        if (me.w < sh) { atomicMin(sm.misc + M_DH0, v); atomicMax(sm.misc + M_DH1, v); }
        if (sm.capE[e] < se) { atomicMin(sm.misc + M_DE0, e); atomicMax(sm.misc + M_DE1, e); }
        if (sm.capP[d] < sp) { atomicMin(sm.misc + M_DP0, d); atomicMax(sm.misc + M_DP1, d); }
    }
}

// ---------------------------------------------------------------- criteria
// Per-host criteria for one container.  xs rows (N ints each): [0, nc) the
// criteria values, nc the feasibility flag, nc+1..nc+5 partial accumulators
// kept across peer chunks.  With STATS the TOPSIS column statistics (exact
// sum of squares, max, min) are accumulated into the LDS slots; they are
// complete after the next barrier.
//
// Feasibility (Eqs. (4)-(5)): CPU and RAM fit; every remote peer's widest
// path carries its demand; and a set of conditions every successful commit
// satisfies, which spare the commit loop from trying servers bound to fail:
// the server's uplink, its edge switch's and its pod's uplinks each carry
// the demand of the peers outside them, and the peer-side deficits.
// With nwg > 1, workgroup wg of nwg takes every nwg-th group of G * BS
// servers (the other workgroups build the same peer tables for theirs).
// T0: the first chunk's table T was built by load_peers<.., true>.
template <int BS, bool STATS, int G = host_group(BS), int CS = 0, bool T0 = false>
__device__ __forceinline__ void criteria_stage(const Topo &t, const State &st, const Method &m, const Smem &sm, int *xs,
                               int cpu_i, int ram_i, int P, int pc_cap, int wg = 0, int nwg = 1) {
    const int N = t.N, nc = crit_count<CS>(m);
    const int nch = P == 0 ? 1 : (P + pc_cap - 1) / pc_cap;
    unsigned long long s2[kMaxCrit];
    int mx[kMaxCrit], mn[kMaxCrit];
#pragma unroll
    for (int c = 0; c < kMaxCrit; ++c) { s2[c] = 0; mx[c] = -kBig - 1; mn[c] = kBig; }
    for (int ch = 0; ch < nch; ++ch) {
        const int pbeg = ch * pc_cap;
        const int pn = min(P, pbeg + pc_cap) - pbeg;
        if (pn > 0) {
            if (ch == 0) peer_deficits<BS>(sm, P);
            if (!(T0 && ch == 0)) {
                if (ch > 0) __syncthreads();            // previous chunk done with the tables
                table_T<BS>(t, st, sm, pbeg, pn, [&](int pc) { return sm.pk[pbeg + pc].y >> 16; });
                __syncthreads();
            }
            table_E<BS>(t, st, sm, pbeg, pn);
            __syncthreads();
        }
        const int dh0 = sm.misc[M_DH0], dh1 = sm.misc[M_DH1];
        const int de0 = sm.misc[M_DE0], de1 = sm.misc[M_DE1];
        const int dp0 = sm.misc[M_DP0], dp1 = sm.misc[M_DP1];
        // G servers per thread at a time: one peer record feeds all of
        // them, and their independent chains hide the LDS latency
        constexpr int kHostGroup = G;
        for (int base = wg * kHostGroup * BS + threadIdx.x; base < N; base += nwg * kHostGroup * BS) {
            int uu[kHostGroup], up_u[kHostGroup], eu[kHostGroup], pu[kHostGroup];
            int pbw_acc[kHostGroup], up_acc[kHostGroup], hop_acc[kHostGroup], feas[kHostGroup];
            int oute[kHostGroup], outp[kHostGroup];
            bool valid[kHostGroup];
#pragma unroll
            for (int g = 0; g < kHostGroup; ++g) {
                const int u = base + g * BS;
                valid[g] = u < N;
                const int us = valid[g] ? u : 0;
                uu[g] = u;
                up_u[g] = st.up[us];
                eu[g] = edge_of(t, us);
                pu[g] = pod_of(t, us);
                if (ch == 0) {
                    pbw_acc[g] = up_u[g]; up_acc[g] = 0; hop_acc[g] = 0; oute[g] = 0; outp[g] = 0;
                    int f = (st.cpu[us] >= cpu_i) & (st.ram[us] >= ram_i);
                    if (!m.route_end) {
                        f &= (dh1 < 0) | ((dh0 == dh1) & (u == dh0));
                        f &= (de1 < 0) | ((de0 == de1) & (eu[g] == de0));
                        f &= (dp1 < 0) | ((dp0 == dp1) & (pu[g] == dp0));
                    }
                    feas[g] = f;
                } else {
                    feas[g] = xs[nc * N + us];
                    pbw_acc[g] = xs[(nc + 1) * N + us];
                    up_acc[g] = xs[(nc + 2) * N + us];
                    hop_acc[g] = xs[(nc + 3) * N + us];
                    oute[g] = xs[(nc + 4) * N + us];
                    outp[g] = xs[(nc + 5) * N + us];
                }
            }
            for (int pc = 0; pc < pn; ++pc) {
                const int4 pk = sm.pk[pbeg + pc];
                const int v = pk.x, bw = pk.z, ev = pk.y & 0xffff, pv = pk.y >> 16;
                const int *te = sm.tabE + pc * t.nsw;
#pragma unroll
                for (int g = 0; g < kHostGroup; ++g) {
                    const bool rem = v != uu[g];             // co-located peers use no link
                    const bool far = ev != eu[g];
                    const int e = te[eu[g]];
                    int w = min(up_u[g], pk.w);
                    w = far ? min(w, e) : w;
                    const int hop = !rem ? 0 : !far ? 2 : (pv == pu[g] ? 4 : 6);
                    pbw_acc[g] = rem ? min(pbw_acc[g], w) : pbw_acc[g];
                    up_acc[g] += rem ? bw : 0;
                    hop_acc[g] += hop;
                    feas[g] &= (!rem) | (w >= bw);
                    oute[g] += (rem & far) ? bw : 0;
                    outp[g] += (rem & far & (pv != pu[g])) ? bw : 0;
                }
            }
#pragma unroll
            for (int g = 0; g < kHostGroup; ++g) {
                if (!valid[g]) continue;
                const int u = uu[g];
                if (ch + 1 < nch) {
                    xs[nc * N + u] = feas[g];
                    xs[(nc + 1) * N + u] = pbw_acc[g];
                    xs[(nc + 2) * N + u] = up_acc[g];
                    xs[(nc + 3) * N + u] = hop_acc[g];
                    xs[(nc + 4) * N + u] = oute[g];
                    xs[(nc + 5) * N + u] = outp[g];
                    continue;
                }
                int f = feas[g] & (up_u[g] >= up_acc[g]);
                if (P > 0 && !m.route_end) f &= (sm.capE[eu[g]] >= oute[g]) & (sm.capP[pu[g]] >= outp[g]);
                xs[nc * N + u] = f;
#pragma unroll
                for (int c = 0; c < kMaxCrit; ++c) {
                    if (c >= nc) break;
                    int x;
                    switch (crit_at<CS>(m, c)) {
                    case CRIT_CPU: x = st.cpu[u]; break;
                    case CRIT_RAM: x = st.ram[u]; break;
                    case CRIT_ACTIVE: x = st.npl[u] > 0 ? 1 : 0; break;
                    case CRIT_PATHBW: x = pbw_acc[g]; break;
                    case CRIT_UPLINK: x = up_u[g]; break;
                    default: x = hop_acc[g]; break;
                    }
                    xs[c * N + u] = x;
                    if (STATS) {
                        s2[c] += static_cast<unsigned long long>(static_cast<long long>(x) * x);
                        mx[c] = max(mx[c], x);
                        mn[c] = min(mn[c], x);
                    }
                }
            }
        }
    }
    if (STATS) {
        // exact column statistics: the 64-bit sum of squares travels as
        // three 17-bit chunks whose wave and block sums cannot overflow;
        // each wave stores its partials in its own slots
        const int lane = threadIdx.x & (kWave - 1), wid = threadIdx.x / kWave;
#pragma unroll
        for (int c = 0; c < kMaxCrit; ++c) {
            if (c >= nc) break;
            const int c0 = wave_sum(static_cast<int>(s2[c] & 0x1ffffu));
            const int c1 = wave_sum(static_cast<int>((s2[c] >> 17) & 0x1ffffu));
            const int c2 = wave_sum(static_cast<int>(s2[c] >> 34));
            const int hi = wave_max(mx[c]), lo = wave_min(mn[c]);
            if (lane < 5) {
                const int v = lane == 0 ? c0 : lane == 1 ? c1 : lane == 2 ? c2 : lane == 3 ? hi : -lo;
                sm.wst[(5 * c + lane) * kMaxWaves + wid] = v;
            }
        }
    }
}

// Block totals of the column statistics from the per-wave slots (after a
// barrier), computed by every wave on its own: the 16 lanes of a row take
// one field's wave partials and reduce them with row DPP.  Fields 5c..5c+2
// sum, 5c+3 and 5c+4 (max and -min) take the maximum.
template <int BS>
__device__ __forceinline__ void finish_stats(const Smem &sm, int nc, unsigned long long *s2, int *mx, int *mn) {
    constexpr int NW = BS / kWave;
    const int lane = threadIdx.x & (kWave - 1), row = lane >> 4, w = lane & 15;
    int fin[kStatFields];
#pragma unroll
    for (int r = 0; r < kStatFields / 4; ++r) {
        if (4 * r >= 5 * nc) break;
        const int f = 4 * r + row;
        const bool is_sum = (f % 5) < 3;
        const int id = is_sum ? 0 : -kBig - 1;
        int v = (w < NW && f < 5 * nc) ? sm.wst[f * kMaxWaves + w] : id;
        int vs = v, vm = v;
        DCS_ROW_REDUCE(vs, op_add, 0);
        DCS_ROW_REDUCE(vm, op_max, -kBig - 1);
        const int res = is_sum ? vs : vm;
#pragma unroll
        for (int q = 0; q < 4; ++q) fin[4 * r + q] = __builtin_amdgcn_readlane(res, 16 * q + 15);
    }
#pragma unroll
    for (int c = 0; c < kMaxCrit; ++c) {
        if (c >= nc) break;
        s2[c] = static_cast<unsigned long long>(static_cast<unsigned>(fin[5 * c])) +
                (static_cast<unsigned long long>(static_cast<unsigned>(fin[5 * c + 1])) << 17) +
                (static_cast<unsigned long long>(static_cast<unsigned>(fin[5 * c + 2])) << 34);
        mx[c] = fin[5 * c + 3];
        mn[c] = -fin[5 * c + 4];
    }
}

// TOPSIS closeness of one server from its integer criteria get(c), c < nc
// (section V-C): Ed+- = sqrt(sum_c q_c (x_c - A+-_c)^2) with q_c = w_c^2 /
// sum_u x_cu^2, Rank = Ed- / (Ed+ + Ed-), 0 when both are 0.  Differences of
// integers below 2^22 are exact in FP32; the square roots and the quotient
// use the hardware square root and reciprocal (1 ulp).  Every form scores
// through this function, so equal criteria and statistics give equal bits.
template <class Get>
__device__ __forceinline__ float topsis_close(int nc, Get get, const float *q, const float *ap, const float *am) {
    float dp2 = 0.f, dm2 = 0.f;
#pragma unroll
    for (int c = 0; c < kMaxCrit; ++c) {
        if (c >= nc) break;
        const float x = static_cast<float>(get(c));
        const float a = x - ap[c], z = x - am[c];
        dp2 = fmaf(q[c] * a, a, dp2);
        dm2 = fmaf(q[c] * z, z, dm2);
    }
    const float dp = __builtin_amdgcn_sqrtf(dp2), dm = __builtin_amdgcn_sqrtf(dm2);
    const float den = dp + dm;
    return den > 0.f ? fminf(dm * __builtin_amdgcn_rcpf(den), 1.0f) : 0.f;
}

// Column statistics when the criteria rows sit in LDS: wave c reduces
// column c over all servers (exact 64-bit sum of squares as three 17-bit
// chunks, maximum, minimum) and its lane 0 turns them into the scoring
// factors q_c = w_c^2 / sum x^2, A+_c and A-_c, kept as floats in the wst
// slots; every thread reads them after the barrier.  Same values as the
// per-wave path of criteria_stage + finish_stats, with 5 wave reductions per
// criterion instead of 5 per criterion in every wave.
template <int BS, int CS = 0>
__device__ __forceinline__ void column_factors_lds(const Smem &sm, const Method &m, const int *xs, int N, float *q,
                                                   float *ap, float *am) {
    constexpr int NW = BS / kWave;
    const int lane = threadIdx.x & (kWave - 1), wid = threadIdx.x / kWave;
    float *f = reinterpret_cast<float *>(sm.wst);
    for (int c = wid; c < crit_count<CS>(m); c += NW) {
        const int *col = xs + static_cast<size_t>(c) * N;
        unsigned long long s2 = 0;
        int hi = -kBig - 1, lo = kBig;
#pragma unroll 8
        for (int u = lane; u < N; u += kWave) {
            const int x = col[u];
            s2 += static_cast<unsigned long long>(static_cast<unsigned>(x)) * static_cast<unsigned>(x);
            hi = max(hi, x);
            lo = min(lo, x);
        }
        const unsigned c0 = static_cast<unsigned>(wave_sum(static_cast<int>(s2 & 0x1ffffu)));
        const unsigned c1 = static_cast<unsigned>(wave_sum(static_cast<int>((s2 >> 17) & 0x1ffffu)));
        const unsigned c2 = static_cast<unsigned>(wave_sum(static_cast<int>(s2 >> 34)));
        hi = wave_max(hi);
        lo = wave_min(lo);
        if (lane == 0) {
            const unsigned long long a = static_cast<unsigned long long>(c0) +
                                         (static_cast<unsigned long long>(c1) << 17) +
                                         (static_cast<unsigned long long>(c2) << 34);
            // the weight by constant indices (scalar loads the compiler
            // hoists), not by the wave's index (a vector load per step)
            float wc = 0.f;
#pragma unroll
            for (int x = 0; x < kMaxCrit; ++x) wc = x == c ? m.w[x] : wc;
            f[c] = a ? (wc * wc) / static_cast<float>(a) : 0.0f;
            f[kMaxCrit + c] = static_cast<float>(crit_cost<CS>(m, c) ? lo : hi);
            f[2 * kMaxCrit + c] = static_cast<float>(crit_cost<CS>(m, c) ? hi : lo);
        }
    }
    __syncthreads();
#pragma unroll
    for (int c = 0; c < kMaxCrit; ++c) {
        q[c] = ap[c] = am[c] = 0.f;
        if (c >= crit_count<CS>(m)) continue;
        q[c] = f[c];
        ap[c] = f[kMaxCrit + c];
        am[c] = f[2 * kMaxCrit + c];
    }
}

__device__ __forceinline__ unsigned long long score_key(float s, int u) {
    return (static_cast<unsigned long long>(__float_as_uint(s) + 1u) << 32) | static_cast<unsigned>(~u);
}

// Trace slot of this step, or -1.  Called by thread 0 only; rid is the
// request id recorded in the slot's metadata.
__device__ __forceinline__ int trace_slot(const Trace &tr, int inst, int rid, int i) {
    if (tr.stride <= 0) return -1;
    const int s = tr.counter[inst];
    tr.counter[inst] = s + 1;
    if (s % tr.stride) return -1;
    const int slot = s / tr.stride;
    if (slot >= tr.cap) return -1;
    tr.meta[4 * slot + 0] = inst;
    tr.meta[4 * slot + 1] = rid;
    tr.meta[4 * slot + 2] = i;
    tr.meta[4 * slot + 3] = s;
    return slot;
}

// Routing after the last unit of request r is placed (section V-D, with
// Method::route_end): every routed pair's widest minimum-hop path is chosen
// on the residuals the placement left, all pairs independently (one wave per
// unit's pairs); then every minimum demand is taken off its links at once.
// If a link goes negative the request does not fit: everything it took is
// given back and it is rejected with failed_at = n.  Otherwise wave 0 tops
// each pair up, in pair order, by what its most loaded link still has, to
// at most the pair's maximum.  host(g) is the server of unit
// g (u for the unit just placed).  Returns true when the request was
// accepted.
template <int BS, class HostFn>
__device__ __forceinline__ bool route_request_end(const Topo &t, const State &st, const Batch &b, int *lds_ok, const StepIn &s,
                                  HostFn host) {
    constexpr int NW = BS / kWave;
    const int lane = threadIdx.x & (kWave - 1), wid = threadIdx.x / kWave;
    // All waves of the workgroup share one CU and its write-through L1, and
    // the link updates below are L2 atomics, so ordering inside the routine
    // needs only workgroup fences; one agent fence at the end of an accepted
    // request orders its link changes before whatever step comes next.
    __threadfence_block();
    if (threadIdx.x == 0) *lds_ok = 1;
    __syncthreads();
    for (int g = wid; g < s.n; g += NW) {
        const int u = host(g), eu = edge_of(t, u), pu = pod_of(t, u);
        for (int x = b.poff[s.g0 + g]; x < b.poff[s.g0 + g + 1]; ++x) {
            const int v = host(b.pj[x]);
            int c = -1;
            if (v != u) {
                const unsigned best = widest_wave(t, st, u, v, eu, pu, edge_of(t, v), pod_of(t, v), lane);
                c = 1023 - static_cast<int>(best & 1023u);
            }
            if (lane == 0) {
                b.code[x] = c;
                b.pbwa[x] = c >= 0 ? b.pbw[x] : b.pbmax[x];
            }
        }
    }
    __threadfence_block();
    __syncthreads();
    for (int g = wid; g < s.n; g += NW) {                  // take every demand off its path
        const int u = host(g);
        for (int x = b.poff[s.g0 + g]; x < b.poff[s.g0 + g + 1]; ++x) {
            const int c = b.code[x];
            if (c >= 0) path_apply_lanes<true>(t, st, u, host(b.pj[x]), c, -b.pbwa[x], lane);
        }
    }
    __threadfence_block();
    __syncthreads();
    for (int g = wid; g < s.n; g += NW) {                  // any link overdrawn?
        const int u = host(g);
        for (int x = b.poff[s.g0 + g]; x < b.poff[s.g0 + g + 1]; ++x) {
            const int c = b.code[x];
            if (c >= 0) {
                const int *l = path_link_lane(t, st, u, host(b.pj[x]), c, lane);
                if (l && __hip_atomic_load(l, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) < 0) *lds_ok = 0;
            }
        }
    }
    __syncthreads();
    if (*lds_ok) {
        if (wid == 0)
            for (int g = 0; g < s.n; ++g) {
                const int u = host(g);
                for (int x = b.poff[s.g0 + g]; x < b.poff[s.g0 + g + 1]; ++x) {
                    const int c = b.code[x], room = b.pbmax[x] - b.pbw[x];
                    if (c < 0 || room <= 0) continue;
                    const int v = host(b.pj[x]);
                    const int *l = path_link_lane(t, st, u, v, c, lane);
                    const int left = l ? __hip_atomic_load(l, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) : kBig;
                    const int add = min(room, wave_min(left));
                    if (add <= 0) continue;
                    path_apply_lanes<true>(t, st, u, v, c, -add, lane);
                    if (lane == 0) b.pbwa[x] = b.pbw[x] + add;
                    __threadfence_block();
                }
            }
        __threadfence();
        vm_drain();
        __syncthreads();
        return true;
    }
    give_back<BS>(t, st, b, s.r, s.n);          // all units and their routes
    __syncthreads();
    if (threadIdx.x == 0) {
        b.status[s.r] = 0;
        b.failat[s.r] = s.n;
        b.tse[s.r] = dev_clock();
    }
    __threadfence_block();
    vm_drain();
    __syncthreads();
    return false;
}

// Select-and-commit loop shared by TOPSIS and AHP: key_of(u) gives the
// score key of a feasible server (score bits + 1 above ~u, so a feasible
// server's key is never 0).  Servers are visited in decreasing key order by
// repeated block argmax (wave max, then one LDS atomic per wave); a server
// whose commit fails is masked in the feasibility row, only its owner
// thread rescans its servers, and the argmax repeats.  Rolls the request
// back when no server is left.  Returns true when the container was placed.
template <int BS, int G, class KeyFn>
__device__ __forceinline__ bool select_commit(const Topo &t, const State &st, const Batch &b, const Smem &sm, int *feas_row,
                              const StepIn &s, const ReqView &rv, int m_route_end, KeyFn key_of) {
    const int lane = threadIdx.x & (kWave - 1);
    auto scan = [&]() {
        unsigned long long kb = 0;
        for (int base = threadIdx.x; base < t.N; base += G * BS) {
#pragma unroll
            for (int g = 0; g < G; ++g) {
                const int u = base + g * BS;
                const int us = u < t.N ? u : 0;
                const unsigned long long k = (u < t.N && feas_row[us]) ? key_of(us) : 0ull;
                kb = k > kb ? k : kb;
            }
        }
        return kb;
    };
    constexpr int NW = BS / kWave;
    const int wid = threadIdx.x / kWave;
    // at most one server per thread, thread u holding server u (N <= BS, a
    // compile-time fact): lanes and waves are in server order, so among
    // equal high words the first lane (wave) holds the lowest server, the
    // largest low word, and a ballot replaces the second reduction
    auto low_of = [&](unsigned hi, unsigned hiw, unsigned lo) -> unsigned {
        if (__builtin_constant_p(t.N) && t.N <= BS) {
            const unsigned long long m = __ballot(hi == hiw);
            return __builtin_amdgcn_readlane(lo, m ? __builtin_ctzll(m) : 0);
        }
        return wave_umax(hi == hiw ? lo : 0u);
    };
    unsigned long long mine = scan();
    for (int it = 0;; ++it) {
        unsigned *shi = sm.ahi + (it & 1) * kMaxWaves, *slo = sm.alo + (it & 1) * kMaxWaves;
        // wave argmax: largest high word, then among those the largest low
        // word; one slot per wave, then every wave reduces the slots
        unsigned hiw = wave_umax(static_cast<unsigned>(mine >> 32));
        unsigned low = low_of(static_cast<unsigned>(mine >> 32), hiw, static_cast<unsigned>(mine));
        if (lane == 0) { shi[wid] = hiw; slo[wid] = low; }
        __syncthreads();
        const unsigned wh = lane < NW ? shi[lane] : 0u, wl = lane < NW ? slo[lane] : 0u;
        hiw = wave_umax(wh);
        low = low_of(wh, hiw, wl);
        const unsigned long long kb = (static_cast<unsigned long long>(hiw) << 32) | low;
        if (hiw == 0) {
            rollback_request<BS>(t, st, b, s.r, s.i, &rv, &s);
            return false;
        }
        const int u = static_cast<int>(~static_cast<unsigned>(kb & 0xffffffffu));
        if (threadIdx.x < kWave) {
            const GPtr<int> o_host = b.host;              // read before the commit's fences
            const GPtr<float> o_score = b.score;
            const GPtr<long long> o_tse = b.tse;
            const bool ok = commit_wave(t, st, b, u, s, m_route_end ? 0 : s.P, sm, sm.pbw, lane);
            if (lane == 0) {
                sm.misc[M_OK] = ok;
                if (ok) {
                    o_host[s.g] = u;
                    if (rv.hosts_out) rv.hosts_out[s.i] = u;
                    o_score[s.g] = __uint_as_float(static_cast<unsigned>(kb >> 32) - 1u);
                    if (s.i == s.n - 1) o_tse[s.r] = dev_clock();
                } else {
                    feas_row[u] = 0;
                }
            }
        }
        __threadfence_block();
        __syncthreads();
        if (sm.misc[M_OK]) {
            if (m_route_end && s.i == s.n - 1)
                return route_request_end<BS>(t, st, b, sm.misc + M_ROUTE, s,
                                             [&](int g) { return g == s.i ? u : rv.hosts[g]; });
            return true;
        }
        if (u % BS == static_cast<int>(threadIdx.x)) mine = scan();
    }
}

// ---------------------------------------------------------------- TOPSIS step (section V-C)
// Scores every server by closeness to the ideal solution: column L2
// normalisation and weighting fold into q_c = w_c^2 / sum_u x_cu^2, so
// Ed+- = sqrt(sum_c q_c (x_cu - A+-_c)^2) with A+- the column max / min in
// raw units (swapped for cost criteria); Rank = Ed- / (Ed+ + Ed-), 0 when
// both are 0.  Column statistics are exact integer reductions.  Returns
// false when the request was rejected at this container.
// XS_LDS: the criteria rows xs are in LDS, so the column statistics are
// taken from them afterwards by one wave per criterion.
template <int BS, int G = host_group(BS), bool XS_LDS = false, int CS = 0>
__device__ __forceinline__ bool topsis_step(const Topo &t, const State &st, const Method &m, const Batch &b, const Smem &sm,
                            int *xs, int pc_cap, const Trace &tr, int inst, const StepIn &s, const ReqView &rv) {
    if (s.i == 0 && threadIdx.x == 0) b.tsb[s.r] = dev_clock();
    if (threadIdx.x == 0) {
        int slot = -1;
        if (tr.stride > 0) {
            slot = trace_slot(tr, inst, b.rid[s.r], s.i);
            vm_drain();
        }
        sm.misc[M_TRACE] = slot;
    }
    load_peers<BS, true, true>(t, st, rv, sm, s.P, pc_cap);
    const int nc = crit_count<CS>(m), N = t.N;
    criteria_stage<BS, !XS_LDS, G, CS, true>(t, st, m, sm, xs, s.cpu, s.ram, s.P, pc_cap);
    __syncthreads();

    float q[kMaxCrit], ap[kMaxCrit], am[kMaxCrit];
    if (XS_LDS) {
        column_factors_lds<BS, CS>(sm, m, xs, N, q, ap, am);
    } else {
        unsigned long long s2[kMaxCrit];
        int mx[kMaxCrit], mn[kMaxCrit];
        finish_stats<BS>(sm, nc, s2, mx, mn);
#pragma unroll
        for (int c = 0; c < kMaxCrit; ++c) {
            q[c] = ap[c] = am[c] = 0.f;
            if (c >= nc) continue;
            const unsigned long long a = s2[c];
            q[c] = a ? (m.w[c] * m.w[c]) / static_cast<float>(a) : 0.0f;
            ap[c] = static_cast<float>(crit_cost<CS>(m, c) ? mn[c] : mx[c]);
            am[c] = static_cast<float>(crit_cost<CS>(m, c) ? mx[c] : mn[c]);
        }
    }
    auto closeness = [&](int u) -> float {
        return topsis_close(nc, [&](int c) { return xs[c * N + u]; }, q, ap, am);
    };
    const int slot = sm.misc[M_TRACE];
    if (slot >= 0)
        for (int u = threadIdx.x; u < N; u += BS) tr.scores[static_cast<size_t>(slot) * N + u] = closeness(u);
    return select_commit<BS, G>(t, st, b, sm, xs + nc * N, s, rv, m.route_end,
                                             [&](int u) { return score_key(closeness(u), u); });
}

}  // namespace dcs
