// libdcsched host runtime: the C ABI of include/dcsched.h over the kernels of
// dc_kernels.hpp.  Owns the device-resident data-center state, uploads
// request batches, drives the plain (one launch per container step) and
// batched (one persistent launch) forms, and collects results.
#include "../../include/dcsched.h"
#include "dc_kernels.hpp"
#include "dc_grid.hpp"
#include "dc_tiles.hpp"

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <chrono>
#include <fstream>
#include <map>
#include <memory>
#include <mutex>
#include <sstream>
#include <string>
#include <thread>
#include <unordered_map>
#include <vector>

using namespace dcs;

namespace {

// Launch shape of the batched kernel: threads per workgroup, servers each
// thread scores together, peers whose path tables are built together.
struct Shape {
    int bs = 1024, g = 1, pc = 1;
    bool operator==(const Shape &o) const { return bs == o.bs && g == o.g && pc == o.pc; }
};

// (threads, servers per thread) pairs the batched kernel is built for.
constexpr int kBatchedShapes[][2] = {{256, 1}, {256, 2}, {256, 4}, {512, 1}, {512, 2}, {512, 4}, {1024, 1}, {1024, 2}};

bool batched_shape_built(int bs, int g) {
    for (const auto &x : kBatchedShapes)
        if (x[0] == bs && x[1] == g) return true;
    return false;
}

// A request's containers and edges as submitted, kept so that what each
// unit and unit pair is given can be handed back to them.
struct Members {
    std::vector<int> cpu, cmax, ram, rmax;   // per container: demand intervals
    std::vector<int> emin, emax;             // per edge: bandwidth interval
    std::vector<int> epair;                  // per edge: the unit pair carrying it (unit CSR index), -1 inside a unit
};

// A request as the device schedules it.  Containers of a pod share one
// server (section II-A, Eq. (8)), so the unit of placement is the pod: one
// unit per pod, in the order of each pod's first container (a container
// without a pod is a pod of its own), asking for the summed CPU and RAM of
// its containers.  The peers of unit g are the earlier units h whose
// containers exchange traffic with g's, each with the summed demand: the two
// pods sit on one server each, so their links share one route.  Traffic
// inside a pod needs no network.  Without pods every container is a unit
// and its peers are the earlier containers it talks to.  Demands are
// intervals (section II-A); minima and maxima are summed separately.
struct Units {
    int n = 0;                         // containers
    std::vector<int> cpu, ram;         // per unit, minima
    std::vector<int> cmax, rmax;       // per unit, maxima
    std::vector<int> poff, pj, pbw;    // peers of each unit (CSR), ascending unit index, minimum demand
    std::vector<int> pbmax;            // maximum demand of each peer pair
    std::vector<int> unit_of;          // container -> unit
    std::vector<int> first;            // unit -> its smallest container index
    Members mem;
    int nu() const { return (int)cpu.size(); }
};

// Builds the units of a validated request; DC_EINVAL when a summed demand
// reaches past the 2^22 bound of capacities.  pod[i] >= 0 names container
// i's pod (equal ids, same pod); pod[i] < 0 or pod == NULL: no pod.
// cpu_max, ram_max, bw_max (per edge) are the maxima, or NULL for fixed
// demands.
int build_units(int n, const int *cpu, const int *cpu_max, const int *ram, const int *ram_max, int m,
                const int *edges, const int *bw_max, const int *pod, Units &u) {
    constexpr long long kCap = 1LL << 22;
    u = Units{};
    u.n = n;
    u.unit_of.assign(n, -1);
    std::vector<long long> uc, ur, ucx, urx;
    std::map<int, int> pod_unit;
    Members &M = u.mem;
    for (int i = 0; i < n; ++i) {
        int g = -1;
        if (pod && pod[i] >= 0) {
            auto it = pod_unit.find(pod[i]);
            if (it != pod_unit.end()) g = it->second;
            else pod_unit[pod[i]] = g = (int)uc.size();
        } else {
            g = (int)uc.size();
        }
        if (g == (int)uc.size()) {
            uc.push_back(0);
            ur.push_back(0);
            ucx.push_back(0);
            urx.push_back(0);
            u.first.push_back(i);
        }
        u.unit_of[i] = g;
        M.cpu.push_back(cpu[i]);
        M.ram.push_back(ram[i]);
        M.cmax.push_back(cpu_max ? cpu_max[i] : cpu[i]);
        M.rmax.push_back(ram_max ? ram_max[i] : ram[i]);
        uc[g] += cpu[i];
        ur[g] += ram[i];
        ucx[g] += M.cmax.back();
        urx[g] += M.rmax.back();
    }
    const int nu = (int)uc.size();
    for (int g = 0; g < nu; ++g) {
        if (ucx[g] > kCap || urx[g] > kCap) return DC_EINVAL;
        u.cpu.push_back((int)uc[g]);
        u.ram.push_back((int)ur[g]);
        u.cmax.push_back((int)ucx[g]);
        u.rmax.push_back((int)urx[g]);
    }
    std::vector<long long> bw((size_t)nu * nu, 0), bwx((size_t)nu * nu, 0);
    for (int q = 0; q < m; ++q) {
        const int a = u.unit_of[edges[3 * q]], b = u.unit_of[edges[3 * q + 1]];
        M.emin.push_back(edges[3 * q + 2]);
        M.emax.push_back(bw_max ? bw_max[q] : edges[3 * q + 2]);
        if (a == b) continue;
        bw[(size_t)a * nu + b] += edges[3 * q + 2];
        bw[(size_t)b * nu + a] += edges[3 * q + 2];
        bwx[(size_t)a * nu + b] += M.emax.back();
        bwx[(size_t)b * nu + a] += M.emax.back();
    }
    std::vector<int> pidx((size_t)nu * nu, -1);
    u.poff.assign(1, 0);
    for (int g = 0; g < nu; ++g) {
        for (int h = 0; h < g; ++h) {
            const long long w = bw[(size_t)g * nu + h], wx = bwx[(size_t)g * nu + h];
            if (wx > kCap) return DC_EINVAL;
            if (w > 0) {
                pidx[(size_t)g * nu + h] = pidx[(size_t)h * nu + g] = (int)u.pj.size();
                u.pj.push_back(h);
                u.pbw.push_back((int)w);
                u.pbmax.push_back((int)wx);
            }
        }
        u.poff.push_back((int)u.pj.size());
    }
    for (int q = 0; q < m; ++q)
        M.epair.push_back(pidx[(size_t)u.unit_of[edges[3 * q]] * nu + u.unit_of[edges[3 * q + 1]]]);
    return DC_OK;
}

// Hands the allocation a of a unit (or unit pair) back to its members who[]
// in order: each first gets its minimum, then what is left goes up to each
// one's maximum in turn.
void hand_back(long long a, const std::vector<int> &who, const std::vector<int> &mn, const std::vector<int> &mx,
               int32_t *out) {
    for (int x : who) { out[x] = mn[x]; a -= mn[x]; }
    for (int x : who) {
        const long long t = std::min<long long>(a, (long long)mx[x] - mn[x]);
        out[x] += (int32_t)t;
        a -= t;
    }
}

// Allocations per container and per edge from those of the units (ua_cpu,
// ua_ram, nu entries) and unit pairs (pa, relative to the request's first
// pair).  An edge inside a unit uses no link and gets its maximum.
void members_alloc(const Members &M, const std::vector<int> &unit_of, int nu, const int *ua_cpu,
                   const int *ua_ram, const int *pa, int32_t *cpu, int32_t *ram, int32_t *bw) {
    const int n = (int)M.cpu.size(), m = (int)M.emin.size();
    std::vector<std::vector<int>> who(nu);
    for (int i = 0; i < n; ++i) who[unit_of[i]].push_back(i);
    for (int g = 0; g < nu; ++g) {
        if (cpu) hand_back(ua_cpu[g], who[g], M.cpu, M.cmax, cpu);
        if (ram) hand_back(ua_ram[g], who[g], M.ram, M.rmax, ram);
    }
    if (!bw) return;
    std::map<int, std::vector<int>> by_pair;
    for (int q = 0; q < m; ++q) {
        if (M.epair[q] < 0) bw[q] = M.emax[q];
        else by_pair[M.epair[q]].push_back(q);
    }
    for (const auto &kv : by_pair) hand_back(pa[kv.first], kv.second, M.emin, M.emax, bw);
}

// One uploaded set of requests (the pending queue at a dc_schedule call).
struct DevBatch {
    int R = 0, Ct = 0, Pt = 0, I = 0;
    int *dmem = nullptr;           // device: inputs then outputs
    size_t in_ints = 0, out_ints = 0;
    Batch view{};
    std::vector<int64_t> ids;      // request id per batch request
    std::vector<int> inst, coff, poff, pj, pbw, cpu, ram, iroff;   // unit level (coff: units per request)
    std::vector<int> cmax, rmax, pbmax;                            // unit level maxima
    std::vector<Members> mem;                                      // per request
    size_t o_alloc = 0;                                            // output offset of cpua, rama, pbwa
    std::vector<int> cnt, cuoff, unit_of, first;                   // containers per request, their units, first containers
    std::vector<int> host, status, failat;
    std::vector<float> score;
    std::vector<long long> tsb, tse;
    hipGraphExec_t gexec = nullptr;    // batched form: captured launch of this batch
    Shape gshape{0, 0, 0};             // launch shape it was captured with
    int *pinned = nullptr;             // pinned host copy of the outputs, route codes left out
    ~DevBatch() {
        if (gexec) (void)hipGraphExecDestroy(gexec);
        if (pinned) (void)hipHostFree(pinned);
    }
};

struct ReqLoc {
    int batch = -1, r = -1;
    bool released = false;
};

// Serving form: one live request's slot in the device arena.
struct ServeSlot {
    size_t off = 0, ints = 0;      // offset and size in the arena (int32 units)
    int n = 0, P = 0;              // units and peer pairs as the device sees them
    int nc = 0;                    // containers
    std::vector<int> unit_of, first;
    Members mem;
    int status = -1;               // -1 pending, 1 accepted, 0 rejected
    bool released = false;
    std::vector<int> hosts;        // attempt record from the completion
};

// Serving form state: rings in coherent pinned host memory, the device slot
// arena with a first-fit allocator, and the host's ring positions.
struct Serve {
    Cmd *cmds = nullptr;
    Comp *comps = nullptr;
    int *ctrl = nullptr;
    int *staging = nullptr;
    int *arena = nullptr;
    size_t arena_ints = 0;
    std::map<size_t, size_t> free_list;     // offset -> size, int32 units
    int cap = 1024, stage_ints = 0, bs = 1024, pc = 1;
    size_t lds = 0;
    long long idle_ticks = 100000000LL;     // 1 s of device clock
    int64_t host_pos = 0, comp_pos = 0;     // commands published / completions consumed
    std::unordered_map<int64_t, ServeSlot> slots;
    std::unordered_map<int, int64_t> rid_to_id;
    std::vector<std::pair<int64_t, float>> service_us;
    hipStream_t aux = nullptr;              // copies while the persistent kernel runs
    bool launched = false;
};

bool serve_alloc(Serve &sv, size_t ints, size_t *off) {
    ints = (ints + 3) & ~size_t(3);
    for (auto it = sv.free_list.begin(); it != sv.free_list.end(); ++it) {
        if (it->second >= ints) {
            *off = it->first;
            const size_t rest = it->second - ints, roff = it->first + ints;
            sv.free_list.erase(it);
            if (rest) sv.free_list[roff] = rest;
            return true;
        }
    }
    return false;
}

void serve_free(Serve &sv, size_t off, size_t ints) {
    ints = (ints + 3) & ~size_t(3);
    auto it = sv.free_list.emplace(off, ints).first;
    auto nx = std::next(it);
    if (nx != sv.free_list.end() && it->first + it->second == nx->first) {
        it->second += nx->second;
        sv.free_list.erase(nx);
    }
    if (it != sv.free_list.begin()) {
        auto pv = std::prev(it);
        if (pv->first + pv->second == it->first) {
            pv->second += it->second;
            sv.free_list.erase(it);
        }
    }
}

}  // namespace

struct dc_ctx {
    dc_config cfg{};
    Topo t{};
    Method m{};
    int N = 0, I = 0;
    hipStream_t stream = nullptr;
    bool own_stream = false;
    bool poisoned = false;
    int *d_state = nullptr;        // [I][6][N]
    int *d_init = nullptr;         // [I][6][N]
    int *d_xs = nullptr;           // [I][nc+6][N]
    int *d_colpart = nullptr;      // AHP [nc][nI][N]
    float *d_rowpart = nullptr;    // AHP [nc][nJ][N]
    int ti = 0, tj = 0, nI = 0, nJ = 0;
    bool ahp_sorted = false;       // AHP on the 1-9 scale through the sorted passes
    int *d_ysort = nullptr;        // [nc][N]
    int *d_runs = nullptr;         // [nc][sort_runs][1024] sorted runs before their merge
    double *d_wsort = nullptr;     // [nc][N]
    int sort_runs = 1;             // sorted passes: runs of 1,024 values sorted apart, then merged
    int *d_tmeta = nullptr, *d_tcount = nullptr;
    float *d_tscore = nullptr;
    int plain_bs = 1024;
    Shape bshape{};                // batched form: current launch shape
    int pc_plain = 1, pc_batched = 1;  // peer chunk of the plain form; largest the batched LDS holds
    bool plain_res = false;        // plain kernel stages state + scratch in LDS
    size_t lds_plain = 0, lds_select = 0;
    std::vector<std::unique_ptr<DevBatch>> batches;
    std::vector<int> queued;       // batches uploaded and waiting to run
    std::vector<int> pend_inst;
    std::vector<Units> pend_units;
    std::vector<int64_t> pend_ids;
    std::unordered_map<int64_t, ReqLoc> loc;
    int64_t next_id = 0;
    std::vector<dc_result> ready;  // decided results not yet handed out, from ready_head on
    size_t ready_head = 0;
    hipEvent_t ev0 = nullptr, ev1 = nullptr;
    float last_ms = 0.f;
    int64_t last_launches = 0, last_steps = 0;
    std::unique_ptr<Serve> sv;     // serving form only
    // cooperative (one workgroup per pod) TOPSIS step
    bool use_grid = false;
    GridCtl grid{};
    int *d_grid = nullptr;         // backing allocation of grid
    size_t lds_grid = 0;
    long long grid_timeout = 10000000LL;   // 100 ms of device clock per barrier wait
    hipError_t launch_err = hipSuccess;    // first failed cooperative launch of a run
    hipStream_t cap_stream = nullptr;      // graph capture (batched form)
};

#define HIPCHK(expr)                                       \
    do {                                                   \
        hipError_t e_ = (expr);                            \
        if (e_ != hipSuccess) {                            \
            ctx->poisoned = true;                          \
            std::fprintf(stderr, "libdcsched: %s failed: %s\n", #expr, hipGetErrorString(e_)); \
            return DC_EDEVICE;                             \
        }                                                  \
    } while (0)

namespace {

int check_config(const dc_config *c) {
    if (!c) return DC_EINVAL;
    if (c->k < 4 || c->k > 64 || (c->k & 1)) return DC_EINVAL;
    if (c->n_instances < 1 || c->n_instances > 65536) return DC_EINVAL;
    if (c->mode < DC_MODE_PLAIN || c->mode > DC_MODE_SERVING) return DC_EINVAL;
    if (c->method != DC_TOPSIS && c->method != DC_AHP) return DC_EINVAL;
    if (c->method == DC_AHP && c->ahp_scale != DC_AHP_SAATY9 && c->ahp_scale != DC_AHP_RATIO &&
        c->ahp_scale != DC_AHP_DIFF)
        return DC_EINVAL;
    if (c->method == DC_AHP && c->mode != DC_MODE_PLAIN) return DC_EINVAL;
    const int caps[5] = {c->host_cpu, c->host_ram, c->bw_host_edge, c->bw_edge_agg, c->bw_agg_core};
    for (int v : caps)
        if (v < 0 || v >= (1 << 22)) return DC_EINVAL;   // exact in FP32; fits the 22-bit path keys
    if (c->ncrit < 1 || c->ncrit > DC_MAX_CRIT) return DC_EINVAL;
    double ws = 0.0;
    for (int i = 0; i < c->ncrit; ++i) {
        if (c->crit[i] < DC_CRIT_CPU || c->crit[i] > DC_CRIT_HOPS) return DC_EINVAL;
        if (!(c->weight[i] > 0.f) || !std::isfinite(c->weight[i])) return DC_EINVAL;
        ws += c->weight[i];
    }
    if (std::fabs(ws - 1.0) > 1e-5) return DC_EINVAL;
    if (c->block != 0 && c->block != 64 && c->block != 256 && c->block != 512 && c->block != 1024) return DC_EINVAL;
    if (c->trace_stride < 0 || c->trace_cap < 0) return DC_EINVAL;
    if (c->grid < 0 || c->grid > 2) return DC_EINVAL;
    if (c->graph < 0 || c->graph > 2) return DC_EINVAL;
    if (c->grid_timeout_us < 0) return DC_EINVAL;
    if (c->routing < 0 || c->routing > 1) return DC_EINVAL;
    return DC_OK;
}

// Links of the path between servers u != v for candidate c, as global link
// ids (level * N + index); returns the count.
int host_path_links(const Topo &t, int u, int v, int c, int *out) {
    const int eu = u / t.h, ev = v / t.h, pu = u / t.hh, pv = v / t.hh;
    int a = 0, j = 0;
    if (pu == pv) a = c; else { a = c / t.h; j = c - a * t.h; }
    int nl = 0;
    out[nl++] = u;
    if (eu != ev) out[nl++] = t.N + eu * t.h + a;
    if (pu != pv) {
        out[nl++] = 2 * t.N + (pu * t.h + a) * t.h + j;
        out[nl++] = 2 * t.N + (pv * t.h + a) * t.h + j;
    }
    if (eu != ev) out[nl++] = t.N + ev * t.h + a;
    out[nl++] = v;
    return nl;
}

template <class K>
int set_lds(dc_ctx *ctx, K kernel, size_t bytes) {
    HIPCHK(hipFuncSetAttribute(reinterpret_cast<const void *>(kernel), hipFuncAttributeMaxDynamicSharedMemorySize,
                               static_cast<int>(bytes)));
    return DC_OK;
}

State state_of(dc_ctx *ctx, int inst) {
    int *s = ctx->d_state + (size_t)inst * 6 * ctx->N;
    const int N = ctx->N;
    return State{s, s + N, s + 2 * N, s + 3 * N, s + 4 * N, s + 5 * N};
}

Params base_params(dc_ctx *ctx, const DevBatch &b, int inst) {
    Params p{};
    p.t = ctx->t;
    p.st = state_of(ctx, inst);
    p.m = ctx->m;
    ahp_p1(ctx->m, p.p1);
    p.b = b.view;
    p.tr = Trace{ctx->d_tmeta, ctx->d_tscore, ctx->d_tcount, ctx->cfg.trace_stride, ctx->cfg.trace_cap};
    p.xs = ctx->d_xs + (size_t)inst * xs_rows(ctx->m.nc) * ctx->N;
    p.pc_cap = ctx->pc_plain;
    p.inst = inst;
    p.state_base = ctx->d_state;
    p.state_stride = 6LL * ctx->N;
    p.colpart = ctx->d_colpart;
    p.rowpart = ctx->d_rowpart;
    p.ysort = ctx->d_ysort;
    p.wsort = ctx->d_wsort;
    p.ti = ctx->ti; p.tj = ctx->tj; p.nI = ctx->nI; p.nJ = ctx->nJ;
    return p;
}

// Output region of a batch: host[Ct], code[Pt], failat[R] (all -1), then
// status[R] (1), then score[Ct], tsb[R], tse[R] (0; the stamps are int64).
int reset_outputs(dc_ctx *ctx, DevBatch &b) {
    int *out = b.dmem + b.in_ints;
    const long long neg = (long long)b.Ct + b.Pt + b.R;
    hipLaunchKernelGGL(k_fill_i32, dim3(64), dim3(256), 0, ctx->stream, out, -1, neg);
    hipLaunchKernelGGL(k_fill_i32, dim3(16), dim3(256), 0, ctx->stream, out + neg, 1, (long long)b.R);
    hipLaunchKernelGGL(k_fill_i32, dim3(64), dim3(256), 0, ctx->stream, out + neg + b.R, 0,
                       (long long)b.out_ints - neg - b.R);
    HIPCHK(hipGetLastError());
    return DC_OK;
}

// Turn the pending queue into one uploaded batch (requests grouped by
// instance, FCFS order kept within an instance).
int upload_pending(dc_ctx *ctx) {
    const size_t R = ctx->pend_ids.size();
    if (R == 0) return DC_OK;
    auto B = std::make_unique<DevBatch>();
    DevBatch &b = *B;
    b.R = (int)R;
    b.I = ctx->I;
    std::vector<int> order(R);
    for (size_t r = 0; r < R; ++r) order[r] = (int)r;
    std::stable_sort(order.begin(), order.end(),
                     [&](int a, int c) { return ctx->pend_inst[a] < ctx->pend_inst[c]; });
    b.coff.assign(1, 0);
    b.poff.assign(1, 0);
    b.iroff.assign(ctx->I + 1, 0);
    b.cuoff.assign(1, 0);
    for (int idx : order) {
        const Units &U = ctx->pend_units[idx];
        b.ids.push_back(ctx->pend_ids[idx]);
        b.inst.push_back(ctx->pend_inst[idx]);
        b.iroff[ctx->pend_inst[idx] + 1]++;
        const int pbase = (int)b.pj.size();
        for (int g = 0; g < U.nu(); ++g) {
            b.cpu.push_back(U.cpu[g]);
            b.ram.push_back(U.ram[g]);
            b.cmax.push_back(U.cmax[g]);
            b.rmax.push_back(U.rmax[g]);
            b.first.push_back(U.first[g]);
            b.poff.push_back(pbase + U.poff[g + 1]);
        }
        b.pj.insert(b.pj.end(), U.pj.begin(), U.pj.end());
        b.pbw.insert(b.pbw.end(), U.pbw.begin(), U.pbw.end());
        b.pbmax.insert(b.pbmax.end(), U.pbmax.begin(), U.pbmax.end());
        b.mem.push_back(std::move(ctx->pend_units[idx].mem));
        b.coff.push_back((int)b.cpu.size());
        b.cnt.push_back(U.n);
        b.unit_of.insert(b.unit_of.end(), U.unit_of.begin(), U.unit_of.end());
        b.cuoff.push_back((int)b.unit_of.size());
    }
    for (int i = 0; i < ctx->I; ++i) b.iroff[i + 1] += b.iroff[i];
    b.Ct = (int)b.cpu.size();
    b.Pt = (int)b.pj.size();
    // device layout: inputs coff, cpu, ram, poff, pj, pbw, iroff, rid, cmax,
    // rmax, pbmax; outputs host, code, failat, status, score, stamps, then
    // the allocations cpua, rama, pbwa
    size_t n_in = (size_t)(b.R + 1) + 2 * b.Ct + (b.Ct + 1) + 2 * (size_t)b.Pt + (b.I + 1) + b.R + 2 * b.Ct + b.Pt;
    n_in += n_in & 1;   // keeps the int64 stamps in the output region 8-byte aligned
    b.o_alloc = (size_t)b.Ct + b.Pt + b.R + b.R + b.Ct + 1 + 4 * (size_t)b.R;
    const size_t n_out = b.o_alloc + 2 * (size_t)b.Ct + b.Pt;
    b.in_ints = n_in;
    b.out_ints = n_out;
    std::vector<int> img(n_in, 0);
    size_t o = 0;
    auto put = [&](const std::vector<int> &v) { std::memcpy(img.data() + o, v.data(), v.size() * sizeof(int)); o += v.size(); };
    const size_t o_coff = o; put(b.coff);
    const size_t o_cpu = o; put(b.cpu);
    const size_t o_ram = o; put(b.ram);
    const size_t o_poff = o; put(b.poff);
    const size_t o_pj = o; put(b.pj);
    const size_t o_pbw = o; put(b.pbw);
    const size_t o_iroff = o; put(b.iroff);
    std::vector<int> rid32(b.R);
    for (int r = 0; r < b.R; ++r) rid32[r] = (int)(b.ids[r] & 0x7fffffff);
    const size_t o_rid = o; put(rid32);
    const size_t o_cmax = o; put(b.cmax);
    const size_t o_rmax = o; put(b.rmax);
    const size_t o_pbmax = o; put(b.pbmax);
    HIPCHK(hipMalloc(&b.dmem, (n_in + n_out) * sizeof(int)));
    HIPCHK(hipMemcpyAsync(b.dmem, img.data(), n_in * sizeof(int), hipMemcpyHostToDevice, ctx->stream));
    int *d = b.dmem;
    int *out = d + n_in;
    b.view.coff = d + o_coff;
    b.view.cpu = d + o_cpu;
    b.view.ram = d + o_ram;
    b.view.poff = d + o_poff;
    b.view.pj = d + o_pj;
    b.view.pbw = d + o_pbw;
    b.view.iroff = d + o_iroff;
    b.view.rid = d + o_rid;
    b.view.cmax = d + o_cmax;
    b.view.rmax = d + o_rmax;
    b.view.pbmax = d + o_pbmax;
    b.view.cpua = out + b.o_alloc;
    b.view.rama = out + b.o_alloc + b.Ct;
    b.view.pbwa = out + b.o_alloc + 2 * b.Ct;
    b.view.host = out;
    b.view.code = out + b.Ct;
    b.view.failat = out + b.Ct + b.Pt;
    b.view.status = out + b.Ct + b.Pt + b.R;
    b.view.score = reinterpret_cast<float *>(out + b.Ct + b.Pt + 2 * b.R);
    {
        size_t o_ts = (size_t)b.Ct + b.Pt + 2 * b.R + b.Ct;
        o_ts += o_ts & 1;   // n_in is even, so this makes the stamps 8-byte aligned
        b.view.tsb = reinterpret_cast<long long *>(out + o_ts);
        b.view.tse = b.view.tsb + b.R;
    }
    int rc = reset_outputs(ctx, b);
    if (rc) return rc;
    HIPCHK(hipStreamSynchronize(ctx->stream));   // img is pageable host memory
    const int bi = (int)ctx->batches.size();
    for (int r = 0; r < b.R; ++r) ctx->loc[b.ids[r]] = ReqLoc{bi, r, false};
    ctx->batches.push_back(std::move(B));
    ctx->queued.push_back(bi);
    ctx->pend_ids.clear(); ctx->pend_inst.clear(); ctx->pend_units.clear();
    return DC_OK;
}

// The large AHP case: k = K with CPU, RAM, uplink, path bandwidth and hops
// (a cost), the list the CS = 5 kernels are compiled for.
bool specialised_ahp5(const dc_ctx *ctx, int K) {
    static const int crit[5] = {DC_CRIT_CPU, DC_CRIT_RAM, DC_CRIT_UPLINK, DC_CRIT_PATHBW, DC_CRIT_HOPS};
    if (ctx->t.k != K || ctx->m.method != DC_AHP || ctx->m.nc != 5) return false;
    for (int c = 0; c < 5; ++c)
        if (ctx->m.crit[c] != crit[c] || ctx->m.cost[c] != (c == 4)) return false;
    return true;
}

// Whether the context runs k = K fat-trees on the four default criteria
// (CPU, RAM, active, path bandwidth; all benefits, TOPSIS), for which
// kernels are also compiled with these as compile-time constants.
bool specialised(const dc_ctx *ctx, int K) {
    if (ctx->t.k != K || ctx->m.method != DC_TOPSIS || ctx->m.nc != 4) return false;
    for (int c = 0; c < 4; ++c)
        if (ctx->m.crit[c] != c || ctx->m.cost[c] != 0) return false;
    return true;
}

// The cooperative kernels compiled for k = 48 (the large data center of the
// serving form) on the default criteria, or for any case.
constexpr int kGridK = 48;
const void *grid_step_kernel(const dc_ctx *ctx) {
    return specialised(ctx, kGridK) ? reinterpret_cast<const void *>(k_topsis_grid<kGridBlock, kGridK>)
                                    : reinterpret_cast<const void *>(k_topsis_grid<kGridBlock, 0>);
}
const void *grid_serve_kernel(const dc_ctx *ctx) {
    return specialised(ctx, kGridK) ? reinterpret_cast<const void *>(k_serve_grid<kGridBlock, kGridK>)
                                    : reinterpret_cast<const void *>(k_serve_grid<kGridBlock, 0>);
}

// The plain kernel (state staged in LDS, 1,024 threads) compiled for k = 16
// on the default criteria.
constexpr int kPlainK = 16;
// The AHP criteria kernel compiled for k = 32 (8,192 servers) on five criteria.
constexpr int kAhpK = 32;

template <int BS>
void launch_plain_step(dc_ctx *ctx, const Params &p) {
    if (ctx->use_grid) {
        Params pp = p;
        GridCtl g = ctx->grid;
        long long timeout = ctx->grid_timeout;
        void *args[] = {&pp, &g, &timeout};
        const hipError_t e = hipLaunchCooperativeKernel(grid_step_kernel(ctx), dim3(ctx->t.k), dim3(kGridBlock), args,
                                                        ctx->lds_grid, ctx->stream);
        if (e != hipSuccess && ctx->launch_err == hipSuccess) ctx->launch_err = e;
        ctx->last_launches += 1;
        return;
    }
    if (ctx->m.method == DC_TOPSIS) {
        if (ctx->plain_res)
            if (BS == 1024 && specialised(ctx, kPlainK))
                hipLaunchKernelGGL((k_topsis_plain<1024, true, kPlainK>), dim3(1), dim3(1024), ctx->lds_plain,
                                   ctx->stream, p);
            else
                hipLaunchKernelGGL((k_topsis_plain<BS, true>), dim3(1), dim3(BS), ctx->lds_plain, ctx->stream, p);
        else
            hipLaunchKernelGGL((k_topsis_plain<BS, false>), dim3(1), dim3(BS), ctx->lds_plain, ctx->stream, p);
        ctx->last_launches += 1;
    } else {
        const int bx = (ctx->N + kAhpBlock - 1) / kAhpBlock;
        // criteria over several workgroups, each with G * BS servers at a time
        const int ncw = (ctx->N + host_group(BS) * BS - 1) / (host_group(BS) * BS);
        if (BS == 1024 && specialised_ahp5(ctx, kAhpK))
            hipLaunchKernelGGL((k_criteria_plain<1024, kAhpK, 5>), dim3(ncw), dim3(BS), ctx->lds_plain, ctx->stream,
                               p);
        else
            hipLaunchKernelGGL((k_criteria_plain<BS>), dim3(ncw), dim3(BS), ctx->lds_plain, ctx->stream, p);
        if (ctx->ahp_sorted) {
            Params q = p;
            q.nJ = 1;
            const dim3 gs(ctx->sort_runs, 1, ctx->m.nc), bs(kAhpSortBlock);
            hipLaunchKernelGGL(k_ahp_sort_runs, gs, bs, 0, ctx->stream, q, ctx->d_runs);
            if (ctx->sort_runs > 1) {
                hipLaunchKernelGGL(k_ahp_merge_runs, gs, bs, 0, ctx->stream, q, ctx->d_runs);
                ctx->last_launches += 1;
            }
            hipLaunchKernelGGL(k_ahp_sort_col, dim3(bx, 1, ctx->m.nc), dim3(kAhpBlock), 0, ctx->stream, q);
            hipLaunchKernelGGL(k_ahp_sort_row, dim3(bx, 1, ctx->m.nc), dim3(kAhpBlock), 0, ctx->stream, q);
            hipLaunchKernelGGL(k_ahp_pg, dim3(bx), dim3(kAhpBlock), 0, ctx->stream, q);
            hipLaunchKernelGGL((k_ahp_select<BS>), dim3(1), dim3(BS), ctx->lds_select, ctx->stream, q);
            ctx->last_launches += 6;
        } else {
            hipLaunchKernelGGL(k_ahp_colsum, dim3(bx, ctx->nI, ctx->m.nc), dim3(kAhpBlock), 0, ctx->stream, p);
            hipLaunchKernelGGL(k_ahp_rowsum, dim3(bx, ctx->nJ, ctx->m.nc), dim3(kAhpBlock), 0, ctx->stream, p);
            hipLaunchKernelGGL(k_ahp_pg, dim3(bx), dim3(kAhpBlock), 0, ctx->stream, p);
            hipLaunchKernelGGL((k_ahp_select<BS>), dim3(1), dim3(BS), ctx->lds_select, ctx->stream, p);
            ctx->last_launches += 5;
        }
    }
}

int run_plain(dc_ctx *ctx, DevBatch &b) {
    ctx->launch_err = hipSuccess;
    for (int r = 0; r < b.R; ++r) {
        Params p = base_params(ctx, b, b.inst[r]);
        const int g0 = b.coff[r], n = b.coff[r + 1] - g0;
        for (int i = 0; i < n; ++i) {
            const int g = g0 + i;
            p.s = StepIn{r, i, n, g0, g, b.poff[g], b.poff[g + 1] - b.poff[g], b.cpu[g], b.ram[g], b.cmax[g], b.rmax[g]};
            for (int q = 0; q < p.s.P; ++q) {
                p.pj[q] = b.pj[p.s.p0 + q];
                p.pbw[q] = b.pbw[p.s.p0 + q];
                p.pbmax[q] = b.pbmax[p.s.p0 + q];
            }
            switch (ctx->plain_bs) {
            case 64: launch_plain_step<64>(ctx, p); break;
            case 256: launch_plain_step<256>(ctx, p); break;
            case 512: launch_plain_step<512>(ctx, p); break;
            default: launch_plain_step<1024>(ctx, p); break;
            }
        }
        ctx->last_steps += n;
        HIPCHK(ctx->launch_err);
    }
    HIPCHK(hipGetLastError());
    return DC_OK;
}

size_t batched_lds(const dc_ctx *ctx, int pc) {
    return step_lds_bytes(pc, ctx->t.nsw, (size_t)xs_rows(ctx->m.nc) * ctx->N, 6 * (size_t)ctx->N + req_lds_ints());
}

// The batched kernel compiled for k = 16 fat-trees scored on the four
// default criteria (the constants fold into the kernel), or for any case.
constexpr int kBatchedK = 16;
bool batched_specialised(const dc_ctx *ctx) { return specialised(ctx, kBatchedK); }

template <int BS, int G>
void launch_batched_k(dc_ctx *ctx, const Params &p, size_t lds, hipStream_t stream) {
    if (batched_specialised(ctx))
        hipLaunchKernelGGL((k_topsis_batched<BS, G, kBatchedK>), dim3(ctx->I), dim3(BS), lds, stream, p);
    else
        hipLaunchKernelGGL((k_topsis_batched<BS, G, 0>), dim3(ctx->I), dim3(BS), lds, stream, p);
}

template <int BS, int G>
int set_lds_batched(dc_ctx *ctx, size_t lds) {
    return batched_specialised(ctx) ? set_lds(ctx, k_topsis_batched<BS, G, kBatchedK>, lds)
                                    : set_lds(ctx, k_topsis_batched<BS, G, 0>, lds);
}

// sh must be a built shape with 1 <= sh.pc <= ctx->pc_batched (callers check)
void launch_batched(dc_ctx *ctx, DevBatch &b, const Shape &sh, hipStream_t stream) {
    Params p = base_params(ctx, b, 0);
    p.pc_cap = sh.pc;
    const size_t lds = batched_lds(ctx, sh.pc);
    switch (sh.bs * 10 + sh.g) {
    case 2561: launch_batched_k<256, 1>(ctx, p, lds, stream); break;
    case 2562: launch_batched_k<256, 2>(ctx, p, lds, stream); break;
    case 2564: launch_batched_k<256, 4>(ctx, p, lds, stream); break;
    case 5121: launch_batched_k<512, 1>(ctx, p, lds, stream); break;
    case 5122: launch_batched_k<512, 2>(ctx, p, lds, stream); break;
    case 5124: launch_batched_k<512, 4>(ctx, p, lds, stream); break;
    case 10242: launch_batched_k<1024, 2>(ctx, p, lds, stream); break;
    default: launch_batched_k<1024, 1>(ctx, p, lds, stream); break;
    }
}

// Captures the batch's launch into a graph on a private stream (capture is
// not allowed on the legacy default stream a caller may have handed in).
int capture_batched(dc_ctx *ctx, DevBatch &b, const Shape &sh) {
    if (b.gexec) {
        HIPCHK(hipGraphExecDestroy(b.gexec));
        b.gexec = nullptr;
    }
    if (!ctx->cap_stream) HIPCHK(hipStreamCreateWithFlags(&ctx->cap_stream, hipStreamNonBlocking));
    hipGraph_t g = nullptr;
    HIPCHK(hipStreamBeginCapture(ctx->cap_stream, hipStreamCaptureModeThreadLocal));
    launch_batched(ctx, b, sh, ctx->cap_stream);
    const hipError_t le = hipGetLastError();
    const hipError_t ce = hipStreamEndCapture(ctx->cap_stream, &g);
    HIPCHK(le);
    HIPCHK(ce);
    const hipError_t ie = hipGraphInstantiate(&b.gexec, g, nullptr, nullptr, 0);
    (void)hipGraphDestroy(g);
    HIPCHK(ie);
    b.gshape = sh;
    return DC_OK;
}

int run_batched(dc_ctx *ctx, DevBatch &b, const Shape &sh) {
    if (ctx->cfg.graph == 1) {
        launch_batched(ctx, b, sh, ctx->stream);
    } else {
        if (!b.gexec || !(b.gshape == sh)) {
            const int rc = capture_batched(ctx, b, sh);
            if (rc) return rc;
        }
        HIPCHK(hipGraphLaunch(b.gexec, ctx->stream));
    }
    HIPCHK(hipGetLastError());
    ctx->last_launches += 1;
    ctx->last_steps += b.Ct;   // upper bound: containers queued (steps stop at a rejection)
    return DC_OK;
}

// Copies the outputs back through a pinned buffer: the servers, then
// everything after the route codes (failed_at, status, scores, timestamps).
// The route codes stay on the device; dc_get_paths fetches the few it needs.
int collect(dc_ctx *ctx, DevBatch &b) {
    const int *dout = b.dmem + b.in_ints;
    const size_t tail0 = (size_t)b.Ct + b.Pt, tail = b.o_alloc - tail0;   // the allocations stay on the device
    if (!b.pinned) HIPCHK(hipHostMalloc(reinterpret_cast<void **>(&b.pinned), (b.Ct + tail) * sizeof(int), 0));
    int *out = b.pinned;
    HIPCHK(hipMemcpyAsync(out, dout, (size_t)b.Ct * sizeof(int), hipMemcpyDeviceToHost, ctx->stream));
    HIPCHK(hipMemcpyAsync(out + b.Ct, dout + tail0, tail * sizeof(int), hipMemcpyDeviceToHost, ctx->stream));
    HIPCHK(hipStreamSynchronize(ctx->stream));
    const int *t0 = out + b.Ct;                        // output offset tail0 maps here
    b.host.assign(out, out + b.Ct);
    b.failat.assign(t0, t0 + b.R);
    b.status.assign(t0 + b.R, t0 + 2 * b.R);
    b.score.resize(b.Ct);
    std::memcpy(b.score.data(), t0 + 2 * b.R, sizeof(float) * b.Ct);
    b.tsb.resize(b.R);
    b.tse.resize(b.R);
    const long long *ts = b.view.tsb;
    const size_t o_ts = (size_t)(reinterpret_cast<const int *>(ts) - dout) - tail0;
    std::memcpy(b.tsb.data(), t0 + o_ts, sizeof(long long) * b.R);
    std::memcpy(b.tse.data(), t0 + o_ts + 2 * (size_t)b.R, sizeof(long long) * b.R);
    // results in request id order
    std::vector<int> order(b.R);
    for (int r = 0; r < b.R; ++r) order[r] = r;
    std::sort(order.begin(), order.end(), [&](int a, int c) { return b.ids[a] < b.ids[c]; });
    const size_t at = ctx->ready.size();
    ctx->ready.resize(at + order.size());
    for (size_t k = 0; k < order.size(); ++k) {
        const int r = order[k];
        dc_result &res = ctx->ready[at + k];
        const int g0 = b.coff[r], c0 = b.cuoff[r];
        res.req_id = b.ids[r];
        res.instance = b.inst[r];
        res.status = b.status[r];
        res.n = b.cnt[r];
        const int nu = b.coff[r + 1] - g0;       // failat == nu: the links did not fit
        res.failed_at = b.status[r] ? -1 : (b.failat[r] < nu ? b.first[g0 + b.failat[r]] : b.cnt[r]);
        // a container gets its pod's server and score; a rejected request
        // places nothing (its attempt stays readable through dc_get_attempt)
        for (int i = 0; i < res.n; ++i) {
            const int g = g0 + b.unit_of[c0 + i];
            res.host[i] = res.status ? b.host[g] : -1;
            res.score[i] = b.score[g];
        }
        std::fill(res.host + res.n, res.host + DC_MAX_CONTAINERS, -1);
        std::fill(res.score + res.n, res.score + DC_MAX_CONTAINERS, 0.f);
    }
    return DC_OK;
}

// ---------------------------------------------------------------- cooperative step
int grid_init(dc_ctx *ctx) {
    const int G = ctx->t.k, h = ctx->t.h;
    if (h > kRecCapP - kRecCapE || G > kWave) return DC_EINVAL;
    // count, gen, err, round, flag[kGridFlags], then 8-byte aligned: kslot[2][G], rflag, rec[G][kRecWords]
    const size_t ints = 4 + kGridFlags + 2 + 2 * (2 * (size_t)G + 1 + (size_t)G * kRecWords);
    HIPCHK(hipMalloc(&ctx->d_grid, ints * sizeof(int)));
    hipLaunchKernelGGL(k_fill_i32, dim3(16), dim3(256), 0, ctx->stream, ctx->d_grid, 0, (long long)ints);
    HIPCHK(hipGetLastError());
    int *p = ctx->d_grid;
    GridCtl &g = ctx->grid;
    g.count = reinterpret_cast<unsigned *>(p);
    g.gen = reinterpret_cast<unsigned *>(p + 1);
    g.err = p + 2;
    g.round = reinterpret_cast<unsigned *>(p + 3);
    g.flag = p + 4;
    int *k = g.flag + kGridFlags;
    k += (reinterpret_cast<uintptr_t>(k) & 7) ? 1 : 0;
    g.kslot = reinterpret_cast<unsigned long long *>(k);
    g.rflag = g.kslot + 2 * G;
    g.rec = g.rflag + 1;
    ctx->lds_grid = gsmem_bytes(h, ctx->t.hh, ctx->m.nc);
    const size_t serve_lds = align4(ctx->lds_grid / sizeof(int)) * sizeof(int) + req_lds_ints() * sizeof(int);
    if (serve_lds > 159 * 1024) return DC_EINVAL;
    if (hipFuncSetAttribute(grid_step_kernel(ctx), hipFuncAttributeMaxDynamicSharedMemorySize, (int)ctx->lds_grid) !=
            hipSuccess ||
        hipFuncSetAttribute(grid_serve_kernel(ctx), hipFuncAttributeMaxDynamicSharedMemorySize, (int)serve_lds) !=
            hipSuccess)
        return DC_EDEVICE;
    ctx->use_grid = true;
    return DC_OK;
}

// A cooperative step that timed out at a barrier poisons the context.
int grid_check(dc_ctx *ctx) {
    if (!ctx->use_grid) return DC_OK;
    int err = 0;
    HIPCHK(hipMemcpy(&err, ctx->grid.err, sizeof(int), hipMemcpyDeviceToHost));
    if (err) {
        ctx->poisoned = true;
        std::fprintf(stderr, "libdcsched: a cooperative step timed out at a grid barrier\n");
        return DC_EDEVICE;
    }
    return DC_OK;
}

// ---------------------------------------------------------------- serving form
int serve_init(dc_ctx *ctx) {
    auto sv = std::make_unique<Serve>();
    const size_t budget = ctx->cfg.mem_budget ? ctx->cfg.mem_budget : (size_t)256 << 20;
    sv->arena_ints = budget / sizeof(int);
    sv->stage_ints = slot_layout(kMaxN, kMaxPairs).in_end;
    const unsigned fl = hipHostMallocCoherent | hipHostMallocMapped;
    HIPCHK(hipHostMalloc(reinterpret_cast<void **>(&sv->cmds), sizeof(Cmd) * sv->cap, fl));
    HIPCHK(hipHostMalloc(reinterpret_cast<void **>(&sv->comps), sizeof(Comp) * sv->cap, fl));
    HIPCHK(hipHostMalloc(reinterpret_cast<void **>(&sv->ctrl), sizeof(int) * 4, fl));
    HIPCHK(hipHostMalloc(reinterpret_cast<void **>(&sv->staging), sizeof(int) * (size_t)sv->stage_ints * sv->cap, fl));
    std::memset(sv->cmds, 0, sizeof(Cmd) * sv->cap);
    std::memset(sv->comps, 0, sizeof(Comp) * sv->cap);
    std::memset(sv->ctrl, 0, sizeof(int) * 4);
    HIPCHK(hipMalloc(&sv->arena, sv->arena_ints * sizeof(int)));
    sv->free_list[0] = sv->arena_ints & ~size_t(3);
    HIPCHK(hipStreamCreateWithFlags(&sv->aux, hipStreamNonBlocking));
    sv->bs = ctx->N <= 256 ? 256 : 512;
    const size_t lds_max = 159 * 1024;   // 160 KiB of LDS, 1 KiB left for static shared memory
    const size_t base = step_lds_bytes(0, ctx->t.nsw, req_lds_ints(), 0);
    sv->pc = (int)std::max<size_t>(1, std::min<size_t>(kMaxN, (lds_max - base) / (8 * (size_t)ctx->t.nsw)));
    sv->lds = step_lds_bytes(sv->pc, ctx->t.nsw, req_lds_ints(), 0);
    if (sv->lds > lds_max) return DC_EINVAL;
    if (set_lds(ctx, k_serve<256>, sv->lds) || set_lds(ctx, k_serve<512>, sv->lds)) return DC_EDEVICE;
    ctx->sv = std::move(sv);
    return DC_OK;
}

// (Re)launches the persistent kernel when commands wait and none runs.
int serve_ensure_running(dc_ctx *ctx) {
    Serve &sv = *ctx->sv;
    const int dev_pos = __atomic_load_n(sv.ctrl, __ATOMIC_ACQUIRE);
    if (dev_pos >= sv.host_pos) return DC_OK;
    if (sv.launched) {
        const hipError_t q = hipStreamQuery(ctx->stream);
        if (q == hipErrorNotReady) return DC_OK;      // still running: it will reach the command
        HIPCHK(q);
    }
    Params p{};
    p.t = ctx->t;
    p.st = state_of(ctx, 0);
    p.m = ctx->m;
    p.tr = Trace{nullptr, nullptr, nullptr, 0, 0};
    p.xs = ctx->d_xs;
    p.pc_cap = sv.pc;
    ServeArgs a{sv.cmds, sv.comps, sv.ctrl, sv.staging, sv.arena, sv.cap, sv.stage_ints, dev_pos, 0, sv.idle_ticks};
    __atomic_store_n(sv.ctrl + 1, 0, __ATOMIC_RELEASE);
    if (ctx->use_grid) {
        GridCtl g = ctx->grid;
        long long timeout = ctx->grid_timeout;
        void *args[] = {&p, &a, &g, &timeout};
        const size_t lds = align4(ctx->lds_grid / sizeof(int)) * sizeof(int) + req_lds_ints() * sizeof(int);
        HIPCHK(hipLaunchCooperativeKernel(grid_serve_kernel(ctx), dim3(ctx->t.k), dim3(kGridBlock), args, lds,
                                          ctx->stream));
    } else if (sv.bs == 256) {
        hipLaunchKernelGGL((k_serve<256>), dim3(1), dim3(256), sv.lds, ctx->stream, p, a);
    } else {
        hipLaunchKernelGGL((k_serve<512>), dim3(1), dim3(512), sv.lds, ctx->stream, p, a);
    }
    HIPCHK(hipGetLastError());
    sv.launched = true;
    return DC_OK;
}

// Publishes one command; the caller has checked ring space.
void serve_publish(Serve &sv, int type, int n, int P, size_t off, int rid) {
    Cmd &c = sv.cmds[sv.host_pos % sv.cap];
    c.type = type;
    c.n = n;
    c.npair = P;
    c.slot_off = (int)off;
    c.rid = rid;
    __atomic_store_n(&c.seq, (int)(sv.host_pos + 1), __ATOMIC_RELEASE);
    ++sv.host_pos;
}

int serve_poll(dc_ctx *ctx) {
    Serve &sv = *ctx->sv;
    if (ctx->use_grid && sv.launched && hipStreamQuery(ctx->stream) == hipSuccess) {
        int rc = grid_check(ctx);
        if (rc) return rc;
    }
    while (sv.comp_pos < sv.host_pos) {
        Comp &c = sv.comps[sv.comp_pos % sv.cap];
        if (__atomic_load_n(&c.seq, __ATOMIC_ACQUIRE) != (int)(sv.comp_pos + 1)) break;
        auto rit = sv.rid_to_id.find(c.rid);
        if (rit != sv.rid_to_id.end()) {
            const int64_t id = rit->second;
            ServeSlot &sl = sv.slots[id];
            if (c.type == CMD_SUBMIT) {
                sl.status = c.status;
                sl.hosts.resize(sl.nc);
                dc_result res;
                std::memset(&res, 0, sizeof res);
                res.req_id = id;
                res.instance = 0;
                res.status = c.status;
                res.n = sl.nc;
                res.failed_at = c.status ? -1 : (c.failat < sl.n ? sl.first[c.failat] : sl.nc);
                for (int i = 0; i < DC_MAX_CONTAINERS; ++i) res.host[i] = -1;
                for (int i = 0; i < sl.nc; ++i) {           // each container takes its pod's result
                    const int g = sl.unit_of[i];
                    sl.hosts[i] = c.host[g];
                    res.host[i] = c.status ? c.host[g] : -1;
                    res.score[i] = c.score[g];
                }
                ctx->ready.push_back(res);
                sv.service_us.emplace_back(id, (float)((c.t_decide - c.t_admit) / 100.0));
                if (!c.status) serve_free(sv, sl.off, sl.ints);   // rejected: nothing left to release
            } else {
                serve_free(sv, sl.off, sl.ints);                   // departure done
            }
        }
        ++sv.comp_pos;
    }
    return serve_ensure_running(ctx);
}

int serve_submit(dc_ctx *ctx, Units &U, int64_t *req_id) {
    Serve &sv = *ctx->sv;
    int rc = serve_poll(ctx);
    if (rc) return rc;
    const int n = U.nu();
    const std::vector<int> &poff = U.poff, &pj = U.pj, &pbw = U.pbw;
    const int *cpu = U.cpu.data(), *ram = U.ram.data();
    const int P = (int)pj.size();
    const SlotLayout L = slot_layout(n, P);
    if (sv.host_pos - sv.comp_pos >= sv.cap) return DC_EAGAIN;
    size_t off = 0;
    if (!serve_alloc(sv, (size_t)L.total, &off)) return DC_EAGAIN;
    const int64_t id = ctx->next_id++;
    const int rid = (int)(id & 0x7fffffff);
    int *stg = sv.staging + (size_t)(sv.host_pos % sv.cap) * sv.stage_ints;
    stg[L.coff] = 0;
    stg[L.coff + 1] = n;
    std::memcpy(stg + L.cpu, cpu, sizeof(int) * n);
    std::memcpy(stg + L.ram, ram, sizeof(int) * n);
    std::memcpy(stg + L.poff, poff.data(), sizeof(int) * (n + 1));
    std::memcpy(stg + L.cmax, U.cmax.data(), sizeof(int) * n);
    std::memcpy(stg + L.rmax, U.rmax.data(), sizeof(int) * n);
    if (P) {
        std::memcpy(stg + L.pj, pj.data(), sizeof(int) * P);
        std::memcpy(stg + L.pbw, pbw.data(), sizeof(int) * P);
        std::memcpy(stg + L.pbmax, U.pbmax.data(), sizeof(int) * P);
    }
    stg[L.rid] = rid;
    ServeSlot sl;
    sl.off = off;
    sl.ints = (size_t)L.total;
    sl.n = n;
    sl.P = P;
    sl.nc = U.n;
    sl.unit_of = std::move(U.unit_of);
    sl.first = std::move(U.first);
    sl.mem = std::move(U.mem);
    sv.slots[id] = std::move(sl);
    sv.rid_to_id[rid] = id;
    serve_publish(sv, CMD_SUBMIT, n, P, off, rid);
    if (req_id) *req_id = id;
    return serve_ensure_running(ctx);
}

int serve_release(dc_ctx *ctx, int64_t req_id) {
    Serve &sv = *ctx->sv;
    int rc = serve_poll(ctx);
    if (rc) return rc;
    auto it = sv.slots.find(req_id);
    if (it == sv.slots.end() || it->second.released) return DC_ENOENT;
    ServeSlot &sl = it->second;
    if (sl.status < 0) return DC_EAGAIN;          // not decided yet
    if (sl.status == 0) return DC_ENOENT;         // rejected: holds nothing
    if (sv.host_pos - sv.comp_pos >= sv.cap) return DC_EAGAIN;
    sl.released = true;
    serve_publish(sv, CMD_RELEASE, sl.n, sl.P, sl.off, (int)(req_id & 0x7fffffff));
    return serve_ensure_running(ctx);
}

// Stops the persistent kernel: publishes STOP and waits (bounded) for it.
int serve_stop(dc_ctx *ctx) {
    Serve &sv = *ctx->sv;
    if (!sv.launched) return DC_OK;
    const auto t0 = std::chrono::steady_clock::now();
    while (sv.host_pos - sv.comp_pos >= sv.cap) {
        int rc = serve_poll(ctx);
        if (rc) return rc;
        if (std::chrono::steady_clock::now() - t0 > std::chrono::seconds(60)) return DC_EDEVICE;
    }
    if (hipStreamQuery(ctx->stream) == hipErrorNotReady) serve_publish(sv, CMD_STOP, 0, 0, 0, -1);
    while (hipStreamQuery(ctx->stream) == hipErrorNotReady) {
        std::this_thread::sleep_for(std::chrono::microseconds(100));
        if (std::chrono::steady_clock::now() - t0 > std::chrono::seconds(60)) return DC_EDEVICE;
    }
    sv.launched = false;
    return DC_OK;
}

}  // namespace

namespace {

// A shape the current context can launch: a built (threads, servers per
// thread) pair and a peer chunk its LDS holds (batched form), or a plain
// workgroup size with its fixed grouping and chunk.
bool shape_ok(const dc_ctx *ctx, const Shape &sh) {
    if (ctx->cfg.mode == DC_MODE_BATCHED)
        return batched_shape_built(sh.bs, sh.g) && sh.pc >= 1 && sh.pc <= ctx->pc_batched;
    return (sh.bs == 64 || sh.bs == 256 || sh.bs == 512 || sh.bs == 1024) && sh.g == host_group(sh.bs) &&
           sh.pc == ctx->pc_plain;
}

// Cache key of a tuned shape: device architecture, form, method, servers,
// criteria.
std::string tune_key(const dc_ctx *ctx) {
    std::string arch = "unknown";
    int dev = 0;
    hipDeviceProp_t prop{};
    if (hipGetDevice(&dev) == hipSuccess && hipGetDeviceProperties(&prop, dev) == hipSuccess) {
        arch = prop.gcnArchName;
        const size_t colon = arch.find(':');
        if (colon != std::string::npos) arch.resize(colon);
    }
    const char *mode = ctx->cfg.mode == DC_MODE_BATCHED ? "batched" : "plain";
    const char *method = ctx->cfg.method == DC_AHP ? "ahp" : "topsis";
    return arch + "|" + mode + "|" + method + "|N=" + std::to_string(ctx->N) + "|C=" + std::to_string(ctx->m.nc);
}

// The cache is a text file of JSON objects, one per line:
// {"key": "...", "block": B, "host_group": G, "peer_chunk": P, "ms": T}
bool field_int(const std::string &line, const char *name, int *v) {
    const std::string pat = std::string("\"") + name + "\": ";
    const size_t at = line.find(pat);
    return at != std::string::npos && std::sscanf(line.c_str() + at + pat.size(), "%d", v) == 1;
}

std::string line_key(const std::string &line) {
    const std::string pat = "\"key\": \"";
    const size_t at = line.find(pat);
    if (at == std::string::npos) return std::string();
    const size_t end = line.find('"', at + pat.size());
    return end == std::string::npos ? std::string() : line.substr(at + pat.size(), end - at - pat.size());
}

bool cache_read(const char *path, const std::string &key, Shape *sh, float *ms) {
    std::ifstream in(path);
    std::string line;
    while (std::getline(in, line)) {
        if (line_key(line) != key) continue;
        int bs = 0, g = 0, pc = 0;
        if (!field_int(line, "block", &bs) || !field_int(line, "host_group", &g) || !field_int(line, "peer_chunk", &pc))
            return false;
        const size_t at = line.find("\"ms\": ");
        *ms = at == std::string::npos ? 0.f : std::strtof(line.c_str() + at + 6, nullptr);
        *sh = Shape{bs, g, pc};
        return true;
    }
    return false;
}

// Replaces (or adds) the key's line; written to a temporary file and renamed
// into place.  A cache that cannot be written is left as it was.
void cache_write(const char *path, const std::string &key, const Shape &sh, float ms) {
    std::vector<std::string> lines;
    {
        std::ifstream in(path);
        std::string line;
        while (std::getline(in, line))
            if (!line.empty() && line_key(line) != key) lines.push_back(line);
    }
    char buf[512];
    std::snprintf(buf, sizeof(buf), "{\"key\": \"%s\", \"block\": %d, \"host_group\": %d, \"peer_chunk\": %d, \"ms\": %.4f}",
                  key.c_str(), sh.bs, sh.g, sh.pc, ms);
    lines.push_back(buf);
    const std::string tmp = std::string(path) + ".tmp";
    {
        std::ofstream o(tmp, std::ios::trunc);
        if (!o) return;
        for (const auto &l : lines) o << l << "\n";
        if (!o) return;
    }
    (void)std::rename(tmp.c_str(), path);
}

}  // namespace

namespace {

// Which kernels score a set of tiles: one wavefront per tile (matrices a
// wavefront's registers hold), slices of one tile over several workgroups
// with partials in scratch (few large tiles), or one workgroup per tile.
enum { TILE_WAVE = 0, TILE_SPLIT = 1, TILE_GEN = 2 };
struct TilePath {
    int kind = TILE_GEN, C = 0, V = 0;
};

int tiles_prepare(int64_t T, int32_t C, int32_t N, const int32_t *x, const uint8_t *feasible, const int32_t *cost,
                  const float *weight, float *scores, int32_t *best, float *best_score, TileArgs *a, TilePath *path) {
    if (T < 0 || T > 0x7fffffffLL || C < 1 || C > DC_MAX_CRIT || N < 1 || N > (1 << 20)) return DC_EINVAL;
    if (T == 0) return DC_OK;
    if (!x || !best || !weight) return DC_EINVAL;
    *a = TileArgs{};
    a->x = x;
    a->feas = feasible;
    a->scores = scores;
    a->best = best;
    a->best_score = best_score;
    a->C = C;
    a->N = N;
    for (int c = 0; c < C; ++c) {
        if (!(weight[c] > 0.f) || !std::isfinite(weight[c])) return DC_EINVAL;
        a->w[c] = weight[c];
        a->cost[c] = cost ? (cost[c] != 0) : 0;
    }
    auto al = [](const void *p, uintptr_t m) { return (reinterpret_cast<uintptr_t>(p) & (m - 1)) == 0; };
    const bool vec = N % 4 == 0 && al(x, 16) && (!scores || al(scores, 16)) && (!feasible || al(feasible, 4));
    // four-server groups per lane when one wavefront holds the tile
    const int V = (N + 4 * kWave - 1) / (4 * kWave);
    const int Vp = V <= 1 ? 1 : V <= 2 ? 2 : V <= 4 ? 4 : V <= 8 ? 8 : 16;   // 16: too large
    path->C = C;
    path->V = Vp;
    if (vec && Vp <= 8 && C * Vp <= 16) path->kind = TILE_WAVE;
    else if (N >= 2 * kSplitSlice && T <= kSplitMaxTiles) path->kind = TILE_SPLIT;
    else path->kind = TILE_GEN;
    return DC_OK;
}

// work: split_scratch_bytes(T, N, C) device bytes for the split path
// (unused otherwise).
int tiles_launch(const TileArgs &a, int64_t T, const TilePath &path, void *work, hipStream_t st) {
    if (path.kind == TILE_WAVE) {
        // persistent grid: as many workgroups as fit on the device at once,
        // never more than needed for one wavefront per tile
        int dev = 0, cus = 0;
        if (hipGetDevice(&dev) != hipSuccess ||
            hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess)
            return DC_EDEVICE;
        const dim3 block(kTileBlock);
        auto pgrid = [&](const void *k) {
            int per = 0;
            if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per, k, kTileBlock, 0) != hipSuccess || per < 1) per = 1;
            const long long need = (T + kTileWaves - 1) / kTileWaves;
            return dim3(static_cast<unsigned>(std::min<long long>(need, (long long)per * cus)));
        };
#define DCS_TILES_LAUNCH(CC, VV)                                                                         \
    hipLaunchKernelGGL((k_topsis_tiles_wave<CC, VV>),                                                    \
                       pgrid(reinterpret_cast<const void *>(k_topsis_tiles_wave<CC, VV>)), block, 0, st, a, (long long)T)
        switch (path.C * 100 + path.V) {
        case 101: DCS_TILES_LAUNCH(1, 1); break;
        case 102: DCS_TILES_LAUNCH(1, 2); break;
        case 104: DCS_TILES_LAUNCH(1, 4); break;
        case 108: DCS_TILES_LAUNCH(1, 8); break;
        case 201: DCS_TILES_LAUNCH(2, 1); break;
        case 202: DCS_TILES_LAUNCH(2, 2); break;
        case 204: DCS_TILES_LAUNCH(2, 4); break;
        case 208: DCS_TILES_LAUNCH(2, 8); break;
        case 301: DCS_TILES_LAUNCH(3, 1); break;
        case 302: DCS_TILES_LAUNCH(3, 2); break;
        case 304: DCS_TILES_LAUNCH(3, 4); break;
        case 401: DCS_TILES_LAUNCH(4, 1); break;
        case 402: DCS_TILES_LAUNCH(4, 2); break;
        case 404: DCS_TILES_LAUNCH(4, 4); break;
        case 501: DCS_TILES_LAUNCH(5, 1); break;
        case 502: DCS_TILES_LAUNCH(5, 2); break;
        case 601: DCS_TILES_LAUNCH(6, 1); break;
        case 602: DCS_TILES_LAUNCH(6, 2); break;
        case 701: DCS_TILES_LAUNCH(7, 1); break;
        case 702: DCS_TILES_LAUNCH(7, 2); break;
        case 801: DCS_TILES_LAUNCH(8, 1); break;
        case 802: DCS_TILES_LAUNCH(8, 2); break;
        default: return DC_EINVAL;          // unreachable: V <= 8, C * V <= 16
        }
#undef DCS_TILES_LAUNCH
    } else if (path.kind == TILE_SPLIT) {
        const TileSplit sp = split_carve(work, T, a.N, a.C);
        const dim3 grid(static_cast<unsigned>(sp.S), static_cast<unsigned>(T));
        hipLaunchKernelGGL(k_tiles_split_stats, grid, dim3(kTileBlock), 0, st, a, sp);
        hipLaunchKernelGGL(k_tiles_split_score, grid, dim3(kTileBlock), 0, st, a, sp);
        hipLaunchKernelGGL(k_tiles_split_select, dim3(static_cast<unsigned>(T)), dim3(kWave), 0, st, a, sp);
    } else {
        hipLaunchKernelGGL(k_topsis_tiles_gen, dim3(static_cast<unsigned>(T)), dim3(kTileBlock), 0, st, a);
    }
    if (hipGetLastError() != hipSuccess) return DC_EDEVICE;
    return DC_OK;
}

// Scratch of dc_topsis_tiles_noalloc: the split path's partials in a
// static device array, one copy per device, held until the process ends.
// Host code never passes the array's name to a kernel (on the host it is a
// stand-in, not a device address): the address comes from
// hipGetSymbolAddress, resolved once per device with that device current.
constexpr size_t kStaticScratchBytes = DC_STATIC_SCRATCH_BYTES;
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void *g_scratch_addr[kMaxDevices] = {};

}  // namespace

static __device__ __align__(256) unsigned char scratch[kStaticScratchBytes];

namespace {

// Device address of the current device's copy of `scratch`.
int static_scratch(void **out) {
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= kMaxDevices) return DC_EDEVICE;
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_addr[dev]) {
        void *p = nullptr;
        if (hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) != hipSuccess || !p) return DC_EDEVICE;
        g_scratch_addr[dev] = p;
    }
    *out = g_scratch_addr[dev];
    return DC_OK;
}

}  // namespace

extern "C" {

const char *dc_strerror(int code) {
    switch (code) {
    case DC_OK: return "ok";
    case DC_EINVAL: return "invalid argument";
    case DC_ENOMEM: return "out of memory";
    case DC_EAGAIN: return "memory budget full, retry later";
    case DC_ENOENT: return "unknown or not accepted request";
    case DC_EDEVICE: return "device error (context poisoned)";
    case DC_ESTATE: return "call not valid in this mode or state";
    case DC_ETOOBIG: return "needs more scratch than the static buffer holds";
    default: return "unknown error";
    }
}

int dc_create(const dc_config *cfg, dc_ctx **out) {
    if (!out) return DC_EINVAL;
    *out = nullptr;
    int rc = check_config(cfg);
    if (rc) return rc;
    const int k = cfg->k, h = k / 2, N = k * k * k / 4, I = cfg->n_instances;
    // background load must stay within capacity
    if (cfg->host_used)
        for (long long x = 0; x < (long long)I * 2 * N; ++x) {
            const int cap = ((x / N) % 2) ? cfg->host_ram : cfg->host_cpu;
            if (cfg->host_used[x] < 0 || cfg->host_used[x] > cap) return DC_EINVAL;
        }
    if (cfg->link_used)
        for (long long x = 0; x < (long long)I * 3 * N; ++x) {
            const int lvl = (int)((x / N) % 3);
            const int cap = lvl == 0 ? cfg->bw_host_edge : lvl == 1 ? cfg->bw_edge_agg : cfg->bw_agg_core;
            if (cfg->link_used[x] < 0 || cfg->link_used[x] > cap) return DC_EINVAL;
        }
    auto ctx = std::make_unique<dc_ctx>();
    ctx->cfg = *cfg;
    ctx->cfg.host_used = nullptr;
    ctx->cfg.link_used = nullptr;
    ctx->t = Topo{k, h, h * h, N, k * k / 2, 1.0f / h, 1.0f / (h * h), 1.0f / (k * k / 2)};
    ctx->N = N;
    ctx->I = I;
    ctx->m.method = cfg->method;
    ctx->m.scale = cfg->ahp_scale;
    ctx->m.nc = cfg->ncrit;
    ctx->m.route_end = cfg->routing;
    for (int c = 0; c < DC_MAX_CRIT; ++c) {
        ctx->m.crit[c] = c < cfg->ncrit ? cfg->crit[c] : 0;
        ctx->m.cost[c] = c < cfg->ncrit ? (cfg->crit_cost[c] != 0) : 0;
        ctx->m.w[c] = c < cfg->ncrit ? cfg->weight[c] : 0.f;
    }
    dc_ctx *c = ctx.get();
    if (cfg->stream) {
        c->stream = static_cast<hipStream_t>(cfg->stream);
    } else {
        if (hipStreamCreateWithFlags(&c->stream, hipStreamNonBlocking) != hipSuccess) return DC_EDEVICE;
        c->own_stream = true;
    }
    // initial state
    std::vector<int> init((size_t)I * 6 * N);
    for (int i = 0; i < I; ++i) {
        int *s = init.data() + (size_t)i * 6 * N;
        for (int u = 0; u < N; ++u) {
            s[u] = cfg->host_cpu - (cfg->host_used ? cfg->host_used[((size_t)i * 2) * N + u] : 0);
            s[N + u] = cfg->host_ram - (cfg->host_used ? cfg->host_used[((size_t)i * 2 + 1) * N + u] : 0);
            s[2 * N + u] = 0;
            const int caps[3] = {cfg->bw_host_edge, cfg->bw_edge_agg, cfg->bw_agg_core};
            for (int l = 0; l < 3; ++l)
                s[(3 + l) * N + u] = caps[l] - (cfg->link_used ? cfg->link_used[((size_t)i * 3 + l) * N + u] : 0);
        }
    }
    const size_t sbytes = init.size() * sizeof(int);
    if (hipMalloc(&c->d_state, sbytes) != hipSuccess || hipMalloc(&c->d_init, sbytes) != hipSuccess) {
        dc_destroy(ctx.release());
        return DC_ENOMEM;
    }
    if (hipMemcpy(c->d_init, init.data(), sbytes, hipMemcpyHostToDevice) != hipSuccess ||
        hipMemcpy(c->d_state, init.data(), sbytes, hipMemcpyHostToDevice) != hipSuccess) {
        c->poisoned = true;
        dc_destroy(ctx.release());
        return DC_EDEVICE;
    }
    const int nc = cfg->ncrit;
    if (hipMalloc(&c->d_xs, (size_t)I * xs_rows(nc) * N * sizeof(int)) != hipSuccess) {
        dc_destroy(ctx.release());
        return DC_ENOMEM;
    }
    // launch shapes
    c->plain_bs = cfg->block ? cfg->block : (N <= 64 ? 64 : N <= 256 ? 256 : 1024);
    c->bshape.bs = cfg->block ? std::max(256, cfg->block) : 1024;
    c->bshape.g = c->bshape.bs >= 1024 ? 1 : host_group(c->bshape.bs);
    const size_t lds_max = 159 * 1024;   // 160 KiB of LDS, 1 KiB left for static shared memory
    {
        // plain: state + scratch in LDS when they fit with at least 8 peer tables
        const size_t res_fixed = step_lds_bytes(0, c->t.nsw, (size_t)xs_rows(nc) * N, 6 * (size_t)N);
        const size_t per_peer = 8 * (size_t)c->t.nsw;
        c->plain_res = res_fixed + 8 * per_peer <= lds_max;
        if (c->plain_res) {
            c->pc_plain = (int)std::min<size_t>(kMaxN, (lds_max - res_fixed) / per_peer);
            c->lds_plain = step_lds_bytes(c->pc_plain, c->t.nsw, (size_t)xs_rows(nc) * N, 6 * (size_t)N);
        } else {
            c->pc_plain = (int)std::max<size_t>(1, std::min<size_t>(kMaxN, 64 * 1024 / per_peer));
            c->lds_plain = step_lds_bytes(c->pc_plain, c->t.nsw, 0, 0);
        }
    }
    c->lds_select = step_lds_bytes(0, c->t.nsw, 0, 0);
    if (cfg->mode == DC_MODE_BATCHED) {
        const size_t fixed = step_lds_bytes(0, c->t.nsw, (size_t)xs_rows(nc) * N, 6 * (size_t)N + req_lds_ints());
        if (fixed + 8 * (size_t)c->t.nsw > lds_max) { dc_destroy(ctx.release()); return DC_EINVAL; }
        c->pc_batched = (int)std::min<size_t>(kMaxN, (lds_max - fixed) / (8 * (size_t)c->t.nsw));
        c->bshape.pc = c->pc_batched;
        const size_t lb = batched_lds(c, c->pc_batched);
        if (set_lds_batched<256, 1>(c, lb) || set_lds_batched<256, 2>(c, lb) || set_lds_batched<256, 4>(c, lb) ||
            set_lds_batched<512, 1>(c, lb) || set_lds_batched<512, 2>(c, lb) || set_lds_batched<512, 4>(c, lb) ||
            set_lds_batched<1024, 1>(c, lb) || set_lds_batched<1024, 2>(c, lb)) {
            dc_destroy(ctx.release());
            return DC_EDEVICE;
        }
    }
    if (set_lds(c, k_topsis_plain<64, true>, c->lds_plain) || set_lds(c, k_topsis_plain<64, false>, c->lds_plain) ||
        set_lds(c, k_topsis_plain<256, true>, c->lds_plain) || set_lds(c, k_topsis_plain<256, false>, c->lds_plain) ||
        set_lds(c, k_topsis_plain<512, true>, c->lds_plain) || set_lds(c, k_topsis_plain<512, false>, c->lds_plain) ||
        set_lds(c, k_topsis_plain<1024, true>, c->lds_plain) || set_lds(c, k_topsis_plain<1024, false>, c->lds_plain) ||
        set_lds(c, k_topsis_plain<1024, true, kPlainK>, c->lds_plain)) {
        dc_destroy(ctx.release());
        return DC_EDEVICE;
    }
    if (cfg->method == DC_AHP) {
        const int bx = (N + kAhpBlock - 1) / kAhpBlock;
        c->tj = std::min(N, 512);
        c->nJ = (N + c->tj - 1) / c->tj;
        c->nI = std::max(1, std::min(bx * 4, (2048 + bx * nc - 1) / (bx * nc)));
        c->ti = (N + c->nI - 1) / c->nI;
        c->nI = (N + c->ti - 1) / c->ti;
        // the 1-9 scale takes the sorted passes while a criterion's sorted
        // values and their prefix sums fit one workgroup's LDS
        c->ahp_sorted = cfg->ahp_scale == DC_AHP_SAATY9 && N <= kAhpSortMax;
        c->sort_runs = (N + kAhpSortBlock - 1) / kAhpSortBlock;
        const size_t colpart = (size_t)c->nI * sizeof(long long);
        if (hipMalloc(&c->d_colpart, (size_t)nc * N * colpart) != hipSuccess ||
            hipMalloc(&c->d_rowpart, (size_t)nc * c->nJ * N * sizeof(float)) != hipSuccess ||
            (c->ahp_sorted && (hipMalloc(&c->d_ysort, (size_t)nc * N * sizeof(int)) != hipSuccess ||
                               hipMalloc(&c->d_wsort, (size_t)nc * N * sizeof(double)) != hipSuccess ||
                               (c->sort_runs > 1 &&
                                hipMalloc(&c->d_runs, (size_t)nc * c->sort_runs * kAhpSortBlock * sizeof(int)) !=
                                    hipSuccess)))) {
            dc_destroy(ctx.release());
            return DC_ENOMEM;
        }
    }
    if (cfg->trace_stride > 0 && cfg->trace_cap > 0) {
        if (hipMalloc(&c->d_tmeta, (size_t)cfg->trace_cap * 4 * sizeof(int)) != hipSuccess ||
            hipMalloc(&c->d_tscore, (size_t)cfg->trace_cap * N * sizeof(float)) != hipSuccess ||
            hipMalloc(&c->d_tcount, (size_t)I * sizeof(int)) != hipSuccess) {
            dc_destroy(ctx.release());
            return DC_ENOMEM;
        }
        hipLaunchKernelGGL(k_fill_i32, dim3(1), dim3(256), 0, c->stream, c->d_tcount, 0, (long long)I);
    }
    const bool grid_ok = cfg->method == DC_TOPSIS && cfg->mode != DC_MODE_BATCHED && I == 1;
    // automatic: the persistent serving kernel from k = 32 on; per-step
    // cooperative launches cost more to launch than they save, so the plain
    // form takes them only when asked (grid = 2)
    if (grid_ok && (cfg->grid == 2 || (cfg->grid == 0 && k >= 32 && cfg->mode == DC_MODE_SERVING))) {
        if (cfg->grid_timeout_us > 0) c->grid_timeout = 100LL * cfg->grid_timeout_us;   // 100 MHz clock
        const int grc = grid_init(c);
        if (grc) { dc_destroy(ctx.release()); return grc; }
    }
    if (cfg->mode == DC_MODE_SERVING) {
        if (I != 1) { dc_destroy(ctx.release()); return DC_EINVAL; }
        const int src = serve_init(c);
        if (src) { dc_destroy(ctx.release()); return src; }
    }
    if (hipEventCreate(&c->ev0) != hipSuccess || hipEventCreate(&c->ev1) != hipSuccess ||
        hipStreamSynchronize(c->stream) != hipSuccess) {
        c->poisoned = true;
        dc_destroy(ctx.release());
        return DC_EDEVICE;
    }
    *out = ctx.release();
    return DC_OK;
}

int dc_submit_request_ranged(dc_ctx *ctx, int32_t instance, int32_t n, const int32_t *cpu_min,
                             const int32_t *cpu_max, const int32_t *ram_min, const int32_t *ram_max, int32_t m,
                             const int32_t *edges, const int32_t *bw_max, const int32_t *pod, int64_t *req_id) {
    if (!ctx) return DC_EINVAL;
    if (ctx->poisoned) return DC_EDEVICE;
    if (instance < 0 || instance >= ctx->I || n < 1 || n > DC_MAX_CONTAINERS || !cpu_min || !ram_min) return DC_EINVAL;
    if (m < 0 || m > n * (n - 1) / 2 || (m > 0 && !edges)) return DC_EINVAL;
    constexpr int kCap = 1 << 22;
    std::vector<char> seen((size_t)n * n, 0);
    for (int q = 0; q < m; ++q) {
        const int i = edges[3 * q], j = edges[3 * q + 1], bw = edges[3 * q + 2];
        const int bx = bw_max ? bw_max[q] : bw;
        if (i < 0 || j < 0 || i >= n || j >= n || i == j || bw <= 0 || bx < bw || bx > kCap) return DC_EINVAL;
        if (seen[(size_t)i * n + j]) return DC_EINVAL;
        seen[(size_t)i * n + j] = seen[(size_t)j * n + i] = 1;
    }
    for (int i = 0; i < n; ++i) {
        const int cx = cpu_max ? cpu_max[i] : cpu_min[i], rx = ram_max ? ram_max[i] : ram_min[i];
        if (cpu_min[i] < 0 || ram_min[i] < 0 || cx < cpu_min[i] || rx < ram_min[i] || cx > kCap || rx > kCap)
            return DC_EINVAL;
    }
    Units U;
    const int urc = build_units(n, cpu_min, cpu_max, ram_min, ram_max, m, edges, bw_max, pod, U);
    if (urc) return urc;
    if (ctx->sv) return serve_submit(ctx, U, req_id);
    ctx->pend_inst.push_back(instance);
    ctx->pend_units.push_back(std::move(U));
    const int64_t id = ctx->next_id++;
    ctx->pend_ids.push_back(id);
    if (req_id) *req_id = id;
    return DC_OK;
}

int dc_submit_request(dc_ctx *ctx, int32_t instance, int32_t n, const int32_t *cpu, const int32_t *ram,
                      int32_t m, const int32_t *edges, const int32_t *pod, int64_t *req_id) {
    return dc_submit_request_ranged(ctx, instance, n, cpu, nullptr, ram, nullptr, m, edges, nullptr, pod, req_id);
}

int dc_schedule(dc_ctx *ctx, int32_t max_results, dc_result *out, int32_t *n_out) {
    if (!ctx || max_results < 0 || (max_results > 0 && !out)) return DC_EINVAL;
    if (ctx->poisoned) return DC_EDEVICE;
    int rc = ctx->sv ? serve_poll(ctx) : upload_pending(ctx);
    if (rc) return rc;
    if (!ctx->sv && !ctx->queued.empty()) {
        ctx->last_launches = 0;
        ctx->last_steps = 0;
        HIPCHK(hipEventRecord(ctx->ev0, ctx->stream));
        for (int bi : ctx->queued) {
            DevBatch &b = *ctx->batches[bi];
            rc = ctx->cfg.mode == DC_MODE_BATCHED ? run_batched(ctx, b, ctx->bshape) : run_plain(ctx, b);
            if (rc) return rc;
        }
        HIPCHK(hipEventRecord(ctx->ev1, ctx->stream));
        HIPCHK(hipGetLastError());
        for (int bi : ctx->queued) {
            rc = collect(ctx, *ctx->batches[bi]);
            if (rc) return rc;
        }
        rc = grid_check(ctx);
        if (rc) return rc;
        HIPCHK(hipEventElapsedTime(&ctx->last_ms, ctx->ev0, ctx->ev1));
        ctx->queued.clear();
    }
    int k = 0;
    const size_t avail = ctx->ready.size() - ctx->ready_head;
    k = (int)std::min<size_t>((size_t)max_results, avail);
    if (k > 0) std::memcpy(out, ctx->ready.data() + ctx->ready_head, sizeof(dc_result) * (size_t)k);
    ctx->ready_head += (size_t)k;
    if (ctx->ready_head == ctx->ready.size()) {
        ctx->ready.clear();
        ctx->ready_head = 0;
    }
    if (n_out) *n_out = k;
    return DC_OK;
}

int dc_release(dc_ctx *ctx, int64_t req_id) {
    if (!ctx) return DC_EINVAL;
    if (ctx->poisoned) return DC_EDEVICE;
    if (ctx->sv) return serve_release(ctx, req_id);
    auto it = ctx->loc.find(req_id);
    if (it == ctx->loc.end() || it->second.released) return DC_ENOENT;
    DevBatch &b = *ctx->batches[it->second.batch];
    const int r = it->second.r;
    for (int bi : ctx->queued)
        if (bi == it->second.batch) return DC_ENOENT;   // not scheduled yet
    if ((int)b.status.size() <= r || b.status[r] != 1) return DC_ENOENT;
    Params p = base_params(ctx, b, b.inst[r]);
    p.s.r = r;
    hipLaunchKernelGGL((k_release<256>), dim3(1), dim3(256), 0, ctx->stream, p);
    HIPCHK(hipGetLastError());
    it->second.released = true;
    return DC_OK;
}

int dc_get_paths(dc_ctx *ctx, int64_t req_id, int32_t cap, int32_t *link_ids, int32_t *n) {
    if (!ctx || cap < 0 || (cap > 0 && !link_ids)) return DC_EINVAL;
    if (ctx->sv) {
        auto sit = ctx->sv->slots.find(req_id);
        if (sit == ctx->sv->slots.end() || sit->second.status != 1 || sit->second.released) return DC_ENOENT;
        const ServeSlot &sl = sit->second;
        std::vector<int> slot(sl.ints);
        HIPCHK(hipMemcpyAsync(slot.data(), ctx->sv->arena + sl.off, sl.ints * sizeof(int), hipMemcpyDeviceToHost,
                              ctx->sv->aux));
        HIPCHK(hipStreamSynchronize(ctx->sv->aux));
        const SlotLayout L = slot_layout(sl.n, sl.P);
        int q = 0;
        for (int g = 0; g < sl.n; ++g)
            for (int x = slot[L.poff + g]; x < slot[L.poff + g + 1]; ++x, ++q) {
                if (q >= cap) continue;
                int *dst = link_ids + 6 * (size_t)q;
                for (int l = 0; l < 6; ++l) dst[l] = -1;
                const int u = slot[L.host + g], v = slot[L.host + slot[L.pj + x]], c = slot[L.code + x];
                if (u != v && c >= 0) host_path_links(ctx->t, u, v, c, dst);
            }
        if (n) *n = q;
        return DC_OK;
    }
    auto it = ctx->loc.find(req_id);
    if (it == ctx->loc.end()) return DC_ENOENT;
    DevBatch &b = *ctx->batches[it->second.batch];
    const int r = it->second.r;
    if ((int)b.status.size() <= r || b.status[r] != 1) return DC_ENOENT;
    const int g0 = b.coff[r], g1 = b.coff[r + 1];
    const int x0 = b.poff[g0], nx = b.poff[g1] - x0;
    std::vector<int> code(std::max(nx, 1));
    if (nx > 0) {
        HIPCHK(hipMemcpyAsync(code.data(), b.view.code + x0, nx * sizeof(int), hipMemcpyDeviceToHost, ctx->stream));
        HIPCHK(hipStreamSynchronize(ctx->stream));
    }
    int q = 0;
    for (int g = g0; g < g1; ++g)
        for (int x = b.poff[g]; x < b.poff[g + 1]; ++x, ++q) {
            if (q >= cap) continue;
            int *dst = link_ids + 6 * (size_t)q;
            for (int l = 0; l < 6; ++l) dst[l] = -1;
            const int u = b.host[g], v = b.host[g0 + b.pj[x]], c = code[x - x0];
            if (u != v && c >= 0) host_path_links(ctx->t, u, v, c, dst);
        }
    if (n) *n = q;
    return DC_OK;
}

int dc_get_alloc(dc_ctx *ctx, int64_t req_id, int32_t *cpu, int32_t *ram, int32_t *bw) {
    if (!ctx) return DC_EINVAL;
    if (ctx->sv) {
        auto sit = ctx->sv->slots.find(req_id);
        if (sit == ctx->sv->slots.end() || sit->second.status != 1 || sit->second.released) return DC_ENOENT;
        const ServeSlot &sl = sit->second;
        std::vector<int> slot(sl.ints);
        HIPCHK(hipMemcpyAsync(slot.data(), ctx->sv->arena + sl.off, sl.ints * sizeof(int), hipMemcpyDeviceToHost,
                              ctx->sv->aux));
        HIPCHK(hipStreamSynchronize(ctx->sv->aux));
        const SlotLayout L = slot_layout(sl.n, sl.P);
        members_alloc(sl.mem, sl.unit_of, sl.n, slot.data() + L.cpua, slot.data() + L.rama, slot.data() + L.pbwa,
                      cpu, ram, bw);
        return DC_OK;
    }
    auto it = ctx->loc.find(req_id);
    if (it == ctx->loc.end()) return DC_ENOENT;
    DevBatch &b = *ctx->batches[it->second.batch];
    const int r = it->second.r;
    if ((int)b.status.size() <= r || b.status[r] != 1) return DC_ENOENT;
    const int g0 = b.coff[r], nu = b.coff[r + 1] - g0;
    const int x0 = b.poff[g0], nx = b.poff[g0 + nu] - x0;
    std::vector<int> ua(2 * (size_t)nu + std::max(nx, 1));
    HIPCHK(hipMemcpyAsync(ua.data(), b.view.cpua + g0, nu * sizeof(int), hipMemcpyDeviceToHost, ctx->stream));
    HIPCHK(hipMemcpyAsync(ua.data() + nu, b.view.rama + g0, nu * sizeof(int), hipMemcpyDeviceToHost, ctx->stream));
    if (nx > 0)
        HIPCHK(hipMemcpyAsync(ua.data() + 2 * nu, b.view.pbwa + x0, nx * sizeof(int), hipMemcpyDeviceToHost,
                              ctx->stream));
    HIPCHK(hipStreamSynchronize(ctx->stream));
    const std::vector<int> uo(b.unit_of.begin() + b.cuoff[r], b.unit_of.begin() + b.cuoff[r + 1]);
    members_alloc(b.mem[r], uo, nu, ua.data(), ua.data() + nu, ua.data() + 2 * nu, cpu, ram, bw);
    return DC_OK;
}

int dc_get_attempt(dc_ctx *ctx, int64_t req_id, int32_t cap, int32_t *hosts, int32_t *n) {
    if (!ctx || cap < 0 || (cap > 0 && !hosts)) return DC_EINVAL;
    if (ctx->sv) {
        auto sit = ctx->sv->slots.find(req_id);
        if (sit == ctx->sv->slots.end() || sit->second.status < 0) return DC_ENOENT;
        const std::vector<int> &hv = sit->second.hosts;
        for (int i = 0; i < (int)hv.size() && i < cap; ++i) hosts[i] = hv[i];
        if (n) *n = (int)hv.size();
        return DC_OK;
    }
    auto it = ctx->loc.find(req_id);
    if (it == ctx->loc.end()) return DC_ENOENT;
    DevBatch &b = *ctx->batches[it->second.batch];
    const int r = it->second.r;
    if ((int)b.status.size() <= r) return DC_ENOENT;
    const int g0 = b.coff[r], c0 = b.cuoff[r], cnt = b.cnt[r];
    for (int i = 0; i < cnt && i < cap; ++i) hosts[i] = b.host[g0 + b.unit_of[c0 + i]];
    if (n) *n = cnt;
    return DC_OK;
}

int dc_get_latency(dc_ctx *ctx, int32_t cap, float *service_us, int32_t *n) {
    if (!ctx || cap < 0 || (cap > 0 && !service_us)) return DC_EINVAL;
    std::vector<std::pair<int64_t, float>> v;
    if (ctx->sv) v = ctx->sv->service_us;
    for (auto &B : ctx->batches) {
        const DevBatch &b = *B;
        for (int r = 0; r < (int)b.tse.size(); ++r)
            v.emplace_back(b.ids[r], (float)((b.tse[r] - b.tsb[r]) / 100.0));   // 100 MHz clock
    }
    std::sort(v.begin(), v.end());
    int k = 0;
    for (; k < (int)v.size() && k < cap; ++k) service_us[k] = v[k].second;
    if (n) *n = (int)v.size();
    return DC_OK;
}

int dc_get_state(dc_ctx *ctx, int32_t instance, int32_t *out) {
    if (!ctx || !out || instance < 0 || instance >= ctx->I) return DC_EINVAL;
    if (ctx->poisoned) return DC_EDEVICE;
    hipStream_t s = ctx->stream;
    if (ctx->sv) {
        int rc = serve_poll(ctx);
        if (rc) return rc;
        if (ctx->sv->comp_pos != ctx->sv->host_pos) return DC_EAGAIN;   // commands still in flight
        s = ctx->sv->aux;
    }
    HIPCHK(hipMemcpyAsync(out, ctx->d_state + (size_t)instance * 6 * ctx->N, 6 * (size_t)ctx->N * sizeof(int),
                          hipMemcpyDeviceToHost, s));
    HIPCHK(hipStreamSynchronize(s));
    return DC_OK;
}

int dc_rewind(dc_ctx *ctx) {
    if (!ctx) return DC_EINVAL;
    if (ctx->poisoned) return DC_EDEVICE;
    if (ctx->sv) return DC_ESTATE;
    int rc = upload_pending(ctx);
    if (rc) return rc;
    HIPCHK(hipMemcpyAsync(ctx->d_state, ctx->d_init, (size_t)ctx->I * 6 * ctx->N * sizeof(int),
                          hipMemcpyDeviceToDevice, ctx->stream));
    if (ctx->d_tcount)
        hipLaunchKernelGGL(k_fill_i32, dim3(1), dim3(256), 0, ctx->stream, ctx->d_tcount, 0, (long long)ctx->I);
    ctx->queued.clear();
    for (size_t bi = 0; bi < ctx->batches.size(); ++bi) {
        rc = reset_outputs(ctx, *ctx->batches[bi]);
        if (rc) return rc;
        ctx->queued.push_back((int)bi);
        for (int64_t id : ctx->batches[bi]->ids) ctx->loc[id].released = false;
    }
    ctx->ready.clear();
    ctx->ready_head = 0;
    ctx->ready_head = 0;
    return DC_OK;
}

int dc_get_trace(dc_ctx *ctx, int32_t cap, int32_t *meta, float *scores, int32_t *n) {
    if (!ctx || cap < 0) return DC_EINVAL;
    if (!ctx->d_tmeta) { if (n) *n = 0; return DC_OK; }
    std::vector<int> cnt(ctx->I);
    HIPCHK(hipMemcpyAsync(cnt.data(), ctx->d_tcount, ctx->I * sizeof(int), hipMemcpyDeviceToHost, ctx->stream));
    HIPCHK(hipStreamSynchronize(ctx->stream));
    long long steps = 0;
    for (int v : cnt) steps = std::max<long long>(steps, v);
    int rec = (int)std::min<long long>(ctx->cfg.trace_cap, (steps + ctx->cfg.trace_stride - 1) / ctx->cfg.trace_stride);
    if (ctx->I > 1) rec = 0;   // per-instance counters share slots; recording is meant for one instance
    rec = std::min(rec, cap);
    if (rec > 0) {
        if (meta) HIPCHK(hipMemcpy(meta, ctx->d_tmeta, (size_t)rec * 4 * sizeof(int), hipMemcpyDeviceToHost));
        if (scores) HIPCHK(hipMemcpy(scores, ctx->d_tscore, (size_t)rec * ctx->N * sizeof(float), hipMemcpyDeviceToHost));
    }
    if (n) *n = rec;
    return DC_OK;
}

int dc_autotune(dc_ctx *ctx, int32_t *block) {
    dc_tune t{};
    const int rc = dc_autotune_cached(ctx, nullptr, &t);
    if (rc == DC_OK && block) *block = t.block;
    return rc;
}

int dc_autotune_cached(dc_ctx *ctx, const char *cache_path, dc_tune *out) {
    if (!ctx) return DC_EINVAL;
    if (ctx->poisoned) return DC_EDEVICE;
    if (ctx->cfg.mode == DC_MODE_SERVING) return DC_ESTATE;
    const bool batched = ctx->cfg.mode == DC_MODE_BATCHED;
    int rc = upload_pending(ctx);
    if (rc) return rc;
    const std::string key = tune_key(ctx);
    if (cache_path && *cache_path) {
        Shape sh;
        float ms = 0.f;
        if (cache_read(cache_path, key, &sh, &ms) && shape_ok(ctx, sh)) {
            if (batched) ctx->bshape = sh; else ctx->plain_bs = sh.bs;
            if (out) *out = dc_tune{sh.bs, sh.g, sh.pc, 1, ms, 0};
            return DC_OK;
        }
    }
    if (ctx->queued.empty()) return DC_ESTATE;
    std::vector<Shape> cand;
    if (batched) {
        std::vector<int> pcs{ctx->pc_batched};
        for (int pc : {32, 16})
            if (pc < ctx->pc_batched) pcs.push_back(pc);
        for (const auto &x : kBatchedShapes)
            for (int pc : pcs) cand.push_back(Shape{x[0], x[1], pc});
    } else {
        for (int bs : {256, 512, 1024})
            if (bs == 256 || bs <= ctx->N) cand.push_back(Shape{bs, host_group(bs), ctx->pc_plain});   // no idle waves
    }
    // tuning runs record no trace and leave the state, the queue, the trace
    // counters and the current shape as they were
    struct Restore {
        dc_ctx *c;
        int stride, plain_bs;
        int *saved = nullptr;
        ~Restore() {
            c->cfg.trace_stride = stride;
            c->plain_bs = plain_bs;
            if (saved) (void)hipFree(saved);
        }
    } guard{ctx, ctx->cfg.trace_stride, ctx->plain_bs};
    ctx->cfg.trace_stride = 0;
    const size_t sbytes = (size_t)ctx->I * 6 * ctx->N * sizeof(int);
    HIPCHK(hipMalloc(&guard.saved, sbytes));
    HIPCHK(hipMemcpyAsync(guard.saved, ctx->d_state, sbytes, hipMemcpyDeviceToDevice, ctx->stream));
    float best_ms = 1e30f;
    Shape best = batched ? ctx->bshape : Shape{ctx->plain_bs, host_group(ctx->plain_bs), ctx->pc_plain};
    for (const Shape &sh : cand) {
        for (int rep = 0; rep < 2; ++rep) {   // first run warms up
            HIPCHK(hipMemcpyAsync(ctx->d_state, guard.saved, sbytes, hipMemcpyDeviceToDevice, ctx->stream));
            for (int bi : ctx->queued) if ((rc = reset_outputs(ctx, *ctx->batches[bi]))) return rc;
            HIPCHK(hipEventRecord(ctx->ev0, ctx->stream));
            ctx->plain_bs = sh.bs;
            for (int bi : ctx->queued) {
                if (batched) {
                    launch_batched(ctx, *ctx->batches[bi], sh, ctx->stream);   // timed eagerly
                    HIPCHK(hipGetLastError());
                } else if ((rc = run_plain(ctx, *ctx->batches[bi]))) {
                    return rc;
                }
            }
            HIPCHK(hipEventRecord(ctx->ev1, ctx->stream));
            HIPCHK(hipEventSynchronize(ctx->ev1));
            float ms = 0.f;
            HIPCHK(hipEventElapsedTime(&ms, ctx->ev0, ctx->ev1));
            if (rep == 1 && ms < best_ms) { best_ms = ms; best = sh; }
        }
    }
    HIPCHK(hipMemcpyAsync(ctx->d_state, guard.saved, sbytes, hipMemcpyDeviceToDevice, ctx->stream));
    for (int bi : ctx->queued) if ((rc = reset_outputs(ctx, *ctx->batches[bi]))) return rc;
    HIPCHK(hipStreamSynchronize(ctx->stream));
    if (batched) ctx->bshape = best; else guard.plain_bs = best.bs;
    if (cache_path && *cache_path) cache_write(cache_path, key, best, best_ms);
    if (out) *out = dc_tune{best.bs, best.g, best.pc, 0, best_ms, (int32_t)cand.size()};
    return DC_OK;
}

int dc_set_shape(dc_ctx *ctx, const dc_tune *shape) {
    if (!ctx || !shape) return DC_EINVAL;
    if (ctx->poisoned) return DC_EDEVICE;
    if (ctx->cfg.mode != DC_MODE_BATCHED) return DC_ESTATE;
    const Shape sh{shape->block, shape->host_group, shape->peer_chunk};
    if (!shape_ok(ctx, sh)) return DC_EINVAL;
    ctx->bshape = sh;
    return DC_OK;
}

int dc_get_shape(dc_ctx *ctx, dc_tune *shape) {
    if (!ctx || !shape) return DC_EINVAL;
    const Shape sh = ctx->cfg.mode == DC_MODE_BATCHED ? ctx->bshape
                                                       : Shape{ctx->plain_bs, host_group(ctx->plain_bs), ctx->pc_plain};
    *shape = dc_tune{sh.bs, sh.g, sh.pc, 0, 0.f, 0};
    return DC_OK;
}

int dc_pending(dc_ctx *ctx, int64_t *n) {
    if (!ctx || !n) return DC_EINVAL;
    if (ctx->poisoned) return DC_EDEVICE;
    if (ctx->sv) {
        int rc = serve_poll(ctx);
        if (rc) return rc;
        *n = ctx->sv->host_pos - ctx->sv->comp_pos;
    } else {
        int64_t q = (int64_t)ctx->pend_ids.size();
        for (int bi : ctx->queued) q += ctx->batches[bi]->R;
        *n = q;
    }
    return DC_OK;
}

int dc_topsis_tiles(int64_t T, int32_t C, int32_t N, const int32_t *x, const uint8_t *feasible,
                    const int32_t *cost, const float *weight, float *scores, int32_t *best, float *best_score,
                    void *stream) {
    TileArgs a{};
    TilePath path{};
    int rc = tiles_prepare(T, C, N, x, feasible, cost, weight, scores, best, best_score, &a, &path);
    if (rc || T == 0) return rc;
    const hipStream_t st = static_cast<hipStream_t>(stream);
    if (path.kind != TILE_SPLIT) return tiles_launch(a, T, path, nullptr, st);
    // the split path's partials: stream-ordered allocation, freed behind the
    // launches (or, where the device has no stream-ordered allocator,
    // allocated and freed around a synchronised launch)
    void *scr = nullptr;
    const size_t bytes = split_scratch_bytes(T, N, C);
    if (hipMallocAsync(&scr, bytes, st) == hipSuccess) {
        rc = tiles_launch(a, T, path, scr, st);
        if (hipFreeAsync(scr, st) != hipSuccess) return DC_EDEVICE;
        return rc;
    }
    (void)hipGetLastError();
    if (hipMalloc(&scr, bytes) != hipSuccess) return DC_ENOMEM;
    rc = tiles_launch(a, T, path, scr, st);
    const bool done = hipStreamSynchronize(st) == hipSuccess;
    if (done) (void)hipFree(scr);      // left allocated if the device did not finish
    return done ? rc : DC_EDEVICE;
}

int dc_topsis_tiles_noalloc(int64_t T, int32_t C, int32_t N, const int32_t *x, const uint8_t *feasible,
                            const int32_t *cost, const float *weight, float *scores, int32_t *best,
                            float *best_score, void *stream) {
    TileArgs a{};
    TilePath path{};
    int rc = tiles_prepare(T, C, N, x, feasible, cost, weight, scores, best, best_score, &a, &path);
    if (rc) return rc;
    void *work = nullptr;
    if ((rc = static_scratch(&work))) return rc;     // the first call on a device resolves the address
    if (T == 0) return DC_OK;
    if (path.kind == TILE_SPLIT && split_scratch_bytes(T, N, C) > kStaticScratchBytes) return DC_ETOOBIG;
    return tiles_launch(a, T, path, work, static_cast<hipStream_t>(stream));
}

int dc_last_timing(dc_ctx *ctx, float *ms, int64_t *launches, int64_t *steps) {
    if (!ctx) return DC_EINVAL;
    if (ms) *ms = ctx->last_ms;
    if (launches) *launches = ctx->last_launches;
    if (steps) *steps = ctx->last_steps;
    return DC_OK;
}

void dc_destroy(dc_ctx *ctx) {
    if (!ctx) return;
    if (ctx->sv && !ctx->poisoned && serve_stop(ctx) != DC_OK) ctx->poisoned = true;
    // every kernel of this library ends on its own (bounded waits, idle exit),
    // so waiting for the streams is safe even on a poisoned context; memory is
    // freed only once nothing can still use it
    bool quiet = !ctx->stream || hipStreamSynchronize(ctx->stream) == hipSuccess;
    if (ctx->sv && ctx->sv->aux) quiet = hipStreamSynchronize(ctx->sv->aux) == hipSuccess && quiet;
    if (ctx->sv) {
        Serve &sv = *ctx->sv;
        if (quiet) {
            if (sv.cmds) (void)hipHostFree(sv.cmds);
            if (sv.comps) (void)hipHostFree(sv.comps);
            if (sv.ctrl) (void)hipHostFree(sv.ctrl);
            if (sv.staging) (void)hipHostFree(sv.staging);
            if (sv.arena) (void)hipFree(sv.arena);
        }
        if (sv.aux) (void)hipStreamDestroy(sv.aux);
    }
    if (quiet) {
        for (auto &b : ctx->batches)
            if (b->dmem) (void)hipFree(b->dmem);
        int *ptrs[] = {ctx->d_state, ctx->d_init, ctx->d_xs, ctx->d_colpart, ctx->d_tmeta, ctx->d_tcount, ctx->d_grid,
                       ctx->d_ysort, ctx->d_runs};
        for (int *p : ptrs)
            if (p) (void)hipFree(p);
        if (ctx->d_rowpart) (void)hipFree(ctx->d_rowpart);
        if (ctx->d_wsort) (void)hipFree(ctx->d_wsort);
        if (ctx->d_tscore) (void)hipFree(ctx->d_tscore);
    } else {
        std::fprintf(stderr, "libdcsched: the device did not finish this context's work; its memory is left allocated\n");
        for (auto &b : ctx->batches) b->pinned = nullptr;   // left allocated too
    }
    if (ctx->ev0) (void)hipEventDestroy(ctx->ev0);
    if (ctx->ev1) (void)hipEventDestroy(ctx->ev1);
    if (ctx->own_stream && ctx->stream) (void)hipStreamDestroy(ctx->stream);
    if (ctx->cap_stream) (void)hipStreamDestroy(ctx->cap_stream);
    delete ctx;
}

}  // extern "C"
