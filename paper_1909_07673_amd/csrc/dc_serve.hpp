// Serving form: one persistent workgroup keeps a data center's state
// resident in device memory and takes requests and departures from a
// command ring in coherent pinned host memory, in submission (FCFS) order,
// writing a completion record per command.  Each request lives in a slot of
// a device arena whose size bounds admission; the slot holds the request as
// a one-request Batch, so every step runs the same code as the other forms.
#pragma once
#include "dc_kernels.hpp"

namespace dcs {

enum { CMD_SUBMIT = 1, CMD_RELEASE = 2, CMD_STOP = 3 };

// Command ring entry (host writes the fields, then seq = position + 1 with
// release semantics).
struct Cmd {
    int seq, type, n, npair, slot_off, rid, pad0, pad1;
};

// Completion record (device writes the fields, then seq = position + 1).
struct Comp {
    int seq, type, rid, status, failat, n;
    long long t_admit, t_decide;     // device clock (100 MHz)
    int host[kMaxN];
    float score[kMaxN];
};

// Layout of a request slot, in int32 units: inputs (copied from the
// staging area) then outputs.
struct SlotLayout {
    int coff, cpu, ram, poff, pj, pbw, cmax, rmax, pbmax, rid, in_end;
    int host, code, failat, status, score, cpua, rama, pbwa, ts, total;
};

__host__ __device__ inline SlotLayout slot_layout(int n, int P) {
    SlotLayout L;
    int o = 0;
    L.coff = o; o += 2;
    L.cpu = o; o += n;
    L.ram = o; o += n;
    L.poff = o; o += n + 1;
    L.pj = o; o += P;
    L.pbw = o; o += P;
    L.cmax = o; o += n;
    L.rmax = o; o += n;
    L.pbmax = o; o += P;
    L.rid = o; o += 1;
    L.in_end = o;
    L.host = o; o += n;
    L.code = o; o += P;
    L.failat = o; o += 1;
    L.status = o; o += 1;
    L.score = o; o += n;
    L.cpua = o; o += n;
    L.rama = o; o += n;
    L.pbwa = o; o += P;
    o += o & 1;
    L.ts = o; o += 4;               // tsb, tse (int64)
    L.total = o;
    return L;
}

__device__ __forceinline__ Batch slot_batch(int *sb, const SlotLayout &L) {
    Batch b;
    b.coff = sb + L.coff;
    b.cpu = sb + L.cpu;
    b.ram = sb + L.ram;
    b.poff = sb + L.poff;
    b.pj = sb + L.pj;
    b.pbw = sb + L.pbw;
    b.cmax = sb + L.cmax;
    b.rmax = sb + L.rmax;
    b.pbmax = sb + L.pbmax;
    b.cpua = sb + L.cpua;
    b.rama = sb + L.rama;
    b.pbwa = sb + L.pbwa;
    b.host = sb + L.host;
    b.score = reinterpret_cast<float *>(sb + L.score);
    b.code = sb + L.code;
    b.status = sb + L.status;
    b.failat = sb + L.failat;
    b.iroff = nullptr;
    b.rid = sb + L.rid;
    b.tsb = reinterpret_cast<long long *>(sb + L.ts);
    b.tse = b.tsb + 1;
    return b;
}

struct ServeArgs {
    Cmd *cmds;               // [cap] command ring (pinned, coherent)
    Comp *comps;             // [cap] completion ring (pinned, coherent)
    int *ctrl;               // [2] device position, exit flag (pinned, coherent)
    const int *staging;      // [cap][stage_ints] request inputs (pinned, coherent)
    int *arena;              // device slot arena
    int cap, stage_ints, start, pad;
    long long idle_ticks;    // exit after this long (device clock) without a command
};

template <int BS>
__global__ __launch_bounds__(BS) void k_serve(Params p, ServeArgs a) {
    extern __shared__ __align__(16) char dsm[];
    Smem sm = carve(dsm, p.pc_cap, p.t.nsw);
    int *rq_host = lds_after_tables(dsm, p.pc_cap, p.t.nsw);
    int *rq_cpu = rq_host + kMaxN, *rq_ram = rq_cpu + kMaxN, *rq_poff = rq_ram + kMaxN;
    int *rq_pj = rq_poff + kMaxN + 4, *rq_pbw = rq_pj + kMaxPairs, *rq_pbmax = rq_pbw + kMaxPairs;
    int *rq_cmax = rq_pbmax + kMaxPairs, *rq_rmax = rq_cmax + kMaxN;
    __shared__ int cmdv[8];
    int pos = a.start;
    long long idle0 = dev_clock();
    for (;;) {
        if (threadIdx.x == 0) {
            Cmd *c = a.cmds + (pos % a.cap);
            int got = 0;
            for (;;) {        // bounded wait: every wave leaves after idle_ticks without work
                if (__hip_atomic_load(&c->seq, __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_SYSTEM) == pos + 1) {
                    got = 1;
                    break;
                }
                if (dev_clock() - idle0 > a.idle_ticks) break;
                __builtin_amdgcn_s_sleep(8);
            }
            cmdv[0] = got ? __hip_atomic_load(&c->type, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM) : CMD_STOP;
            if (got) {
                cmdv[1] = __hip_atomic_load(&c->n, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
                cmdv[2] = __hip_atomic_load(&c->npair, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
                cmdv[3] = __hip_atomic_load(&c->slot_off, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
                cmdv[4] = __hip_atomic_load(&c->rid, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
            }
            cmdv[5] = got;
        }
        __syncthreads();
        const int type = cmdv[0], n = cmdv[1], P = cmdv[2], rid = cmdv[4];
        if (type == CMD_STOP) {
            if (threadIdx.x == 0 && cmdv[5]) ++pos;     // a STOP command is consumed
            break;
        }
        int *sb = a.arena + cmdv[3];
        const SlotLayout L = slot_layout(n, P);
        const Batch b = slot_batch(sb, L);
        __shared__ Batch lb;                  // the steps read the slot's pointers from LDS
        if (threadIdx.x == 0) lb = b;         // (read after the copy loops' barrier)
        const long long t_admit = dev_clock();
        if (type == CMD_SUBMIT) {
            // copy the request into its device slot and into LDS
            const int *stg = a.staging + (size_t)(pos % a.cap) * a.stage_ints;
            for (int x = threadIdx.x; x < L.in_end; x += BS) sb[x] = stg[x];
            for (int x = threadIdx.x; x <= n; x += BS) {
                rq_poff[x] = stg[L.poff + x];
                if (x < n) {
                    rq_cpu[x] = stg[L.cpu + x];
                    rq_ram[x] = stg[L.ram + x];
                    rq_cmax[x] = stg[L.cmax + x];
                    rq_rmax[x] = stg[L.rmax + x];
                    rq_host[x] = -1;
                    sb[L.host + x] = -1;
                    sb[L.score + x] = 0;
                }
            }
            for (int x = threadIdx.x; x < P; x += BS) {
                rq_pj[x] = stg[L.pj + x];
                rq_pbw[x] = stg[L.pbw + x];
                rq_pbmax[x] = stg[L.pbmax + x];
                sb[L.code + x] = -1;
            }
            if (threadIdx.x == 0) {
                sb[L.failat] = -1;
                sb[L.status] = 1;
            }
            __syncthreads();
            for (int i = 0; i < n; ++i) {
                const int q0 = rq_poff[i];
                const StepIn s{0, i, n, 0, i, q0, rq_poff[i + 1] - q0, rq_cpu[i], rq_ram[i], rq_cmax[i], rq_rmax[i]};
                const ReqView rv{rq_pj + q0, rq_pbw + q0, rq_host, rq_host, rq_pbmax + q0, rq_poff, rq_pj};
                if (!topsis_step<BS, BS >= 1024 ? 1 : host_group(BS)>(p.t, p.st, p.m, lb, sm, p.xs, p.pc_cap, p.tr, 0,
                                                                      s, rv))
                    break;
            }
            __syncthreads();
        } else {
            give_back<BS>(p.t, p.st, b, 0, n);       // departure of an accepted request
            __syncthreads();
        }
        // completion record, then its sequence number with release semantics
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
        ++pos;
        if (threadIdx.x == 0) {
            __hip_atomic_store(&cp->seq, pos, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_SYSTEM);
            __hip_atomic_store(a.ctrl, pos, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_SYSTEM);
        }
        idle0 = dev_clock();
    }
    if (threadIdx.x == 0) {
        __hip_atomic_store(a.ctrl, pos, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_SYSTEM);
        __hip_atomic_store(a.ctrl + 1, 1, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_SYSTEM);
    }
}

}  // namespace dcs
