/*
 * dcsched.h -- C ABI of libdcsched, a GPU (AMD MI355X / gfx950) implementation
 * of the per-container host scoring, selection and commit of
 * "Network-Aware Container Scheduling in Multi-Tenant Data Center"
 * (arXiv 1909.07673).
 *
 * Model (section II-A, Table I): a k-ary fat-tree data center G^s(N^s,E^s)
 * (section IV-B) with N = k^3/4 servers, each with available CPU and RAM
 * c^s_u[r], and one available bandwidth bw^s_uv per undirected link (the
 * shared u->v / v->u link of section V-D).  A tenant request Req(N^c,E^c)
 * has n containers with CPU/RAM demands and bandwidth demands between
 * container pairs.  The library decides accept/reject (section II-A) and
 * returns the mappings M_c (container -> server) and M_ec (pair -> path).
 *
 * Per container, in FCFS request order and container index order, every
 * server is scored on the criteria of section V (available CPU and RAM,
 * the fragmentation flag f_u, bw^s_u, the path bandwidth to already placed
 * peers of the same request, the hop count to them) by TOPSIS (section
 * V-C) or AHP (section V-B); servers are then visited in decreasing score,
 * lowest index first on equal scores, and the first on which the container
 * and the widest shortest paths to its placed peers (section V-D) fit
 * (Eqs. (4)-(5)) is committed.  If no server fits, every container of the
 * request is undone and the request is rejected (all or nothing).
 *
 * Units are integers: CPU cores, RAM GB, bandwidth Mbps.
 *
 * Indexing shared with the inputs (k even, h = k/2):
 *   server  u = p*h*h + e*h + s      (pod p, edge switch e, slot s)
 *   link level 0: server uplink u; level 1: edge-aggregation (u/h)*h + a;
 *   level 2: aggregation-core (p*h + a)*h + j, joining aggregation switch
 *   (p, a) and core switch a*h + j.  Each level has N links.
 *
 * Errors: every int-returning call returns DC_OK (0) or a negative code;
 * nothing is thrown across the ABI.  After DC_EDEVICE the context is
 * poisoned and only dc_destroy is valid.  A context is not thread safe.
 * The caller owns every buffer it passes; inputs are copied before the
 * call returns, outputs are written into caller memory.
 */
#ifndef DCSCHED_H
#define DCSCHED_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define DC_MAX_CONTAINERS 64
#define DC_MAX_CRIT 8

enum dc_status {
    DC_OK = 0,
    DC_EINVAL = -1,   /* bad argument: odd k, n > 64, i == j, bw <= 0, ...    */
    DC_ENOMEM = -2,   /* device or host allocation failed                     */
    DC_EAGAIN = -3,   /* serving admission: memory budget full, retry later   */
    DC_ENOENT = -4,   /* unknown request id, or request not accepted          */
    DC_EDEVICE = -5,  /* a HIP call failed; the context is poisoned           */
    DC_ESTATE = -6,   /* call not valid in this mode / state                  */
    DC_ETOOBIG = -7   /* needs more scratch than the static buffer holds      */
};

enum dc_method { DC_TOPSIS = 0, DC_AHP = 1 };
/* Pairwise comparison scale of AHP (section V-B) for values p (row server)
 * and q (column server):
 *   DC_AHP_SAATY9: Saaty's 1-9 scale of p / q (rounded half up, clamped to
 *                  9; q = 0 gives 9; p < q gives the reciprocal);
 *   DC_AHP_RATIO:  p / q (a test mode: priorities are then v / sum(v));
 *   DC_AHP_DIFF:   the differences of section V-B's rule: p - q when p > q,
 *                  1 when equal, 1 / (q - p) when p < q.
 * A cost criterion compares q with p instead. */
enum dc_ahp_scale { DC_AHP_SAATY9 = 0, DC_AHP_RATIO = 1, DC_AHP_DIFF = 2 };
enum dc_mode { DC_MODE_PLAIN = 0, DC_MODE_BATCHED = 1, DC_MODE_SERVING = 2 };
enum dc_routing { DC_ROUTE_EACH = 0, DC_ROUTE_END = 1 };

/* Criteria (section V): available CPU, available RAM, fragmentation flag
 * f_u (1 when u hosts a container placed by this library), path bandwidth
 * (bw^s_u narrowed to the widest shortest path to each remote placed peer),
 * bw^s_u itself (available uplink bandwidth), and the summed hop count to
 * the placed peers (normally a cost criterion). */
enum dc_criterion {
    DC_CRIT_CPU = 0, DC_CRIT_RAM = 1, DC_CRIT_ACTIVE = 2,
    DC_CRIT_PATHBW = 3, DC_CRIT_UPLINK = 4, DC_CRIT_HOPS = 5
};

typedef struct dc_ctx dc_ctx;

typedef struct dc_config {
    int32_t k;              /* fat-tree arity, even, 4..64                          */
    int32_t n_instances;    /* independent data centers (batched form), >= 1        */
    int32_t mode;           /* dc_mode                                              */
    int32_t method;         /* dc_method; AHP runs in the plain form only           */
    int32_t ahp_scale;      /* dc_ahp_scale (AHP only)                              */
    int32_t host_cpu, host_ram;                     /* per-server capacity          */
    int32_t bw_host_edge, bw_edge_agg, bw_agg_core; /* per-level link capacity      */
    int32_t ncrit;          /* 1..DC_MAX_CRIT                                       */
    int32_t crit[DC_MAX_CRIT];      /* dc_criterion ids                             */
    int32_t crit_cost[DC_MAX_CRIT]; /* 1 = smaller is better                        */
    float weight[DC_MAX_CRIT];      /* > 0, summing to 1 within 1e-5 (Table IV)     */
    const int32_t *host_used; /* nullable host array [n_instances][2][N]: CPU, RAM already in use */
    const int32_t *link_used; /* nullable host array [n_instances][3][N]: Mbps already in use     */
    void *stream;           /* hipStream_t to launch on (e.g. torch's), NULL = own stream */
    size_t mem_budget;      /* serving: device bytes for live request slots (0 = 256 MiB) */
    int32_t block;          /* threads per workgroup, 0 = automatic / autotuned     */
    int32_t trace_stride;   /* record the score vector of every trace_stride-th step (0 = off) */
    int32_t trace_cap;      /* at most this many recorded steps                     */
    int32_t grid;           /* TOPSIS plain and serving forms: 0 = automatic (the
                               serving form from k = 32 on runs one cooperative
                               workgroup per pod; the plain form one workgroup),
                               1 = one workgroup per step, 2 = one workgroup per pod */
    int32_t graph;          /* batched form: 0 = automatic (on), 1 = launch directly,
                               2 = capture each queued batch's launch in a HIP graph
                               once per workgroup size and replay it afterwards   */
    int32_t grid_timeout_us; /* cooperative step: longest wait at one grid barrier
                               before the step gives up and the context reports
                               DC_EDEVICE (0 = 100000 us)                         */
    int32_t routing;        /* 0 = each unit's links are routed when it is placed;
                               1 = a request's links are routed after its last
                               unit is placed (section V-D): every pair's widest
                               path on the residuals the placement left, then all
                               demands taken at once; a request whose demands do
                               not fit is rejected with failed_at = n            */
    int32_t reserved[1];
} dc_config;

typedef struct dc_result {
    int64_t req_id;
    int32_t instance;
    int32_t status;         /* 1 accepted, 0 rejected                               */
    int32_t n;              /* containers                                           */
    int32_t failed_at;      /* rejected: first container of the first pod with no
                               server, or n when the links did not fit (routing
                               at the end of the request); accepted: -1            */
    int32_t host[DC_MAX_CONTAINERS];  /* M_c; -1 when rejected                     */
    float score[DC_MAX_CONTAINERS];   /* score of the chosen server                */
} dc_result;

/* Create a context: device-resident state for n_instances data centers
 * G^s(N^s, E^s) (section II-A, Table I), each a k-ary fat-tree of
 * section IV-B (DC configuration) with the per-server CPU / RAM and
 * per-level link capacities of cfg, with the background load applied (the
 * available capacities c^s_u[r] and bw^s_uv of section II-A).  The context
 * owns all device memory; cfg and its arrays are copied.  Returns DC_EINVAL for odd or out of
 * range k, ncrit out of range, unknown criterion, non-positive weights or
 * weights not summing to 1, DC_ENOMEM, DC_EDEVICE. */
int dc_create(const dc_config *cfg, dc_ctx **out);

/* Queue one tenant request for data center `instance` (section II-A).
 * cpu[n], ram[n]: container demands (>= 0).  edges[m][3]: (i, j, bw) with
 * i != j, 0 <= i, j < n, bw > 0, each unordered pair at most once.
 * pod: NULL, or pod[n] with pod[i] >= 0 naming container i's pod (equal
 * ids: same pod) and pod[i] < 0 for a container without one.  Containers of
 * a pod share one server (Eq. (8)): the pod is placed as one unit asking for
 * the summed CPU and RAM of its containers, pods in the order of their first
 * container; traffic inside a pod uses no link, and the links between two
 * pods are routed together, with their summed demand, on one widest path
 * between the two servers.  Without pods every container is its own pod.
 * Summed demands must stay within 2^22 (DC_EINVAL otherwise).  The request
 * id is returned in *req_id; ids grow in submission order, which is the
 * FCFS order.  n must be 1..64. */
int dc_submit_request(dc_ctx *ctx, int32_t instance, int32_t n, const int32_t *cpu,
                      const int32_t *ram, int32_t m, const int32_t *edges,
                      const int32_t *pod, int64_t *req_id);

/* dc_submit_request with demands given as minimum / maximum intervals
 * (section II-A): a container runs with any CPU and RAM in
 * [cpu_min[i], cpu_max[i]] and [ram_min[i], ram_max[i]], a pair with any
 * bandwidth in [edges[q][2], bw_max[q]].  Every feasibility check uses the
 * minima.  Since the utilities U(i), U(ij) (section II-B, Eqs. (1)-(2))
 * grow with what is given, once every minimum fits a placement takes as
 * much CPU and RAM as the chosen server has left, up to the maximum, and
 * each routed pair, in peer order, is topped up by what its path still has,
 * up to its maximum; a pair on one server (or inside a pod) gets its
 * maximum.  A pod asks for the sums of
 * its containers' minima and maxima, and two pods' traffic for the sums of
 * their edges' minima and maxima.  cpu_max, ram_max, bw_max may each be
 * NULL (maximum = minimum, which is dc_submit_request).  DC_EINVAL when a
 * maximum is below its minimum or a summed maximum passes 2^22; otherwise
 * as dc_submit_request.  The caller keeps ownership of every array; they
 * are copied before the call returns. */
int dc_submit_request_ranged(dc_ctx *ctx, int32_t instance, int32_t n, const int32_t *cpu_min,
                             const int32_t *cpu_max, const int32_t *ram_min,
                             const int32_t *ram_max, int32_t m, const int32_t *edges,
                             const int32_t *bw_max, const int32_t *pod, int64_t *req_id);

/* The scheduling decision of section II-A (accept or reject each request,
 * with its mapping M_c) by the selection of section V-C: per container, in
 * FCFS order, every server scored, servers taken in decreasing score (lowest
 * index on ties), the first on which the container and its paths fit
 * (Eqs. (4)-(5)) kept; all or nothing per request.
 * Plain and batched forms: schedule every queued request (FCFS per
 * instance) and block until done; results of the scheduled requests go to
 * out[0..*n_out) in request id order (at most max_results are written; the
 * rest stay available to the next call).  Serving form: non-blocking poll of
 * completed requests, in completion (= submission) order.
 *
 * Serving form (mode DC_MODE_SERVING, one instance): a persistent kernel
 * keeps the state on the device and takes requests and departures in the
 * order dc_submit_request / dc_release publish them, while the caller keeps
 * submitting (continuous batching).  Each live request holds a slot of a
 * device arena of cfg.mem_budget bytes; dc_submit_request returns
 * DC_EAGAIN when the arena or the 1024-entry command ring is full (poll
 * with dc_schedule, release, and retry).  dc_release returns DC_EAGAIN for a
 * request not yet decided.  dc_get_state returns DC_EAGAIN while commands
 * are in flight.  The kernel exits after one second without commands and is
 * relaunched by the next call; dc_destroy stops it. */
int dc_schedule(dc_ctx *ctx, int32_t max_results, dc_result *out, int32_t *n_out);

/* Departure of an accepted request (the end of its duration in the event
 * replay of section VI-A): gives back its CPU, RAM and path bandwidth.  DC_ENOENT for unknown, rejected, pending or released ids. */
int dc_release(dc_ctx *ctx, int64_t req_id);

/* Links of an accepted request's routed pairs (the mapping M_ec of section
 * II-A; each pair's widest shortest path of section V-D): 6 link ids per
 * routed pod pair (a container pair without pods), in the order the pods
 * were placed, then ascending earlier pod, -1 padded (a co-located pair
 * uses no link).  Link id = level*N + index. *n receives the number of
 * pairs; at most cap pairs are written. */
int dc_get_paths(dc_ctx *ctx, int64_t req_id, int32_t cap, int32_t *link_ids, int32_t *n);

/* What an accepted request was given (the [min, max] demands of section
 * II-A, for the utilities of section II-B, Eqs. (1)-(2)): cpu[n], ram[n]
 * per container and bw[m] per edge, in submission order (each may be
 * NULL).  A pod's CPU and RAM, and the
 * bandwidth between two pods, go back to its containers (edges) in order:
 * each first gets its minimum, then what is left up to each one's maximum in
 * turn.  DC_ENOENT for unknown, pending, rejected or (serving form) released
 * ids. */
int dc_get_alloc(dc_ctx *ctx, int64_t req_id, int32_t *cpu, int32_t *ram, int32_t *bw);

/* Servers chosen for each container of a scheduled request, including,
 * for a rejected request, the servers its pods placed before the failing
 * one held before the rollback (-1 for the others).  Meant for lockstep
 * checks.
 * *n receives the container count; at most cap entries are written. */
int dc_get_attempt(dc_ctx *ctx, int64_t req_id, int32_t cap, int32_t *hosts, int32_t *n);

/* Service latency of every scheduled request (first step start to the
 * accept / reject decision, measured with the device's 100 MHz clock), in
 * microseconds, in request id order.  *n receives the count. */
int dc_get_latency(dc_ctx *ctx, int32_t cap, float *service_us, int32_t *n);

/* Copy the current state of one instance to out[6][N] (int32): available
 * CPU, RAM, placed-container count, then link levels 0, 1, 2. */
int dc_get_state(dc_ctx *ctx, int32_t instance, int32_t *out);

/* Plain and batched forms: restore every instance to its state at creation
 * and queue again every request submitted so far, keeping their device
 * copies (no new upload).  Used to replay the same workload. */
int dc_rewind(dc_ctx *ctx);

/* Recorded score vectors (trace_stride > 0): meta[s][4] = (instance,
 * request id (low 31 bits), container, global step number),
 * scores[s][N] float.  *n receives the number of recorded steps. */
int dc_get_trace(dc_ctx *ctx, int32_t cap, int32_t *meta, float *scores, int32_t *n);

/* Launch shape of the scheduling kernel: threads per workgroup, servers
 * each thread scores together in the criteria and selection loops, and
 * placed peers whose path tables are built together (a container with more
 * peers builds them in several chunks).  None of these changes a result:
 * every shape gives bit-identical scores, placements and state. */
typedef struct dc_tune {
    int32_t block;       /* threads per workgroup                                 */
    int32_t host_group;  /* servers per thread per pass                           */
    int32_t peer_chunk;  /* peers per path-table chunk                            */
    int32_t from_cache;  /* 1: read from the cache file, 0: measured              */
    float ms;            /* device time of one pass over the queued work          */
    int32_t candidates;  /* shapes timed (0 when read from the cache)             */
} dc_tune;

/* Plain and batched forms: time every candidate shape on the queued
 * workload (on a scratch copy of the state, recording no trace), keep the
 * fastest for later dc_schedule calls, and return it.  Batched form: every
 * built (block, host_group) pair -- (256|512, 1|2|4) and (1024, 1|2) --
 * with the largest peer chunk the workgroup's LDS holds, 32 and 16; plain
 * form: blocks 256, 512, 1024 (not above the server count) with their fixed
 * grouping.  cache_path (nullable): a text file of JSON objects, one per
 * line, keyed by device architecture, form, method, server count and
 * criterion count; a shape found there for this context is taken without
 * timing, and a measured one is written there (a file that cannot be
 * written is left as it was).  The state, queue and trace are left
 * unchanged.  DC_ESTATE when nothing is queued and the cache has no entry,
 * or in the serving form. */
int dc_autotune_cached(dc_ctx *ctx, const char *cache_path, dc_tune *out);

/* dc_autotune_cached without a cache; *block receives the chosen workgroup
 * size. */
int dc_autotune(dc_ctx *ctx, int32_t *block);

/* Batched form: launch with the given shape from the next dc_schedule on
 * (from_cache, ms and candidates are ignored).  DC_EINVAL for a shape that
 * is not built or a peer chunk outside 1..the largest the LDS holds;
 * DC_ESTATE in the other forms. */
int dc_set_shape(dc_ctx *ctx, const dc_tune *shape);

/* The shape the next dc_schedule launches with (ms and candidates 0). */
int dc_get_shape(dc_ctx *ctx, dc_tune *shape);

/* Work not yet decided: in the serving form the commands (requests and
 * departures) published but not completed, otherwise the requests queued
 * for the next dc_schedule.  Polls completions in the serving form. */
int dc_pending(dc_ctx *ctx, int64_t *n);

/* Milliseconds the last dc_schedule spent on the device, measured with HIP
 * events around its launches on the context's stream, and the number of
 * scheduling kernel launches it made. */
int dc_last_timing(dc_ctx *ctx, float *ms, int64_t *launches, int64_t *steps);

/* TOPSIS scoring and selection (section V-C) on its own, over T decision
 * matrices already in device memory; needs no context.
 *   x          device, [T][C][N] int32, criterion-major, 0 <= value < 2^22
 *              (integer criteria as the container step builds them).
 *   feasible   device, [T][N] uint8 (nonzero = feasible), or NULL (all).
 *   cost       host, [C], 1 = smaller is better, or NULL (all benefit).
 *   weight     host, [C], each > 0 and finite.
 *   scores     device, [T][N] float closeness, or NULL (not written).
 *   best       device, [T] int32: the feasible server of highest closeness,
 *              lowest index on ties; -1 when no server is feasible.
 *   best_score device, [T] float closeness of best (0 when -1), or NULL.
 *   stream     hipStream_t to launch on, NULL = the default stream.
 * Per tile: column L2 norms from exact integer sums of squares, ideal and
 * anti-ideal as column maximum / minimum (swapped for a cost criterion),
 * closeness d-/(d+ + d-) (0 when both distances are 0) in FP32 with the
 * arithmetic of the container step, so its scores are identical to the
 * step's for the same criteria.  Asynchronous on the stream; the caller
 * keeps the buffers alive until it completes.  DC_EINVAL for T < 0 or
 * T >= 2^31, C outside 1..DC_MAX_CRIT, N outside 1..2^20, a null x, best or
 * weight, or a weight that is not positive; DC_ENOMEM when the large-tile
 * path's partials cannot be allocated; DC_EDEVICE when the launch fails.
 * 16-byte aligned x and scores and N % 4 == 0 with a tile a wavefront's
 * registers hold take the fast path (one wavefront per tile); up to 1,024
 * tiles of at least 4,096 servers are split into slices of 2,048 servers
 * over several workgroups, with partials in device memory allocated on the
 * stream for the call (stream-ordered) and freed behind it; other shapes
 * take one workgroup per tile. */
int dc_topsis_tiles(int64_t T, int32_t C, int32_t N, const int32_t *x, const uint8_t *feasible,
                    const int32_t *cost, const float *weight, float *scores, int32_t *best, float *best_score,
                    void *stream);

/* dc_topsis_tiles for callers that cannot allocate device memory: code
 * under HIP graph capture, tight serving loops, harnesses that forbid
 * hipMalloc.  Same arguments, results (bit-identical) and errors, but it
 * calls no hipMalloc, hipFree or allocating routine: the large-tile path's
 * partials live in a static device array of 4 MiB (DC_STATIC_SCRATCH_BYTES),
 * one per device, held until the process ends.  The first call on a device
 * resolves that array's address (hipGetSymbolAddress, which may load the
 * library's code object): make one call, T = 0 will do, before capture.
 * A call whose large-tile partials need more than 4 MiB returns DC_ETOOBIG
 * (about T * ceil(N / 2048) * (16 C + 8) bytes: 1,024 tiles of 27,648
 * servers at C = 8 fit; other shapes use no scratch and have no limit).
 * Every call on one device shares its array: calls that overlap on one
 * device (several streams, several host threads) race and must be
 * serialised by the caller.  The caller passes and owns all inputs and
 * outputs. */
#define DC_STATIC_SCRATCH_BYTES (4u << 20)
int dc_topsis_tiles_noalloc(int64_t T, int32_t C, int32_t N, const int32_t *x, const uint8_t *feasible,
                            const int32_t *cost, const float *weight, float *scores, int32_t *best,
                            float *best_score, void *stream);

void dc_destroy(dc_ctx *ctx);
const char *dc_strerror(int code);

#ifdef __cplusplus
}
#endif

#endif /* DCSCHED_H */
