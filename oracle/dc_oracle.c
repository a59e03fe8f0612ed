/*
 * FP64 CPU oracle for the network-aware container scheduler of
 * "Network-Aware Container Scheduling in Multi-Tenant Data Center"
 * (arXiv 1909.07673).
 *
 * TEST INFRASTRUCTURE ONLY.  Only the tests, the smoke check and the CPU
 * baseline leg of the benchmark may load this file's library.  It shares no
 * code with the GPU library: it builds the data center as an explicit graph
 * and follows the paper's steps in their order, slowly and plainly.
 *
 * What it follows:
 *   - DC graph G^s(N^s,E^s), available capacities c^s_u[r] and available
 *     link bandwidth bw^s_uv:            section II-A, Table I.
 *   - k-ary fat-tree topology:           section IV-B (k^3/4 servers).
 *   - criteria c^s_u + bw^s_u + f_u:     section V, opening paragraphs.
 *   - AHP (M1, M2, pairwise comparison, normalisation, local ranks L1/L2,
 *     global priority PG):               section V-B, Eqs. (9)-(10).
 *   - TOPSIS (evaluation matrix, normalisation, weighting, A+/A-, Ed+/Ed-,
 *     closeness Rank[u], decreasing order): section V-C.
 *   - widest shortest path between hosting servers ("modified Dijkstra")
 *     with one residual per undirected link: section V-D.
 *   - capacity / bandwidth constraints Eqs. (4)-(5) and the accept/reject
 *     decision with mappings M_c, M_ec: sections II-A and III-B.
 *   - demands given as minimum / maximum intervals: section II-A; the
 *     utilities U(i), U(ij) of what is allocated: section II-B,
 *     Eqs. (1)-(2).
 * Readings where the paper is silent or garbled are listed beside the code.
 *
 * Parity pins: every function here is pinned by the CPU tests (hand-worked
 * examples, closed forms, invariants, brute-force enumeration); none is
 * "parity unpinned".
 */
#include <math.h>
#include <omp.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define OR_MAX_CRIT 8
#define OR_INF INT64_MAX

enum { CRIT_CPU = 0, CRIT_RAM = 1, CRIT_ACTIVE = 2, CRIT_PATHBW = 3, CRIT_UPLINK = 4, CRIT_HOPS = 5 };
enum { M_TOPSIS = 0, M_AHP = 1 };
enum { AHP_SAATY9 = 0, AHP_RATIO = 1, AHP_DIFF = 2 };

typedef struct {
    int32_t method, ahp_scale, ncrit;
    int32_t route_end;   /* 1: links routed after the last container is placed (section V-D) */
    int32_t crit[OR_MAX_CRIT];
    int32_t cost[OR_MAX_CRIT];
    double weight[OR_MAX_CRIT];
} or_method;

typedef struct {
    int64_t id;
    int n;
    int *host;          /* n */
    int *cpu, *ram;     /* n, allocated */
    int npath;
    int *plink;         /* npath * 6 link ids, -1 padded */
    int64_t *pbw;       /* npath, allocated */
    int live;
} or_record;

typedef struct {
    int k, half, N, n_edge, n_agg, n_core, n_nodes, n_links;
    int *adj_off, *adj_to, *adj_link;   /* CSR adjacency, neighbours ascending */
    int *link_a, *link_b;               /* endpoints of each undirected link */
    int64_t *link_res;                  /* available bandwidth bw^s_uv (Mbps) */
    int64_t *cpu_res, *ram_res;         /* available c^s_u[CPU], c^s_u[RAM] */
    int *nplaced;                       /* containers placed on u by the scheduler */
    or_record *rec;
    int nrec, caprec;
    /* scratch */
    int *dist, *queue;
    int64_t *best;
} or_dc;

/* ------------------------------------------------------------------ */
/* Explicit fat-tree graph (section IV-B: k-port switches, k^3/4 servers). */
/* Node ids: hosts [0,N), edge switches [N, N+E), aggregation switches     */
/* [N+E, N+2E), core switches after.  Link ids: level*N + index, with the  */
/* index conventions of the shared input format.                           */
/* ------------------------------------------------------------------ */

static void add_link(or_dc *d, int id, int a, int b) { d->link_a[id] = a; d->link_b[id] = b; }

static int cmp_pair(const void *x, const void *y) {
    const int *p = (const int *)x, *q = (const int *)y;
    if (p[0] != q[0]) return p[0] < q[0] ? -1 : 1;
    return p[1] < q[1] ? -1 : (p[1] > q[1]);
}

or_dc *or_create(int k, int host_cpu, int host_ram, int bw_he, int bw_ea, int bw_ac,
                 const int32_t *host_used, const int32_t *link_used) {
    if (k < 2 || (k & 1)) return NULL;
    or_dc *d = (or_dc *)calloc(1, sizeof(or_dc));
    d->k = k; d->half = k / 2; d->N = k * k * k / 4;
    d->n_edge = k * k / 2; d->n_agg = k * k / 2; d->n_core = k * k / 4;
    d->n_nodes = d->N + d->n_edge + d->n_agg + d->n_core;
    d->n_links = 3 * d->N;
    int N = d->N, h = d->half;
    int node_edge = N, node_agg = N + d->n_edge, node_core = N + 2 * d->n_edge;
    d->link_a = (int *)malloc(sizeof(int) * d->n_links);
    d->link_b = (int *)malloc(sizeof(int) * d->n_links);
    d->link_res = (int64_t *)malloc(sizeof(int64_t) * d->n_links);
    for (int u = 0; u < N; ++u) {                       /* host - edge */
        add_link(d, u, u, node_edge + u / h);
        d->link_res[u] = bw_he;
    }
    for (int eg = 0; eg < d->n_edge; ++eg) {            /* edge - aggregation (same pod) */
        int p = eg / h;
        for (int a = 0; a < h; ++a) {
            int id = N + eg * h + a;
            add_link(d, id, node_edge + eg, node_agg + p * h + a);
            d->link_res[id] = bw_ea;
        }
    }
    for (int ag = 0; ag < d->n_agg; ++ag) {             /* aggregation - core */
        int a = ag % h;
        for (int j = 0; j < h; ++j) {
            int id = 2 * N + ag * h + j;
            add_link(d, id, node_agg + ag, node_core + a * h + j);
            d->link_res[id] = bw_ac;
        }
    }
    if (link_used)
        for (int l = 0; l < d->n_links; ++l) d->link_res[l] -= link_used[l];
    /* CSR adjacency with ascending neighbour ids */
    int nl = d->n_links;
    /* triples (from, to, link) sorted by (from, to) */
    int *tri = (int *)malloc(sizeof(int) * 3 * 2 * nl);
    for (int l = 0; l < nl; ++l) {
        tri[6 * l + 0] = d->link_a[l]; tri[6 * l + 1] = d->link_b[l]; tri[6 * l + 2] = l;
        tri[6 * l + 3] = d->link_b[l]; tri[6 * l + 4] = d->link_a[l]; tri[6 * l + 5] = l;
    }
    /* simple insertion into buckets then sort each bucket */
    d->adj_off = (int *)calloc(d->n_nodes + 1, sizeof(int));
    for (int e = 0; e < 2 * nl; ++e) d->adj_off[tri[3 * e] + 1]++;
    for (int v = 0; v < d->n_nodes; ++v) d->adj_off[v + 1] += d->adj_off[v];
    int *fill = (int *)calloc(d->n_nodes, sizeof(int));
    int *tmp = (int *)malloc(sizeof(int) * 2 * 2 * nl);
    for (int e = 0; e < 2 * nl; ++e) {
        int v = tri[3 * e];
        int pos = d->adj_off[v] + fill[v]++;
        tmp[2 * pos] = tri[3 * e + 1]; tmp[2 * pos + 1] = tri[3 * e + 2];
    }
    for (int v = 0; v < d->n_nodes; ++v)
        qsort(tmp + 2 * d->adj_off[v], d->adj_off[v + 1] - d->adj_off[v], 2 * sizeof(int), cmp_pair);
    d->adj_to = (int *)malloc(sizeof(int) * 2 * nl);
    d->adj_link = (int *)malloc(sizeof(int) * 2 * nl);
    for (int e = 0; e < 2 * nl; ++e) { d->adj_to[e] = tmp[2 * e]; d->adj_link[e] = tmp[2 * e + 1]; }
    free(tmp); free(fill); free(tri);

    d->cpu_res = (int64_t *)malloc(sizeof(int64_t) * N);
    d->ram_res = (int64_t *)malloc(sizeof(int64_t) * N);
    d->nplaced = (int *)calloc(N, sizeof(int));
    for (int u = 0; u < N; ++u) {
        d->cpu_res[u] = host_cpu - (host_used ? host_used[u] : 0);
        d->ram_res[u] = host_ram - (host_used ? host_used[N + u] : 0);
    }
    d->dist = (int *)malloc(sizeof(int) * d->n_nodes);
    d->queue = (int *)malloc(sizeof(int) * d->n_nodes);
    d->best = (int64_t *)malloc(sizeof(int64_t) * d->n_nodes);
    return d;
}

void or_destroy(or_dc *d) {
    if (!d) return;
    for (int r = 0; r < d->nrec; ++r) {
        free(d->rec[r].host); free(d->rec[r].cpu); free(d->rec[r].ram);
        free(d->rec[r].plink); free(d->rec[r].pbw);
    }
    free(d->rec);
    free(d->adj_off); free(d->adj_to); free(d->adj_link);
    free(d->link_a); free(d->link_b); free(d->link_res);
    free(d->cpu_res); free(d->ram_res); free(d->nplaced);
    free(d->dist); free(d->queue); free(d->best);
    free(d);
}

int or_num_hosts(const or_dc *d) { return d->N; }

/* Threads the AHP matrices are shared out over (results do not depend on
 * it); returns the count in effect. */
int or_set_threads(int n) {
    if (n > 0) omp_set_num_threads(n);
    return omp_get_max_threads();
}
int or_num_nodes(const or_dc *d) { return d->n_nodes; }

/* State in the shared SoA order: cpu, ram, nplaced, uplink, edge-agg, agg-core. */
void or_get_state(const or_dc *d, int32_t *out) {
    int N = d->N;
    for (int u = 0; u < N; ++u) {
        out[u] = (int32_t)d->cpu_res[u];
        out[N + u] = (int32_t)d->ram_res[u];
        out[2 * N + u] = d->nplaced[u];
    }
    for (int l = 0; l < 3 * N; ++l) out[3 * N + l] = (int32_t)d->link_res[l];
}

void or_set_link(or_dc *d, int link, int64_t res) { d->link_res[link] = res; }

/* Breadth-first distances (in links) from node src over the explicit graph. */
static void bfs(or_dc *d, int src) {
    for (int v = 0; v < d->n_nodes; ++v) d->dist[v] = -1;
    int qh = 0, qt = 0;
    d->dist[src] = 0; d->queue[qt++] = src;
    while (qh < qt) {
        int x = d->queue[qh++];
        for (int e = d->adj_off[x]; e < d->adj_off[x + 1]; ++e) {
            int y = d->adj_to[e];
            if (d->dist[y] < 0) { d->dist[y] = d->dist[x] + 1; d->queue[qt++] = y; }
        }
    }
}

/* Widest minimum-hop path from src to every node (section V-D: the
 * shortest path with the maximum available bandwidth).  Minimum-hop paths
 * to y extend minimum-hop paths to a neighbour one layer closer, so the
 * widest bottleneck follows layer by layer; best[src] = +inf.
 * Writes bottleneck and hop count for every host. */
void or_widest_from(or_dc *d, int src, int64_t *W, int32_t *hops) {
    bfs(d, src);
    int n = d->n_nodes;
    d->best[src] = OR_INF;
    for (int qi = 1; qi < n; ++qi) {
        int y = d->queue[qi];
        int64_t b = -1;
        for (int e = d->adj_off[y]; e < d->adj_off[y + 1]; ++e) {
            int x = d->adj_to[e];
            if (d->dist[x] == d->dist[y] - 1) {
                int64_t r = d->link_res[d->adj_link[e]];
                int64_t via = d->best[x] < r ? d->best[x] : r;
                if (via > b) b = via;
            }
        }
        d->best[y] = b;
    }
    for (int u = 0; u < d->N; ++u) {
        if (W) W[u] = d->best[u];
        if (hops) hops[u] = d->dist[u];
    }
}

/* Enumerates every minimum-hop path from u to v (DFS over the BFS layers
 * towards v, neighbours in ascending id order, hence paths in
 * lexicographic order of their node sequences).  Returns the number of
 * paths; *bott receives the widest bottleneck, links[] (<= 6 entries) the
 * first path (lexicographically) reaching it, *hops the hop count.
 * u == v gives one empty path with bottleneck +inf. */
typedef struct { or_dc *d; int target; int depth; int cur[8]; int64_t best; int bestl[8]; int count; } enum_ctx;

static void dfs_paths(enum_ctx *c, int x, int64_t bott) {
    or_dc *d = c->d;
    if (x == c->target) {
        c->count++;
        if (bott > c->best) {
            c->best = bott;
            for (int i = 0; i < c->depth; ++i) c->bestl[i] = c->cur[i];
        }
        return;
    }
    for (int e = d->adj_off[x]; e < d->adj_off[x + 1]; ++e) {
        int y = d->adj_to[e];
        if (d->dist[y] == d->dist[x] - 1) {
            int64_t r = d->link_res[d->adj_link[e]];
            c->cur[c->depth++] = d->adj_link[e];
            dfs_paths(c, y, bott < r ? bott : r);
            c->depth--;
        }
    }
}

int or_widest_enum(or_dc *d, int u, int v, int64_t *bott, int32_t *links, int32_t *hops) {
    bfs(d, v);
    enum_ctx c;
    memset(&c, 0, sizeof c);
    c.d = d; c.target = v; c.best = -1;
    dfs_paths(&c, u, OR_INF);
    *bott = c.best;
    *hops = d->dist[u];
    for (int i = 0; i < 6; ++i) links[i] = i < d->dist[u] ? c.bestl[i] : -1;
    return c.count;
}

/* ------------------------------------------------------------------ */
/* Section V-C: TOPSIS over the criterion-major evaluation matrix          */
/* M[v*|N|+u] (here X[c*N+u]).  Normalisation: column L2 (Hwang & Yoon);   */
/* a zero column stays zero.  A+ / A-: per-criterion maximum / minimum of  */
/* the weighted matrix over all servers (swapped for a cost criterion).    */
/* Closeness Rank[u] = Ed-/(Ed+ + Ed-), taken as 0 when both are 0.        */
/* ------------------------------------------------------------------ */
void or_topsis(int N, int C, const double *X, const double *w, const int32_t *cost, double *rank) {
    double *V = (double *)malloc(sizeof(double) * (size_t)C * N);
    double Ap[OR_MAX_CRIT], Am[OR_MAX_CRIT];
    for (int c = 0; c < C; ++c) {
        double ss = 0.0;
        for (int u = 0; u < N; ++u) ss += X[(size_t)c * N + u] * X[(size_t)c * N + u];
        double norm = sqrt(ss);
        for (int u = 0; u < N; ++u) {
            double r = norm > 0.0 ? X[(size_t)c * N + u] / norm : 0.0;   /* normalisation */
            V[(size_t)c * N + u] = r * w[c];                            /* weighting */
        }
        double mx = V[(size_t)c * N], mn = V[(size_t)c * N];
        for (int u = 1; u < N; ++u) {
            double x = V[(size_t)c * N + u];
            if (x > mx) mx = x;
            if (x < mn) mn = x;
        }
        Ap[c] = cost[c] ? mn : mx;
        Am[c] = cost[c] ? mx : mn;
    }
    for (int u = 0; u < N; ++u) {
        double sp = 0.0, sm = 0.0;
        for (int c = 0; c < C; ++c) {
            double x = V[(size_t)c * N + u];
            sp += (x - Ap[c]) * (x - Ap[c]);
            sm += (x - Am[c]) * (x - Am[c]);
        }
        double edp = sqrt(sp), edm = sqrt(sm);
        rank[u] = (edp + edm) > 0.0 ? edm / (edp + edm) : 0.0;
    }
    free(V);
}

/* ------------------------------------------------------------------ */
/* Section V-B: AHP.  Pairwise comparison of two values on the 1-9 scale   */
/* (Saaty): equal values compare as 1; a larger value p against a smaller  */
/* q scores the ratio p/q rounded half up and clamped to [1, 9] (q = 0     */
/* scores 9); the reverse comparison is the reciprocal.  The ratio mode    */
/* compares by the plain value ratio p/q.                                  */
/* ------------------------------------------------------------------ */
double or_saaty(double p, double q) {
    if (p == q) return 1.0;
    if (p < q) return 1.0 / or_saaty(q, p);
    if (q == 0.0) return 9.0;
    double s = floor(p / q + 0.5);
    if (s > 9.0) s = 9.0;
    if (s < 1.0) s = 1.0;
    return s;
}

/* The pairwise rule as section V-B states it, on differences: the larger
 * value's entry is the difference, equal values give 1, and the smaller
 * value's entry is the reciprocal of the difference.  The printed rule puts
 * the (negative) difference itself under the reciprocal; its absolute value
 * is taken so that a(j, i) = 1 / a(i, j), as in every AHP comparison
 * matrix. */
double or_diff(double p, double q) {
    if (p == q) return 1.0;
    return p > q ? p - q : 1.0 / (q - p);
}

static double compare(int scale, double p, double q) {
    return scale == AHP_RATIO ? p / q : scale == AHP_DIFF ? or_diff(p, q) : or_saaty(p, q);
}

/* Local rank of a pairwise matrix A (n x n, row-major): normalise each
 * column by its sum, then average each row (Eqs. (9)-(10)). */
/* Threads (OpenMP) share out whole columns and whole rows; each sum still
 * adds its terms in index order, so the results do not depend on the thread
 * count. */
static void local_rank(int n, const double *A, double *L) {
    double *col = (double *)calloc(n, sizeof(double));
    const int J = 64;
#pragma omp parallel for schedule(static) if (n >= 1024)
    for (int j0 = 0; j0 < n; j0 += J)
        for (int i = 0; i < n; ++i)
            for (int j = j0; j < j0 + J && j < n; ++j) col[j] += A[(size_t)i * n + j];
#pragma omp parallel for schedule(static) if (n >= 1024)
    for (int i = 0; i < n; ++i) {
        double s = 0.0;
        for (int j = 0; j < n; ++j) s += A[(size_t)i * n + j] / col[j];
        L[i] = s / n;
    }
    free(col);
}

/* Criteria level: M1 holds the weights; the pairwise matrix compares them
 * by ratio (W[a]/W[b]), whose local rank P1 is W itself when sum(W) = 1.
 * Alternative level: per criterion the |N| x |N| comparison matrix M2 of
 * the server values (a cost criterion compares in reverse), local rank P2.
 * Global priority PG[u] = sum_c P1[c] * P2[c][u]. */
void or_ahp(int N, int C, const double *X, const double *w, const int32_t *cost, int scale,
            double *PG, double *P1_out, double *P2_out) {
    double M1[OR_MAX_CRIT * OR_MAX_CRIT] = {0}, P1[OR_MAX_CRIT] = {0};
    for (int a = 0; a < C; ++a)
        for (int b = 0; b < C; ++b) M1[a * C + b] = w[a] / w[b];
    local_rank(C, M1, P1);
    double *M2 = (double *)malloc(sizeof(double) * (size_t)N * N);
    double *P2 = (double *)malloc(sizeof(double) * (size_t)C * N);
    for (int c = 0; c < C; ++c) {
        const double *x = X + (size_t)c * N;
#pragma omp parallel for schedule(static) if (N >= 1024)
        for (int i = 0; i < N; ++i)
            for (int j = 0; j < N; ++j)
                M2[(size_t)i * N + j] = cost[c] ? compare(scale, x[j], x[i]) : compare(scale, x[i], x[j]);
        local_rank(N, M2, P2 + (size_t)c * N);
    }
    for (int u = 0; u < N; ++u) {
        double s = 0.0;
        for (int c = 0; c < C; ++c) s += P1[c] * P2[(size_t)c * N + u];
        PG[u] = s;
    }
    if (P1_out) memcpy(P1_out, P1, sizeof(double) * C);
    if (P2_out) memcpy(P2_out, P2, sizeof(double) * (size_t)C * N);
    free(M2); free(P2);
}

/* ------------------------------------------------------------------ */
/* Per-container criteria (section V): available CPU and RAM c^s_u, the    */
/* server's fragmentation flag f_u (1 when it hosts a container placed by  */
/* this scheduler), bw^s_u (sum of available bandwidth of links with       */
/* source u), the path bandwidth to already-placed peers (bw^s_u narrowed  */
/* by the widest shortest path to each remote peer), and the hop count to  */
/* peers (cost).  Feasibility from Eqs. (4)-(5): CPU, RAM, the uplink      */
/* carrying the sum of remote peer demands, and each remote peer's widest  */
/* path carrying its demand.                                               */
/* ------------------------------------------------------------------ */
static void criteria(or_dc *d, const or_method *m, int cpu_i, int ram_i, int P,
                     const int *ph, const int *pbw, double *X, int *feas) {
    int N = d->N;
    int64_t *W = (int64_t *)malloc(sizeof(int64_t) * N);
    int32_t *hp = (int32_t *)malloc(sizeof(int32_t) * N);
    int64_t *pathbw = (int64_t *)malloc(sizeof(int64_t) * N);
    int64_t *upsum = (int64_t *)calloc(N, sizeof(int64_t));
    int64_t *hopsum = (int64_t *)calloc(N, sizeof(int64_t));
    int64_t *bwu = (int64_t *)malloc(sizeof(int64_t) * N);
    for (int u = 0; u < N; ++u) {
        int64_t s = 0;                               /* bw^s_u: links with source u */
        for (int e = d->adj_off[u]; e < d->adj_off[u + 1]; ++e) s += d->link_res[d->adj_link[e]];
        bwu[u] = s;
        pathbw[u] = s;
        feas[u] = d->cpu_res[u] >= cpu_i && d->ram_res[u] >= ram_i;
    }
    for (int p = 0; p < P; ++p) {
        or_widest_from(d, ph[p], W, hp);
        for (int u = 0; u < N; ++u) {
            hopsum[u] += hp[u];
            if (u == ph[p]) continue;                /* co-located peer: no link used */
            if (W[u] < pathbw[u]) pathbw[u] = W[u];
            upsum[u] += pbw[p];
            if (W[u] < pbw[p]) feas[u] = 0;
        }
    }
    for (int u = 0; u < N; ++u) {
        if (bwu[u] < upsum[u]) feas[u] = 0;
        for (int c = 0; c < m->ncrit; ++c) {
            double v = 0.0;
            switch (m->crit[c]) {
            case CRIT_CPU: v = (double)d->cpu_res[u]; break;
            case CRIT_RAM: v = (double)d->ram_res[u]; break;
            case CRIT_ACTIVE: v = d->nplaced[u] > 0 ? 1.0 : 0.0; break;
            case CRIT_PATHBW: v = (double)pathbw[u]; break;
            case CRIT_UPLINK: v = (double)bwu[u]; break;
            case CRIT_HOPS: v = (double)hopsum[u]; break;
            }
            X[(size_t)c * N + u] = v;
        }
    }
    free(W); free(hp); free(pathbw); free(upsum); free(hopsum); free(bwu);
}

/* Compute criteria and scores of every server for one container. */
int or_step_scores(or_dc *d, const or_method *m, int cpu_i, int ram_i, int P,
                   const int32_t *ph, const int32_t *pbw, double *X, int32_t *feas, double *score) {
    int N = d->N;
    int *f = (int *)malloc(sizeof(int) * N);
    criteria(d, m, cpu_i, ram_i, P, ph, pbw, X, f);
    if (feas) for (int u = 0; u < N; ++u) feas[u] = f[u];
    if (m->method == M_TOPSIS) or_topsis(N, m->ncrit, X, m->weight, m->cost, score);
    else or_ahp(N, m->ncrit, X, m->weight, m->cost, m->ahp_scale, score, NULL, NULL);
    free(f);
    return 0;
}

/* ------------------------------------------------------------------ */
/* Commit of one container on server u: subtract CPU and RAM, mark u      */
/* active, and route every remote placed peer in ascending order on its   */
/* widest shortest path under the current residuals (ties: the            */
/* lexicographically first path).  Fails, leaving no trace, when a         */
/* resource or a path bottleneck does not cover the minimum demand (Eqs.   */
/* (4)-(5)).                                                               */
/*                                                                          */
/* Demand intervals (section II-A): a container runs with any amount in    */
/* [min, max] and its utility (Eqs. (1)-(2)) grows with the amount.  The   */
/* commit first fits every minimum as above (so whether a server fits does */
/* not depend on the maxima); then CPU and RAM take min(max, residual), and */
/* each routed peer path, in peer order, tops its pair up by what the path */
/* still has, to at most the maximum.  A peer on the same server needs no  */
/* link and gets its maximum.  Fixed demands are the case min = max.       */
/* ------------------------------------------------------------------ */
typedef struct { int nl; int link[6]; int64_t bw; } or_path;

static int64_t min64(int64_t a, int64_t b) { return a < b ? a : b; }

/* Tops path p up from its minimum towards its maximum with what its most
 * loaded link still has. */
static void top_up(or_dc *d, or_path *pp, int64_t max) {
    if (pp->nl == 0 || pp->bw >= max) return;
    int64_t room = max - pp->bw;
    for (int l = 0; l < pp->nl; ++l) room = min64(room, d->link_res[pp->link[l]]);
    if (room <= 0) return;
    for (int l = 0; l < pp->nl; ++l) d->link_res[pp->link[l]] -= room;
    pp->bw += room;
}

/* Cut condition at a peer server v != u: every path that ends at v leaves
 * one of v's links with its demand taken off, so routing all peers held by
 * v needs the summed residual of v's links to cover their summed demand.
 * When it does not, the routing below is bound to fail; returning early
 * gives the same answer without enumerating paths. */
static int peer_cut_short(const or_dc *d, int u, int P, const int *ph, const int *pbw) {
    for (int p = 0; p < P; ++p) {
        const int v = ph[p];
        if (v == u) continue;
        int64_t need = 0, cap = 0;
        for (int q = 0; q < P; ++q) if (ph[q] == v) need += pbw[q];
        for (int e = d->adj_off[v]; e < d->adj_off[v + 1]; ++e) cap += d->link_res[d->adj_link[e]];
        if (cap < need) return 1;
    }
    return 0;
}

static int try_commit(or_dc *d, int u, int cpu_i, int cpu_x, int ram_i, int ram_x, int P, const int *ph,
                      const int *pbw, const int *pbx, or_path *paths, int *cpu_a, int *ram_a) {
    if (d->cpu_res[u] < cpu_i || d->ram_res[u] < ram_i) return 0;
    if (peer_cut_short(d, u, P, ph, pbw)) return 0;
    int routed = 0, ok = 1;
    for (int p = 0; p < P; ++p) {
        paths[p].nl = 0; paths[p].bw = pbx[p];
        if (ph[p] == u) continue;
        int64_t b; int32_t links[6], hops;
        or_widest_enum(d, u, ph[p], &b, links, &hops);
        if (b < pbw[p]) { ok = 0; break; }
        paths[p].nl = hops;
        paths[p].bw = pbw[p];
        for (int l = 0; l < hops; ++l) { paths[p].link[l] = links[l]; d->link_res[links[l]] -= paths[p].bw; }
        routed = p + 1;
    }
    if (!ok) {
        for (int p = routed - 1; p >= 0; --p)
            for (int l = 0; l < paths[p].nl; ++l) d->link_res[paths[p].link[l]] += paths[p].bw;
        return 0;
    }
    for (int p = 0; p < P; ++p) top_up(d, paths + p, pbx[p]);
    *cpu_a = (int)min64(cpu_x, d->cpu_res[u]);
    *ram_a = (int)min64(ram_x, d->ram_res[u]);
    d->cpu_res[u] -= *cpu_a; d->ram_res[u] -= *ram_a; d->nplaced[u] += 1;
    return 1;
}

static void undo_commit(or_dc *d, int u, int cpu_a, int ram_a, int P, const or_path *paths) {
    for (int p = P - 1; p >= 0; --p)
        for (int l = 0; l < paths[p].nl; ++l) d->link_res[paths[p].link[l]] += paths[p].bw;
    d->cpu_res[u] += cpu_a; d->ram_res[u] += ram_a; d->nplaced[u] -= 1;
}

typedef struct { double s; int u; } cand;
static int cmp_cand(const void *x, const void *y) {
    const cand *a = (const cand *)x, *b = (const cand *)y;
    if (a->s != b->s) return a->s > b->s ? -1 : 1;
    return a->u < b->u ? -1 : (a->u > b->u);
}

/* ------------------------------------------------------------------ */
/* One request in FCFS order.  Containers are taken in index order; each   */
/* is scored over all servers, the servers are visited in decreasing score */
/* (lowest index first on equal scores), and the first whose commit        */
/* succeeds hosts the container.  When none does, every container of the   */
/* request is undone and the request is rejected (all or nothing).         */
/*                                                                          */
/* follow (nullable): lockstep mode; commit follow[i] instead of the own    */
/* choice (follow[i] = -1 means the other side rejected at step i).         */
/* Per step outputs (nullable): own choice, its score, the score gap to the */
/* second commit-successful server, the score of the committed server, and */
/* the full score vector (n x N).                                          */
/* tie_low (nullable, per step, lockstep mode): the lowest-index server    */
/* below the followed one whose criteria are identical to it, which is     */
/* feasible and whose commit succeeds, or -1.  Such a server has the same  */
/* score, so the scan in (score desc, index asc) order reaches it first:   */
/* any other entry than -1 means the followed side broke the exact-tie     */
/* rule of the decreasing-order selection (section V-C).                   */
/* Demand intervals (nullable, then max = min): cpu_max, ram_max per       */
/* container, bw_max per edge (edges hold the minimum).  Allocations       */
/* (nullable outputs, accepted requests): cpu_a, ram_a per container and    */
/* bw_a per edge.                                                           */
/* Returns 1 accepted, 0 rejected, -1 invalid request, -2 the followed      */
/* server cannot be committed, -3 the followed side rejected while this one */
/* found a server (or the reverse).                                        */
/* ------------------------------------------------------------------ */
int or_run_request(or_dc *d, const or_method *m, int n, const int32_t *cpu, const int32_t *ram,
                   int ne, const int32_t *edges, const int32_t *cpu_max, const int32_t *ram_max,
                   const int32_t *bw_max, const int32_t *follow,
                   int32_t *host_out, double *score_out, int32_t *ref_host, double *ref_top,
                   double *ref_gap, double *dump, int32_t *failed_at, int64_t *rec_id,
                   int32_t *cpu_a, int32_t *ram_a, int32_t *bw_a, int32_t *tie_low) {
    int N = d->N;
    if (n <= 0) return -1;
    for (int i = 0; i < n; ++i)
        if ((cpu_max && cpu_max[i] < cpu[i]) || (ram_max && ram_max[i] < ram[i])) return -1;
    /* peer lists: for container i, edges (i, j) with j < i, j ascending */
    int64_t *bwm = (int64_t *)calloc((size_t)n * n, sizeof(int64_t));
    int64_t *bwx = (int64_t *)calloc((size_t)n * n, sizeof(int64_t));
    for (int e = 0; e < ne; ++e) {
        int a = edges[3 * e], b = edges[3 * e + 1], bw = edges[3 * e + 2];
        int bx = bw_max ? bw_max[e] : bw;
        if (a < 0 || b < 0 || a >= n || b >= n || a == b || bw <= 0 || bx < bw || bwm[(size_t)a * n + b]) {
            free(bwm); free(bwx); return -1;
        }
        bwm[(size_t)a * n + b] = bw; bwm[(size_t)b * n + a] = bw;
        bwx[(size_t)a * n + b] = bx; bwx[(size_t)b * n + a] = bx;
    }
    int *host = (int *)malloc(sizeof(int) * n);
    int *ca = (int *)malloc(sizeof(int) * n), *ra = (int *)malloc(sizeof(int) * n);
    or_path *paths = (or_path *)malloc(sizeof(or_path) * (size_t)n * n);
    int *npeer = (int *)calloc(n, sizeof(int));
    int *ph = (int *)malloc(sizeof(int) * n), *pbw = (int *)malloc(sizeof(int) * n);
    int *pbx = (int *)malloc(sizeof(int) * n);
    double *X = (double *)malloc(sizeof(double) * (size_t)OR_MAX_CRIT * N);
    int32_t *feas = (int32_t *)malloc(sizeof(int32_t) * N);
    double *score = (double *)malloc(sizeof(double) * N);
    cand *order = (cand *)malloc(sizeof(cand) * N);
    or_path *tmp = (or_path *)malloc(sizeof(or_path) * n);
    int status = 1, fail_i = -1;
    for (int i = 0; i < n; ++i) {
        int P = 0;
        for (int j = 0; j < i; ++j)
            if (bwm[(size_t)i * n + j]) {
                ph[P] = host[j]; pbw[P] = (int)bwm[(size_t)i * n + j]; pbx[P] = (int)bwx[(size_t)i * n + j]; P++;
            }
        or_step_scores(d, m, cpu[i], ram[i], P, ph, pbw, X, feas, score);
        if (dump) memcpy(dump + (size_t)i * N, score, sizeof(double) * N);
        for (int u = 0; u < N; ++u) { order[u].s = score[u]; order[u].u = u; }
        qsort(order, N, sizeof(cand), cmp_cand);
        /* own choice and the runner-up among commit-successful servers */
        int top1 = -1; double s1 = 0.0, s2 = -INFINITY;
        /* routing at the end of the request: a placement takes CPU and RAM only */
        const int Pc = m->route_end ? 0 : P;
        const int cx = cpu_max ? cpu_max[i] : cpu[i], rx = ram_max ? ram_max[i] : ram[i];
        for (int r = 0; r < N; ++r) {
            int u = order[r].u;
            if (!feas[u]) continue;
            int c_a, r_a;
            if (try_commit(d, u, cpu[i], cx, ram[i], rx, Pc, ph, pbw, pbx, tmp, &c_a, &r_a)) {
                undo_commit(d, u, c_a, r_a, Pc, tmp);
                if (top1 < 0) { top1 = u; s1 = order[r].s; if (!ref_gap) break; }
                else { s2 = order[r].s; break; }
            }
        }
        if (ref_host) ref_host[i] = top1;
        if (ref_top) ref_top[i] = top1 >= 0 ? s1 : 0.0;
        if (ref_gap) ref_gap[i] = top1 >= 0 ? s1 - s2 : 0.0;
        int take = top1;
        if (follow) {
            if ((follow[i] < 0) != (top1 < 0)) { status = -3; fail_i = i; break; }
            take = follow[i];
        }
        if (tie_low) {
            tie_low[i] = -1;
            for (int v = 0; take >= 0 && v < take && tie_low[i] < 0; ++v) {
                if (!feas[v]) continue;
                int same = 1;
                for (int c = 0; c < m->ncrit; ++c)
                    if (X[(size_t)c * N + v] != X[(size_t)c * N + take]) same = 0;
                int c_a, r_a;
                if (same && try_commit(d, v, cpu[i], cx, ram[i], rx, Pc, ph, pbw, pbx, tmp, &c_a, &r_a)) {
                    undo_commit(d, v, c_a, r_a, Pc, tmp);
                    tie_low[i] = v;
                }
            }
        }
        if (take < 0) { status = 0; fail_i = i; break; }
        if (!try_commit(d, take, cpu[i], cx, ram[i], rx, Pc, ph, pbw, pbx, paths + (size_t)i * n, ca + i, ra + i)) {
            status = -2; fail_i = i; break;
        }
        npeer[i] = Pc;
        host[i] = take;
        if (host_out) host_out[i] = take;
        if (score_out) score_out[i] = score[take];
    }
    if (status == 1 && m->route_end) {
        /* every pair's widest minimum-hop path on the residuals the placement
         * left, each pair on its own; then all minima at once, and the
         * request fits only if no link goes negative; then each pair, in
         * order, is topped up towards its maximum */
        for (int i = 0; i < n; ++i) {
            int P = 0;
            for (int j = 0; j < i; ++j) {
                if (!bwm[(size_t)i * n + j]) continue;
                or_path *pp = paths + (size_t)i * n + P;
                pp->nl = 0; pp->bw = bwx[(size_t)i * n + j];
                if (host[j] != host[i]) {
                    int64_t b; int32_t links[6], hops;
                    or_widest_enum(d, host[i], host[j], &b, links, &hops);
                    pp->nl = hops;
                    pp->bw = bwm[(size_t)i * n + j];
                    for (int l = 0; l < hops; ++l) pp->link[l] = links[l];
                }
                P++;
            }
            npeer[i] = P;
        }
        int fits = 1;
        for (int i = 0; i < n; ++i)
            for (int p = 0; p < npeer[i]; ++p) {
                const or_path *pp = paths + (size_t)i * n + p;
                for (int l = 0; l < pp->nl; ++l) d->link_res[pp->link[l]] -= pp->bw;
            }
        for (int e = 0; e < 3 * N; ++e) if (d->link_res[e] < 0) fits = 0;
        if (!fits) { status = 0; fail_i = n; }
        else
            for (int i = 0; i < n; ++i) {
                int P = 0;
                for (int j = 0; j < i; ++j)
                    if (bwm[(size_t)i * n + j]) top_up(d, paths + (size_t)i * n + P++, bwx[(size_t)i * n + j]);
            }
    }
    if (status != 1) {
        for (int i = fail_i - 1; i >= 0; --i)
            undo_commit(d, host[i], ca[i], ra[i], npeer[i], paths + (size_t)i * n);
        if (host_out) for (int i = 0; i < n; ++i) host_out[i] = -1;
    }
    if (failed_at) *failed_at = fail_i;
    if (rec_id) *rec_id = -1;
    if (status == 1) {
        if (d->nrec == d->caprec) {
            d->caprec = d->caprec ? 2 * d->caprec : 64;
            d->rec = (or_record *)realloc(d->rec, sizeof(or_record) * d->caprec);
        }
        or_record *R = &d->rec[d->nrec];
        R->id = d->nrec; R->n = n; R->live = 1;
        R->host = (int *)malloc(sizeof(int) * n); R->cpu = (int *)malloc(sizeof(int) * n);
        R->ram = (int *)malloc(sizeof(int) * n);
        int np = 0;
        for (int i = 0; i < n; ++i) np += npeer[i];
        R->npath = np;
        R->plink = (int *)malloc(sizeof(int) * 6 * (np ? np : 1));
        R->pbw = (int64_t *)malloc(sizeof(int64_t) * (np ? np : 1));
        int q = 0;
        for (int i = 0; i < n; ++i) {
            R->host[i] = host[i]; R->cpu[i] = ca[i]; R->ram[i] = ra[i];
            if (cpu_a) cpu_a[i] = ca[i];
            if (ram_a) ram_a[i] = ra[i];
            for (int p = 0; p < npeer[i]; ++p, ++q) {
                const or_path *pp = paths + (size_t)i * n + p;
                R->pbw[q] = pp->bw;
                for (int l = 0; l < 6; ++l) R->plink[6 * q + l] = l < pp->nl ? pp->link[l] : -1;
            }
        }
        if (rec_id) *rec_id = R->id;
        d->nrec++;
        /* per edge: the allocation of its pair's path (peers ascending) */
        if (bw_a)
            for (int e = 0; e < ne; ++e) {
                int a = edges[3 * e], b = edges[3 * e + 1];
                int hi = a > b ? a : b, lo = a > b ? b : a, p = 0;
                for (int j = 0; j < lo; ++j) p += bwm[(size_t)hi * n + j] != 0;
                bw_a[e] = (int32_t)paths[(size_t)hi * n + p].bw;
            }
    }
    free(bwm); free(bwx); free(host); free(ca); free(ra); free(paths); free(npeer); free(ph); free(pbw); free(pbx);
    free(X); free(feas); free(score); free(order); free(tmp);
    return status;
}

/* Pods (section II-A, Eq. (8)): the containers of a pod must share one
 * server.  The oracle schedules a request with pods as a request of pods:
 * pod g, in the order of its first container (a container without a pod,
 * pod[i] < 0, being a pod of its own), asks for the summed CPU and RAM of
 * its containers, and the traffic between two pods, summed over their
 * container pairs, is one demand between the two servers; traffic inside a
 * pod needs no link.  or_units numbers the pods: unit[i] = pod of container
 * i, first[g] = smallest container of pod g; returns the number of pods. */
int or_units(int n, const int32_t *pod, int32_t *unit, int32_t *first) {
    int nu = 0;
    for (int i = 0; i < n; ++i) {
        unit[i] = -1;
        if (pod && pod[i] >= 0)
            for (int j = 0; j < i; ++j)
                if (pod[j] == pod[i]) { unit[i] = unit[j]; break; }
        if (unit[i] < 0) { first[nu] = i; unit[i] = nu++; }
    }
    return nu;
}

/* or_run_request on the pods of a request.  follow, ref_host, ref_top,
 * ref_gap and dump are per pod (its step); host_out and score_out are per
 * container (the pod's server and score); *failed_at is the first container
 * of the pod that found no server.  A pod's interval is the sum of its
 * containers' minima and maxima, and so is the traffic between two pods.
 * What a pod is given goes back to its containers in container order: each
 * first gets its minimum, then the rest up to each one's maximum in turn;
 * likewise a pod pair's bandwidth over its edges in edge order.  An edge
 * inside a pod, or between pods on one server, uses no link and gets its
 * maximum.  Returns as or_run_request, or -1 when a summed demand exceeds
 * the capacity bound 2^22. */
static void split_alloc(int64_t a, int cnt, const int *idx, const int32_t *mn, const int32_t *mx, int32_t *out) {
    for (int x = 0; x < cnt; ++x) { out[idx[x]] = mn[idx[x]]; a -= mn[idx[x]]; }
    for (int x = 0; x < cnt; ++x) {
        int64_t room = (int64_t)mx[idx[x]] - mn[idx[x]], t = a < room ? a : room;
        out[idx[x]] += (int32_t)t; a -= t;
    }
}

int or_run_request_pods(or_dc *d, const or_method *m, int n, const int32_t *cpu, const int32_t *ram,
                        int ne, const int32_t *edges, const int32_t *cpu_max, const int32_t *ram_max,
                        const int32_t *bw_max, const int32_t *pod, const int32_t *follow,
                        int32_t *host_out, double *score_out, int32_t *ref_host, double *ref_top,
                        double *ref_gap, double *dump, int32_t *failed_at, int64_t *rec_id,
                        int32_t *cpu_a, int32_t *ram_a, int32_t *bw_a, int32_t *tie_low) {
    if (n <= 0) return -1;
    int32_t *unit = (int32_t *)malloc(sizeof(int32_t) * n), *first = (int32_t *)malloc(sizeof(int32_t) * n);
    int nu = or_units(n, pod, unit, first);
    int64_t *ucpu = (int64_t *)calloc(nu, sizeof(int64_t)), *uram = (int64_t *)calloc(nu, sizeof(int64_t));
    int64_t *ucx = (int64_t *)calloc(nu, sizeof(int64_t)), *urx = (int64_t *)calloc(nu, sizeof(int64_t));
    int64_t *ubw = (int64_t *)calloc((size_t)nu * nu, sizeof(int64_t));
    int64_t *ubx = (int64_t *)calloc((size_t)nu * nu, sizeof(int64_t));
    int32_t *cu = (int32_t *)malloc(sizeof(int32_t) * nu), *ru = (int32_t *)malloc(sizeof(int32_t) * nu);
    int32_t *cux = (int32_t *)malloc(sizeof(int32_t) * nu), *rux = (int32_t *)malloc(sizeof(int32_t) * nu);
    int32_t *cua = (int32_t *)malloc(sizeof(int32_t) * nu), *rua = (int32_t *)malloc(sizeof(int32_t) * nu);
    const int mcap = nu * (nu - 1) / 2 + 1;
    int32_t *ue = (int32_t *)malloc(sizeof(int32_t) * 3 * (size_t)mcap);
    int32_t *uex = (int32_t *)malloc(sizeof(int32_t) * (size_t)mcap), *uea = (int32_t *)malloc(sizeof(int32_t) * (size_t)mcap);
    int32_t *hu = (int32_t *)malloc(sizeof(int32_t) * nu);
    int *idx = (int *)malloc(sizeof(int) * (size_t)(n > ne ? n : ne) + sizeof(int));
    double *su = (double *)calloc(nu, sizeof(double));
    for (int g = 0; g < nu; ++g) hu[g] = -1;
    int st = -1, fu = -1, mu = 0;
    for (int i = 0; i < n; ++i) {
        int cx = cpu_max ? cpu_max[i] : cpu[i], rx = ram_max ? ram_max[i] : ram[i];
        if (cx < cpu[i] || rx < ram[i]) goto done;
        ucpu[unit[i]] += cpu[i]; uram[unit[i]] += ram[i];
        ucx[unit[i]] += cx; urx[unit[i]] += rx;
    }
    for (int e = 0; e < ne; ++e) {
        int a = edges[3 * e], b = edges[3 * e + 1], bx = bw_max ? bw_max[e] : edges[3 * e + 2];
        if (a < 0 || b < 0 || a >= n || b >= n || a == b || edges[3 * e + 2] <= 0 || bx < edges[3 * e + 2]) goto done;
        a = unit[a]; b = unit[b];
        if (a == b) continue;                       /* inside a pod */
        ubw[(size_t)a * nu + b] += edges[3 * e + 2];
        ubw[(size_t)b * nu + a] += edges[3 * e + 2];
        ubx[(size_t)a * nu + b] += bx;
        ubx[(size_t)b * nu + a] += bx;
    }
    for (int g = 0; g < nu; ++g) {
        if (ucx[g] > (1 << 22) || urx[g] > (1 << 22)) goto done;
        cu[g] = (int32_t)ucpu[g]; ru[g] = (int32_t)uram[g];
        cux[g] = (int32_t)ucx[g]; rux[g] = (int32_t)urx[g];
        for (int h = g + 1; h < nu; ++h) {
            int64_t w = ubw[(size_t)g * nu + h], wx = ubx[(size_t)g * nu + h];
            if (wx > (1 << 22)) goto done;
            if (w > 0) {
                ue[3 * mu] = g; ue[3 * mu + 1] = h; ue[3 * mu + 2] = (int32_t)w; uex[mu] = (int32_t)wx; mu++;
            }
        }
    }
    st = or_run_request(d, m, nu, cu, ru, mu, ue, cux, rux, uex, follow, hu, su, ref_host, ref_top, ref_gap, dump,
                        &fu, rec_id, cua, rua, uea, tie_low);
    for (int i = 0; i < n; ++i) {
        if (host_out) host_out[i] = st == 1 ? hu[unit[i]] : -1;
        if (score_out) score_out[i] = su[unit[i]];
    }
    if (st == 1) {
        for (int g = 0; g < nu; ++g) {
            int cnt = 0;
            for (int i = 0; i < n; ++i) if (unit[i] == g) idx[cnt++] = i;
            if (cpu_a) split_alloc(cua[g], cnt, idx, cpu, cpu_max ? cpu_max : cpu, cpu_a);
            if (ram_a) split_alloc(rua[g], cnt, idx, ram, ram_max ? ram_max : ram, ram_a);
        }
        if (bw_a) {
            int32_t *emin = (int32_t *)malloc(sizeof(int32_t) * (size_t)(ne ? ne : 1));
            int32_t *emax = (int32_t *)malloc(sizeof(int32_t) * (size_t)(ne ? ne : 1));
            for (int e = 0; e < ne; ++e) {
                emin[e] = edges[3 * e + 2]; emax[e] = bw_max ? bw_max[e] : edges[3 * e + 2];
                bw_a[e] = emax[e];                  /* inside a pod: no link */
            }
            for (int q = 0; q < mu; ++q) {
                int cnt = 0;
                for (int e = 0; e < ne; ++e) {
                    int a = unit[edges[3 * e]], b = unit[edges[3 * e + 1]];
                    if ((a == ue[3 * q] && b == ue[3 * q + 1]) || (b == ue[3 * q] && a == ue[3 * q + 1])) idx[cnt++] = e;
                }
                split_alloc(uea[q], cnt, idx, emin, emax, bw_a);
            }
            free(emin); free(emax);
        }
    }
    if (failed_at) *failed_at = fu < 0 ? -1 : fu < nu ? first[fu] : n;   /* nu: the links did not fit */
done:
    free(unit); free(first); free(ucpu); free(uram); free(ucx); free(urx); free(ubw); free(ubx);
    free(cu); free(ru); free(cux); free(rux); free(cua); free(rua); free(ue); free(uex); free(uea); free(hu);
    free(idx); free(su);
    return st;
}

/* Departure of an accepted request: every CPU, RAM and link amount it
 * holds is given back.  Returns 0, or -1 for an unknown / released id. */
int or_release(or_dc *d, int64_t id) {
    if (id < 0 || id >= d->nrec || !d->rec[id].live) return -1;
    or_record *R = &d->rec[id];
    for (int q = 0; q < R->npath; ++q)
        for (int l = 0; l < 6; ++l)
            if (R->plink[6 * q + l] >= 0) d->link_res[R->plink[6 * q + l]] += R->pbw[q];
    for (int i = 0; i < R->n; ++i) {
        d->cpu_res[R->host[i]] += R->cpu[i];
        d->ram_res[R->host[i]] += R->ram[i];
        d->nplaced[R->host[i]] -= 1;
    }
    R->live = 0;
    return 0;
}

/* Links of the accepted request's routed pairs, 6 per pair, -1 padded, in
 * container order then peer order. */
int or_get_paths(const or_dc *d, int64_t id, int cap, int32_t *links, int64_t *bw) {
    if (id < 0 || id >= d->nrec) return -1;
    const or_record *R = &d->rec[id];
    int np = R->npath < cap ? R->npath : cap;
    for (int q = 0; q < np; ++q) {
        for (int l = 0; l < 6; ++l) links[6 * q + l] = R->plink[6 * q + l];
        if (bw) bw[q] = R->pbw[q];
    }
    return R->npath;
}

int or_get_hosts(const or_dc *d, int64_t id, int32_t *hosts) {
    if (id < 0 || id >= d->nrec) return -1;
    for (int i = 0; i < d->rec[id].n; ++i) hosts[i] = d->rec[id].host[i];
    return d->rec[id].n;
}
