/*
 * CPU ORACLE -- test infrastructure only.
 *
 * Plain, slow, obviously correct reference for the sample-based closeness
 * estimators of Cohen, Delling, Pajor & Werneck, "Computing Classic Closeness
 * Centrality, at Scale" (2014).  Only the test suite, the smoke check and the
 * CPU-baseline leg of the benchmark may build, load or call this code; the GPU
 * library neither links nor calls it, and it shares no code with the GPU
 * library.
 *
 * Contents
 *   orc_bfs / orc_dijkstra      single-source distances (Sec. 3: one
 *                               shortest-path computation per sampled node);
 *                               FIFO-queue BFS for unit lengths, binary-heap
 *                               Dijkstra for positive integer arc lengths.
 *   orc_sample_distances        D[v][i] = d(c_i, v) for every node and sample,
 *                               or the round-trip distance d(c_i,v)+d(v,c_i)
 *                               on a strongly connected digraph (Sec. 6.1).
 *   orc_node_estimates          the estimators for ONE node written out from
 *                               their definitions (Sec. 2): pivot and its
 *                               distance, sample average Eq. (5), pivot
 *                               estimate and pivoting upper bound, and the
 *                               hybrid estimate Eq. (6) by an explicit walk
 *                               over every node u of V \ {v} that places u in
 *                               L(v), HC(v) or H(v).
 *                               It also gives the estimated squared error of
 *                               the hybrid estimate (Sec. 4.1).
 *   orc_node_adaptive           the adaptive choice of Sec. 4 / Sec. 8: the
 *                               hybrid estimate for each eps of a list, the
 *                               one with the smallest estimated error kept.
 *   orc_node_sweep              Algorithm 2 / Sec. 4.2: the threshold sweep over
 *                               the pivot's distances to the samples, the
 *                               candidate with the smallest estimated error.
 *   orc_estimate_all            the above for every node, O(n^2): small graphs.
 *   orc_estimate_tails          every node at any size with Algorithm 1's
 *                               accounting (tail sums per pivot sample instead
 *                               of a walk over V per node), O(nk + kn log n);
 *                               the same values as orc_estimate_all.
 *   orc_exact_sums              S(v) for every node by n searches (Eq. (1)).
 *   orc_beta_all                Sec. 5 / Algorithm 3: the node-weighted hybrid
 *                               estimate of S_beta(v) = sum_u beta(u) d(v,u) and its
 *                               variance estimate, by the literal walk over
 *                               V \ {v} with beta-weighted terms and adjusted
 *                               weights on L cap C.
 *   orc_reach_beta              Sec. 6.2 / Algorithm 5: node-weighted reachability
 *                               sampling with priority ranks, from its definition.
 *   orc_reach_all               Sec. 6.2 / Algorithm 4 from its definition:
 *                               for every node v, one full search from v, then
 *                               the k reached nodes u != v first in a random
 *                               order of V (bottom-k sample of the reachability
 *                               set), their distance sum, the position of the
 *                               k-th among V \ {v}, and the average-distance and
 *                               reachability estimates.
 *
 * Readings of the paper used here:
 *   - pivot ties go to the lowest sample index (Alg. 2 updates the pivot only
 *     on a strictly smaller distance while scanning samples in index order);
 *   - u is in L(v) iff d(c(v),u) <= Delta(v)/eps, compared exactly as
 *     d*eps_num <= Delta*eps_den with eps = eps_num/eps_den in (0, 1];
 *   - for v in C every estimator returns the exact S(v) (Sec. 2);
 *   - the sample average is reported as a sum: S_samp = (n-1)/k * sum_i d;
 *   - the hybrid value is the rational N/|L cap C| with
 *     N = (sum_H + sum_HC)*|L cap C| + |L|*sum_{L cap C}, rounded once to
 *     double (N is checked to be below 2^53 so the conversion is exact).
 */
#include <math.h>
#include <pthread.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define ORC_OK 0
#define ORC_EINVAL 1
#define ORC_EUNREACHED 2
#define ORC_ENOMEM 3
#define ORC_EOVERFLOW 4

/* ------------------------------------------------------------------------ */
/* Breadth-first search: dist[v] = number of arcs on a shortest path from src,
 * -1 if unreachable.  Returns the largest finite distance. */
int64_t orc_bfs(int64_t n, const int64_t* rp, const int32_t* col, int32_t src, int64_t* dist) {
    int32_t* queue = (int32_t*)malloc(sizeof(int32_t) * (size_t)(n > 0 ? n : 1));
    if (!queue) return -1;
    for (int64_t v = 0; v < n; v++) dist[v] = -1;
    int64_t head = 0, tail = 0, maxd = 0;
    dist[src] = 0;
    queue[tail++] = src;
    while (head < tail) {
        int32_t v = queue[head++];
        int64_t dv = dist[v];
        if (dv > maxd) maxd = dv;
        for (int64_t e = rp[v]; e < rp[v + 1]; e++) {
            int32_t u = col[e];
            if (dist[u] < 0) {
                dist[u] = dv + 1;
                queue[tail++] = u;
            }
        }
    }
    free(queue);
    return maxd;
}

/* Dijkstra's algorithm with a binary min-heap keyed by tentative distance
 * (lazy deletion: stale heap entries are skipped when popped). */
typedef struct { int64_t d; int32_t v; } orc_item;

static void heap_push(orc_item* h, int64_t* size, orc_item it) {
    int64_t i = (*size)++;
    while (i > 0) {
        int64_t p = (i - 1) / 2;
        if (h[p].d <= it.d) break;
        h[i] = h[p];
        i = p;
    }
    h[i] = it;
}

static orc_item heap_pop(orc_item* h, int64_t* size) {
    orc_item top = h[0];
    orc_item last = h[--(*size)];
    int64_t i = 0;
    for (;;) {
        int64_t l = 2 * i + 1, r = l + 1, m = i;
        int64_t dm = last.d;
        if (l < *size && h[l].d < dm) { m = l; dm = h[l].d; }
        if (r < *size && h[r].d < dm) { m = r; }
        if (m == i) break;
        h[i] = h[m];
        i = m;
    }
    if (*size > 0) h[i] = last;
    return top;
}

int64_t orc_dijkstra(int64_t n, const int64_t* rp, const int32_t* col, const int32_t* w, int32_t src,
                     int64_t* dist) {
    int64_t arcs = rp[n];
    orc_item* heap = (orc_item*)malloc(sizeof(orc_item) * (size_t)(arcs + 2));
    char* done = (char*)calloc((size_t)(n > 0 ? n : 1), 1);
    if (!heap || !done) { free(heap); free(done); return -1; }
    for (int64_t v = 0; v < n; v++) dist[v] = -1;
    int64_t size = 0, maxd = 0;
    dist[src] = 0;
    orc_item s0 = {0, src};
    heap_push(heap, &size, s0);
    while (size > 0) {
        orc_item it = heap_pop(heap, &size);
        int32_t v = it.v;
        if (done[v]) continue;
        done[v] = 1;
        if (it.d > maxd) maxd = it.d;
        for (int64_t e = rp[v]; e < rp[v + 1]; e++) {
            int32_t u = col[e];
            int64_t nd = it.d + (int64_t)w[e];
            if (!done[u] && (dist[u] < 0 || nd < dist[u])) {
                dist[u] = nd;
                orc_item x = {nd, u};
                heap_push(heap, &size, x);
            }
        }
    }
    free(heap); free(done);
    return maxd;
}

/* one search; w == NULL selects BFS */
static int64_t sssp(int64_t n, const int64_t* rp, const int32_t* col, const int32_t* w, int32_t src,
                    int64_t* dist) {
    return w ? orc_dijkstra(n, rp, col, w, src, dist) : orc_bfs(n, rp, col, src, dist);
}

/* ------------------------------------------------------------------------ */
/* Distances from every sample.  D is node-major: D[v*k + i] = d(c_i, v).
 * If rrp != NULL the graph is a digraph and (rrp, rcol, rw) is its transpose;
 * then D holds round-trip distances d(c_i -> v) + d(v -> c_i), the second term
 * being the distance from c_i in the transposed graph.
 * Returns ORC_EUNREACHED if some node is unreachable from some sample. */
typedef struct {
    int64_t n; const int64_t* rp; const int32_t* col; const int32_t* w;
    const int64_t* rrp; const int32_t* rcol; const int32_t* rw;
    int32_t k; const int32_t* samples; int64_t* D;
    int32_t next; pthread_mutex_t lock; int status;
} dist_job;

static void* dist_worker(void* arg) {
    dist_job* J = (dist_job*)arg;
    int64_t* a = (int64_t*)malloc(sizeof(int64_t) * (size_t)J->n);
    int64_t* b = J->rrp ? (int64_t*)malloc(sizeof(int64_t) * (size_t)J->n) : NULL;
    if (!a || (J->rrp && !b)) {
        pthread_mutex_lock(&J->lock); J->status = ORC_ENOMEM; pthread_mutex_unlock(&J->lock);
        free(a); free(b); return NULL;
    }
    for (;;) {
        pthread_mutex_lock(&J->lock);
        int32_t i = J->next++;
        pthread_mutex_unlock(&J->lock);
        if (i >= J->k) break;
        sssp(J->n, J->rp, J->col, J->w, J->samples[i], a);
        if (b) sssp(J->n, J->rrp, J->rcol, J->rw, J->samples[i], b);
        int bad = 0;
        for (int64_t v = 0; v < J->n; v++) {
            int64_t d = a[v];
            if (d < 0 || (b && b[v] < 0)) { bad = 1; d = -1; }
            else if (b) d += b[v];
            J->D[v * J->k + i] = d;
        }
        if (bad) { pthread_mutex_lock(&J->lock); J->status = ORC_EUNREACHED; pthread_mutex_unlock(&J->lock); }
    }
    free(a); free(b);
    return NULL;
}

int orc_sample_distances(int64_t n, const int64_t* rp, const int32_t* col, const int32_t* w,
                         const int64_t* rrp, const int32_t* rcol, const int32_t* rw,
                         int32_t k, const int32_t* samples, int32_t threads, int64_t* D) {
    dist_job J;
    J.n = n; J.rp = rp; J.col = col; J.w = w; J.rrp = rrp; J.rcol = rcol; J.rw = rw;
    J.k = k; J.samples = samples; J.D = D; J.next = 0; J.status = ORC_OK;
    pthread_mutex_init(&J.lock, NULL);
    if (threads < 1) threads = 1;
    if (threads == 1) {
        dist_worker(&J);
    } else {
        pthread_t* th = (pthread_t*)malloc(sizeof(pthread_t) * (size_t)threads);
        for (int32_t t = 0; t < threads; t++) pthread_create(&th[t], NULL, dist_worker, &J);
        for (int32_t t = 0; t < threads; t++) pthread_join(th[t], NULL);
        free(th);
    }
    pthread_mutex_destroy(&J.lock);
    return J.status;
}

/* ------------------------------------------------------------------------ */
/* Estimates for one node v, from the definitions of Sec. 2.
 *
 *   row[i]          = d(v, c_i), i = 0..k-1 (distances to the samples)
 *   colp[u*stride]  = d(c_p, u) for every node u, where p is the pivot of v;
 *                     the caller finds p with orc_pivot(row) first.
 *   sidx[u]         = index i with c_i = u, or -1 when u is not sampled.
 *
 * The walk over u in V \ {v} is the partition of Sec. 2 written out:
 *   d(c_p,u) <= Delta/eps  ->  u in L(v)   (u in C: also in L cap C)
 *   otherwise, u in C      ->  u in HC(v), contributes d(v,u) exactly
 *   otherwise              ->  u in H(v),  contributes d(c_p,u)
 */
typedef struct {
    int32_t pivot;      /* sample index of c(v) */
    int64_t delta;      /* Delta(v) = d(v, c(v)) */
    int64_t sampsum;    /* sum_i d(v, c_i) */
    int64_t S_piv;      /* pivot estimate S(c(v)) */
    int64_t S_pub;      /* pivoting upper bound S(c(v)) + (n-1) Delta(v) */
    double S_samp;      /* sample-average estimate, as a sum */
    double S_hyb;       /* hybrid estimate Eq. (6) */
    /* the parts of Eq. (6), for inspection */
    int64_t L_num, LC_num, HC_num, H_num;
    int64_t LC_sum, HC_sum, H_sum;
    int64_t N;          /* numerator of S_hyb = N / LC_num */
    int32_t overflow;   /* N or (n-1)*sampsum reached 2^53 */
    int32_t sampled;    /* v is in C */
    /* Sec. 4.1, the estimated squared error of S_hyb */
    int64_t LC_sumsq;   /* sum over L cap C of d(v,u)^2 */
    int64_t HC_sqerr;   /* sum over HC of (d(v,u) - d(c(v),u))^2 */
    double S_err;       /* |L|/|L cap C| * sample variance over L cap C + |H| * HC_sqerr/|HC| */
} orc_node_out;

int32_t orc_pivot(int32_t k, const int64_t* row) {
    int32_t p = 0;
    for (int32_t i = 1; i < k; i++)
        if (row[i] < row[p]) p = i; /* strict: ties keep the lower index */
    return p;
}

/* Sec. 4.1: when HC(v) is empty the mean squared pivoting error is taken
 * over a "suffix" of the farthest samples instead; read here as the samples at
 * the largest distance from the pivot (all of them when they tie).  Returns
 * the sum of (d(v,u) - d(c(v),u))^2 over those samples and their number, by a
 * walk over every node u that picks out the sampled ones. */
static __int128 far_suffix_sqerr(int64_t n, const int32_t* sidx, const int64_t* row, const int64_t* colp,
                                 int64_t stride, int64_t* count) {
    int64_t far = -1;
    for (int64_t u = 0; u < n; u++)
        if (sidx[u] >= 0 && colp[u * stride] > far) far = colp[u * stride];
    __int128 sq = 0;
    *count = 0;
    for (int64_t u = 0; u < n; u++) {
        int32_t i = sidx[u];
        if (i < 0 || colp[u * stride] != far) continue;
        sq += (__int128)(row[i] - far) * (row[i] - far);
        (*count)++;
    }
    return sq;
}

int orc_node_estimates(int64_t n, int32_t k, int64_t v, const int32_t* sidx, const int64_t* row,
                       const int64_t* colp, int64_t stride, int64_t eps_num, int64_t eps_den,
                       orc_node_out* out) {
    const int64_t LIM = (int64_t)1 << 53;
    memset(out, 0, sizeof(*out));
    int32_t p = orc_pivot(k, row);
    int64_t delta = row[p];
    int64_t sampsum = 0;
    for (int32_t i = 0; i < k; i++) sampsum += row[i];
    int64_t Sp = 0; /* S(c_p) = sum over all u of d(c_p, u) */
    for (int64_t u = 0; u < n; u++) Sp += colp[u * stride];
    out->pivot = p;
    out->delta = delta;
    out->sampsum = sampsum;
    if (sidx[v] >= 0) {
        /* v = c_j is its own pivot and its distances to all nodes are known */
        out->sampled = 1;
        out->S_piv = out->S_pub = Sp;
        out->S_samp = out->S_hyb = (double)Sp;
        out->N = Sp; out->LC_num = 1;
        out->overflow = Sp >= LIM;
        return Sp >= LIM ? ORC_EOVERFLOW : ORC_OK;
    }
    out->S_piv = Sp;
    out->S_pub = Sp + (n - 1) * delta;
    int64_t ss = (n - 1) * sampsum;
    out->S_samp = (double)ss / (double)k;
    int64_t Lnum = 0, LCnum = 0, HCnum = 0, Hnum = 0, LCsum = 0, HCsum = 0, Hsum = 0;
    __int128 LCsumsq = 0, HCsqerr = 0;
    for (int64_t u = 0; u < n; u++) {
        if (u == v) continue;
        int64_t dpu = colp[u * stride];
        int in_L = dpu * eps_num <= delta * eps_den;
        int32_t i = sidx[u];
        if (in_L) {
            Lnum++;
            if (i >= 0) { LCnum++; LCsum += row[i]; LCsumsq += (__int128)row[i] * row[i]; }
        } else if (i >= 0) {
            HCnum++; HCsum += row[i];
            HCsqerr += (__int128)(row[i] - dpu) * (row[i] - dpu);
        } else {
            Hnum++; Hsum += dpu;
        }
    }
    out->L_num = Lnum; out->LC_num = LCnum; out->HC_num = HCnum; out->H_num = Hnum;
    out->LC_sum = LCsum; out->HC_sum = HCsum; out->H_sum = Hsum;
    /* LCnum >= 1 always: the pivot is in L cap C when eps <= 1 */
    if (LCnum < 1) { out->S_hyb = -1.0; return ORC_EOVERFLOW; }
    /* Sec. 4.1: the sampling part estimates the variance of the L distances by
     * the sample variance over L cap C (sum of squares / count minus squared
     * mean), divided by |L cap C| and scaled by |L|; the pivoting part takes
     * the mean squared difference over HC and scales it by |H|; with HC empty
     * the mean is over the farthest samples (far_suffix_sqerr).  Written with
     * the exact integer LCnum * LCsumsq - LCsum^2 and a fixed order of double
     * operations. */
    __int128 varnum = (__int128)LCnum * LCsumsq - (__int128)LCsum * LCsum;
    int64_t sqcnt = HCnum;
    __int128 sqsum = HCsqerr;
    if (HCnum == 0) sqsum = far_suffix_sqerr(n, sidx, row, colp, stride, &sqcnt);
    int err_ovf = LCsumsq > (__int128)INT64_MAX || sqsum > (__int128)INT64_MAX || varnum > (__int128)INT64_MAX;
    out->LC_sumsq = (int64_t)LCsumsq;
    out->HC_sqerr = (int64_t)HCsqerr;
    {
        double tL = ((double)(int64_t)varnum / (double)(LCnum * LCnum * LCnum)) * (double)Lnum;
        double tH = ((double)(int64_t)sqsum / (double)sqcnt) * (double)Hnum;
        out->S_err = tL + tH;
    }
    /* S_hyb = Hsum + HCsum + Lnum * LCsum / LCnum = N / LCnum */
    __int128 N = (__int128)(Hsum + HCsum) * LCnum + (__int128)Lnum * LCsum;
    int ovf = (N >= (__int128)LIM) || (ss >= LIM) || err_ovf;
    out->N = (int64_t)N;
    out->S_hyb = (double)(int64_t)N / (double)LCnum;
    out->overflow = ovf;
    return ovf ? ORC_EOVERFLOW : ORC_OK;
}

/* Sec. 4 / Sec. 8 adaptive choice: the hybrid estimate for each eps of a
 * list, keeping the one with the smallest estimated squared error (the first
 * in list order on ties).  Sampled nodes: the exact S(v), error 0. */
int orc_node_adaptive(int64_t n, int32_t k, int64_t v, const int32_t* sidx, const int64_t* row,
                      const int64_t* colp, int64_t stride, const int64_t* eps_nums, const int64_t* eps_dens,
                      int32_t n_eps, double* S_ad, double* S_ad_err, int32_t* which) {
    int status = ORC_OK;
    *which = -1;
    for (int32_t e = 0; e < n_eps; e++) {
        orc_node_out o;
        int st = orc_node_estimates(n, k, v, sidx, row, colp, stride, eps_nums[e], eps_dens[e], &o);
        if (st != ORC_OK) status = st;
        if (o.sampled) { *S_ad = o.S_hyb; *S_ad_err = 0.0; *which = 0; return status; }
        if (*which < 0 || o.S_err < *S_ad_err) { *S_ad = o.S_hyb; *S_ad_err = o.S_err; *which = e; }
    }
    return status;
}

/* Sec. 4.2 / Algorithm 2, the threshold sweep: candidates are pure pivoting
 * (S(c(v)), with the mean squared pivot error over all k samples times the
 * n-1-k other unsampled nodes) and, for every distinct distance T from the
 * pivot to a sample, the estimate with the partition of V \ {v} into
 * L = {d(c(v),u) <= T}, HC and H as in Eq. (6) and its error as in Sec. 4.1.
 * The candidate with the smallest error is kept (a later candidate only when
 * strictly smaller, candidates in increasing T after pure pivoting).  Each
 * threshold is evaluated by a literal walk over the nodes. */
int orc_node_sweep(int64_t n, int32_t k, int64_t v, const int32_t* sidx, const int64_t* row, const int64_t* colp,
                   int64_t stride, double* S_out, double* err_out) {
    const int64_t LIM = (int64_t)1 << 53;
    int32_t p = orc_pivot(k, row);
    int64_t Sp = 0;
    for (int64_t u = 0; u < n; u++) Sp += colp[u * stride];
    if (sidx[v] >= 0) { *S_out = (double)Sp; *err_out = 0.0; return Sp >= LIM ? ORC_EOVERFLOW : ORC_OK; }
    /* d(c_p, c_i) for every sample i, from the pivot's column */
    int64_t* dp = (int64_t*)malloc(sizeof(int64_t) * (size_t)k);
    for (int64_t u = 0; u < n; u++) if (sidx[u] >= 0) dp[sidx[u]] = colp[u * stride];
    /* pure pivoting */
    __int128 sq_all = 0;
    for (int32_t i = 0; i < k; i++) sq_all += (__int128)(row[i] - dp[i]) * (row[i] - dp[i]);
    int ovf = Sp >= LIM || sq_all > (__int128)INT64_MAX;
    double best_S = (double)Sp;
    double best_err = ((double)(int64_t)sq_all / (double)k) * (double)(n - 1 - k);
    /* thresholds: the distinct values of dp, ascending */
    int64_t T = -1;
    for (;;) {
        int64_t next = -1;
        for (int32_t i = 0; i < k; i++)
            if (dp[i] > T && (next < 0 || dp[i] < next)) next = dp[i];
        if (next < 0) break;
        T = next;
        int64_t Lnum = 0, LCnum = 0, HCnum = 0, Hnum = 0, LCsum = 0, HCsum = 0, Hsum = 0;
        __int128 LCsumsq = 0, HCsqerr = 0;
        for (int64_t u = 0; u < n; u++) {
            if (u == v) continue;
            int64_t dpu = colp[u * stride];
            int32_t i = sidx[u];
            if (dpu <= T) {
                Lnum++;
                if (i >= 0) { LCnum++; LCsum += row[i]; LCsumsq += (__int128)row[i] * row[i]; }
            } else if (i >= 0) {
                HCnum++; HCsum += row[i];
                HCsqerr += (__int128)(row[i] - dpu) * (row[i] - dpu);
            } else {
                Hnum++; Hsum += dpu;
            }
        }
        if (LCnum < 1) continue; /* cannot happen: the pivot sample is at distance 0 */
        __int128 N = (__int128)(Hsum + HCsum) * LCnum + (__int128)Lnum * LCsum;
        __int128 varnum = (__int128)LCnum * LCsumsq - (__int128)LCsum * LCsum;
        int64_t sqcnt = HCnum;
        __int128 sqsum = HCsqerr;
        if (HCnum == 0) sqsum = far_suffix_sqerr(n, sidx, row, colp, stride, &sqcnt); /* Sec. 4.1's suffix */
        ovf = ovf || N >= (__int128)LIM || varnum > (__int128)INT64_MAX || sqsum > (__int128)INT64_MAX;
        double est = (double)(int64_t)N / (double)LCnum;
        double tL = ((double)(int64_t)varnum / (double)(LCnum * LCnum * LCnum)) * (double)Lnum;
        double tH = ((double)(int64_t)sqsum / (double)sqcnt) * (double)Hnum;
        double err = tL + tH;
        if (err < best_err) { best_err = err; best_S = est; }
    }
    free(dp);
    *S_out = best_S;
    *err_out = best_err;
    return ovf ? ORC_EOVERFLOW : ORC_OK;
}

/* All nodes of a small graph from the full distance matrix D (node-major,
 * n x k).  Output arrays have n entries; any may be NULL. Multithreaded over
 * nodes when threads > 1. */
typedef struct {
    int64_t n; int32_t k; const int32_t* sidx; const int64_t* D; int64_t en, ed;
    int32_t* pivot; int64_t* delta; int64_t* sampsum; int64_t* S_piv; int64_t* S_pub;
    double* S_samp; double* S_hyb; double* S_err;
    const int64_t* ad_nums; const int64_t* ad_dens; int32_t n_ad; double* S_ad; double* S_ad_err;
    double* S_sweep; double* S_sweep_err;
    int64_t next; pthread_mutex_t lock; int status;
} all_job;

static void* all_worker(void* arg) {
    all_job* J = (all_job*)arg;
    for (;;) {
        pthread_mutex_lock(&J->lock);
        int64_t v0 = J->next; J->next += 64;
        pthread_mutex_unlock(&J->lock);
        if (v0 >= J->n) break;
        int64_t v1 = v0 + 64 < J->n ? v0 + 64 : J->n;
        for (int64_t v = v0; v < v1; v++) {
            const int64_t* row = J->D + v * J->k;
            int32_t p = orc_pivot(J->k, row);
            orc_node_out o;
            int st = orc_node_estimates(J->n, J->k, v, J->sidx, row, J->D + p, J->k, J->en, J->ed, &o);
            if (st != ORC_OK) { pthread_mutex_lock(&J->lock); J->status = st; pthread_mutex_unlock(&J->lock); }
            if (J->pivot) J->pivot[v] = o.pivot;
            if (J->delta) J->delta[v] = o.delta;
            if (J->sampsum) J->sampsum[v] = o.sampsum;
            if (J->S_piv) J->S_piv[v] = o.S_piv;
            if (J->S_pub) J->S_pub[v] = o.S_pub;
            if (J->S_samp) J->S_samp[v] = o.S_samp;
            if (J->S_hyb) J->S_hyb[v] = o.S_hyb;
            if (J->S_err) J->S_err[v] = o.sampled ? 0.0 : o.S_err;
            if (J->S_ad && J->n_ad > 0) {
                double a = 0, ae = 0;
                int32_t w = 0;
                st = orc_node_adaptive(J->n, J->k, v, J->sidx, row, J->D + p, J->k, J->ad_nums, J->ad_dens, J->n_ad,
                                       &a, &ae, &w);
                if (st != ORC_OK) { pthread_mutex_lock(&J->lock); J->status = st; pthread_mutex_unlock(&J->lock); }
                J->S_ad[v] = a;
                if (J->S_ad_err) J->S_ad_err[v] = ae;
            }
            if (J->S_sweep) {
                double a = 0, ae = 0;
                st = orc_node_sweep(J->n, J->k, v, J->sidx, row, J->D + p, J->k, &a, &ae);
                if (st != ORC_OK) { pthread_mutex_lock(&J->lock); J->status = st; pthread_mutex_unlock(&J->lock); }
                J->S_sweep[v] = a;
                if (J->S_sweep_err) J->S_sweep_err[v] = ae;
            }
        }
    }
    return NULL;
}

int orc_estimate_all(int64_t n, int32_t k, const int32_t* sidx, const int64_t* D, int64_t eps_num,
                     int64_t eps_den, int32_t threads, int32_t* pivot, int64_t* delta, int64_t* sampsum,
                     int64_t* S_piv, int64_t* S_pub, double* S_samp, double* S_hyb, double* S_err,
                     const int64_t* ad_nums, const int64_t* ad_dens, int32_t n_ad, double* S_ad,
                     double* S_ad_err, double* S_sweep, double* S_sweep_err) {
    all_job J;
    J.n = n; J.k = k; J.sidx = sidx; J.D = D; J.en = eps_num; J.ed = eps_den;
    J.pivot = pivot; J.delta = delta; J.sampsum = sampsum; J.S_piv = S_piv; J.S_pub = S_pub;
    J.S_samp = S_samp; J.S_hyb = S_hyb; J.S_err = S_err;
    J.ad_nums = ad_nums; J.ad_dens = ad_dens; J.n_ad = n_ad; J.S_ad = S_ad; J.S_ad_err = S_ad_err;
    J.S_sweep = S_sweep; J.S_sweep_err = S_sweep_err;
    J.next = 0; J.status = ORC_OK;
    pthread_mutex_init(&J.lock, NULL);
    if (threads <= 1) {
        all_worker(&J);
    } else {
        pthread_t* th = (pthread_t*)malloc(sizeof(pthread_t) * (size_t)threads);
        for (int32_t t = 0; t < threads; t++) pthread_create(&th[t], NULL, all_worker, &J);
        for (int32_t t = 0; t < threads; t++) pthread_join(th[t], NULL);
        free(th);
    }
    pthread_mutex_destroy(&J.lock);
    return J.status;
}

/* ------------------------------------------------------------------------ */
/* Every node at any size, with Algorithm 1's accounting instead of a walk
 * over V per node (Sec. 3): the sums over H(v) come from the unsampled nodes'
 * distances to the pivot, kept per sample as a sorted list with suffix sums
 * ("tail sums for nodes for which c_i is pivot"); the samples are split into
 * L cap C and HC by d(c(v), c_i) against the threshold; |L| = n-1-|H|-|HC|.
 * The estimates and errors are then those of orc_node_estimates (the same
 * exact integers, the same order of double operations), and the adaptive
 * choice that of orc_node_adaptive.  D is node-major n x k with
 * D[u*k + i] = d(c_i, u); distances must be symmetric (undirected or round
 * trip).  Outputs have n entries (src_sum k, dmat k*k); any may be NULL. */
typedef struct {
    int64_t n; int32_t k; const int32_t* sidx; const int64_t* D; const int32_t* piv; const int64_t* bstart;
    const int32_t* bnodes; const int64_t* src_sum; const int64_t* dmat;
    const int64_t* nums; const int64_t* dens; int32_t n_eps;  /* entry 0: the call's eps; 1..: the list */
    int64_t* S_pub; double* S_samp; double* S_hyb; double* S_err; double* S_ad; double* S_ad_err;
    int32_t next; pthread_mutex_t lock; int status;
} tails_job;

static int cmp_i64(const void* a, const void* b) {
    int64_t x = *(const int64_t*)a, y = *(const int64_t*)b;
    return (x > y) - (x < y);
}

/* number of entries of the ascending list srt[0..m) that are > T */
static int64_t count_above(const int64_t* srt, int64_t m, int64_t T) {
    int64_t lo = 0, hi = m;  /* first index with srt[idx] > T */
    while (lo < hi) {
        int64_t mid = lo + (hi - lo) / 2;
        if (srt[mid] > T) hi = mid; else lo = mid + 1;
    }
    return m - lo;
}

static void* tails_worker(void* arg) {
    tails_job* J = (tails_job*)arg;
    const int64_t n = J->n, k = J->k;
    const __int128 LIM = (__int128)1 << 53;
    int64_t* srt = (int64_t*)malloc(sizeof(int64_t) * (size_t)(n + 1));
    int64_t* suf = (int64_t*)malloc(sizeof(int64_t) * (size_t)(n + 1));
    if (!srt || !suf) {
        pthread_mutex_lock(&J->lock); J->status = ORC_ENOMEM; pthread_mutex_unlock(&J->lock);
        free(srt); free(suf); return NULL;
    }
    for (;;) {
        pthread_mutex_lock(&J->lock);
        int32_t p = J->next++;
        pthread_mutex_unlock(&J->lock);
        if (p >= k) break;
        if (J->bstart[p] == J->bstart[p + 1]) continue;  /* no unsampled node has this pivot */
        /* the unsampled nodes' distances to c_p, ascending, with suffix sums */
        int64_t m = 0;
        for (int64_t u = 0; u < n; u++)
            if (J->sidx[u] < 0) srt[m++] = J->D[u * k + p];
        qsort(srt, (size_t)m, sizeof(int64_t), cmp_i64);
        suf[m] = 0;
        for (int64_t t = m - 1; t >= 0; t--) suf[t] = suf[t + 1] + srt[t];
        const int64_t* dp = J->dmat + (int64_t)p * k;  /* d(c_p, c_i) */
        int64_t far = 0;
        for (int32_t i = 0; i < k; i++) if (dp[i] > far) far = dp[i];
        for (int64_t b = J->bstart[p]; b < J->bstart[p + 1]; b++) {
            const int64_t v = J->bnodes[b];
            const int64_t* row = J->D + v * k;
            const int64_t delta = row[p];
            int ovf = 0;
            double ad = 0, ad_err = 0;
            for (int32_t e = 0; e < J->n_eps; e++) {
                const int64_t num = J->nums[e], den = J->dens[e];
                const int64_t T = delta * den / num;  /* d*num <= Delta*den  <=>  d <= T for integer d */
                const int64_t Hnum = count_above(srt, m, T);
                const int64_t Hsum = suf[m - Hnum];
                int64_t LCnum = 0, HCnum = 0, LCsum = 0, HCsum = 0;
                __int128 LCsumsq = 0, HCsqerr = 0, Fsq = 0;
                int64_t Fnum = 0;
                for (int32_t i = 0; i < k; i++) {
                    const int64_t d = row[i];
                    if (dp[i] * num <= delta * den) {
                        LCnum++; LCsum += d; LCsumsq += (__int128)d * d;
                    } else {
                        HCnum++; HCsum += d; HCsqerr += (__int128)(d - dp[i]) * (d - dp[i]);
                    }
                    if (dp[i] == far) { Fnum++; Fsq += (__int128)(d - dp[i]) * (d - dp[i]); }
                }
                const int64_t Lnum = n - 1 - Hnum - (k - LCnum);
                if (LCnum < 1 || Lnum < LCnum) { ovf = 1; continue; }
                __int128 N = (__int128)(Hsum + HCsum) * LCnum + (__int128)Lnum * LCsum;
                __int128 varnum = (__int128)LCnum * LCsumsq - (__int128)LCsum * LCsum;
                int64_t sqcnt = HCnum;
                __int128 sqsum = HCsqerr;
                if (HCnum == 0) { sqcnt = Fnum; sqsum = Fsq; }  /* Sec. 4.1's suffix of the farthest samples */
                ovf = ovf || N >= LIM || varnum > (__int128)INT64_MAX || sqsum > (__int128)INT64_MAX ||
                      LCsumsq > (__int128)INT64_MAX;
                const double est = (double)(int64_t)N / (double)LCnum;
                const double tL = ((double)(int64_t)varnum / (double)(LCnum * LCnum * LCnum)) * (double)Lnum;
                const double tH = ((double)(int64_t)sqsum / (double)sqcnt) * (double)Hnum;
                const double err = tL + tH;
                if (e == 0) {
                    if (J->S_hyb) J->S_hyb[v] = est;
                    if (J->S_err) J->S_err[v] = err;
                } else if (e == 1 || err < ad_err) {
                    ad = est; ad_err = err;
                }
            }
            if (J->S_ad && J->n_eps > 1) J->S_ad[v] = ad;
            if (J->S_ad_err && J->n_eps > 1) J->S_ad_err[v] = ad_err;
            if (ovf) { pthread_mutex_lock(&J->lock); J->status = ORC_EOVERFLOW; pthread_mutex_unlock(&J->lock); }
        }
    }
    free(srt); free(suf);
    return NULL;
}

int orc_estimate_tails(int64_t n, int32_t k, const int32_t* sidx, const int64_t* D, const int64_t* nums,
                       const int64_t* dens, int32_t n_eps, int32_t threads, int32_t* pivot, int64_t* delta,
                       int64_t* sampsum, int64_t* src_sum, int64_t* dmat, int64_t* S_piv, int64_t* S_pub,
                       double* S_samp, double* S_hyb, double* S_err, double* S_ad, double* S_ad_err) {
    const __int128 LIM = (__int128)1 << 53;
    int status = ORC_OK;
    /* S(c_i) = sum over every node of d(c_i, u); the sample distance matrix */
    for (int32_t i = 0; i < k; i++) src_sum[i] = 0;
    for (int64_t u = 0; u < n; u++) {
        const int64_t* row = D + u * k;
        for (int32_t i = 0; i < k; i++) src_sum[i] += row[i];
        if (sidx[u] >= 0)
            for (int32_t i = 0; i < k; i++) dmat[(int64_t)i * k + sidx[u]] = row[i];
    }
    /* per node: pivot (lowest index on ties), Delta, sampsum, and the
     * estimates that need nothing else; sampled nodes get their exact sum */
    int64_t* bstart = (int64_t*)calloc((size_t)k + 2, sizeof(int64_t));
    int32_t* bnodes = (int32_t*)malloc(sizeof(int32_t) * (size_t)(n > 0 ? n : 1));
    if (!bstart || !bnodes) { free(bstart); free(bnodes); return ORC_ENOMEM; }
    for (int64_t v = 0; v < n; v++) {
        const int64_t* row = D + v * k;
        int32_t p = orc_pivot(k, row);
        int64_t ss = 0;
        for (int32_t i = 0; i < k; i++) ss += row[i];
        pivot[v] = p; delta[v] = row[p]; sampsum[v] = ss;
        const int64_t Sp = src_sum[p];
        if (sidx[v] >= 0) {
            S_piv[v] = S_pub[v] = Sp;
            S_samp[v] = (double)Sp;
            if (S_hyb) S_hyb[v] = (double)Sp;
            if (S_err) S_err[v] = 0.0;
            if (S_ad) S_ad[v] = (double)Sp;
            if (S_ad_err) S_ad_err[v] = 0.0;
            if (Sp >= LIM) status = ORC_EOVERFLOW;
            continue;
        }
        S_piv[v] = Sp;
        S_pub[v] = Sp + (n - 1) * row[p];
        const __int128 x = (__int128)(n - 1) * ss;
        if (x >= LIM) status = ORC_EOVERFLOW;
        S_samp[v] = (double)(int64_t)x / (double)k;
        bstart[p + 1]++;
    }
    for (int32_t p = 0; p < k; p++) bstart[p + 1] += bstart[p];
    {
        int64_t* fill = (int64_t*)malloc(sizeof(int64_t) * (size_t)(k + 1));
        if (!fill) { free(bstart); free(bnodes); return ORC_ENOMEM; }
        memcpy(fill, bstart, sizeof(int64_t) * (size_t)(k + 1));
        for (int64_t v = 0; v < n; v++)
            if (sidx[v] < 0) bnodes[fill[pivot[v]]++] = (int32_t)v;
        free(fill);
    }
    tails_job J;
    J.n = n; J.k = k; J.sidx = sidx; J.D = D; J.piv = pivot; J.bstart = bstart; J.bnodes = bnodes;
    J.src_sum = src_sum; J.dmat = dmat; J.nums = nums; J.dens = dens; J.n_eps = n_eps;
    J.S_pub = S_pub; J.S_samp = S_samp; J.S_hyb = S_hyb; J.S_err = S_err; J.S_ad = S_ad; J.S_ad_err = S_ad_err;
    J.next = 0; J.status = ORC_OK;
    pthread_mutex_init(&J.lock, NULL);
    if (threads <= 1) {
        tails_worker(&J);
    } else {
        pthread_t* th = (pthread_t*)malloc(sizeof(pthread_t) * (size_t)threads);
        for (int32_t t = 0; t < threads; t++) pthread_create(&th[t], NULL, tails_worker, &J);
        for (int32_t t = 0; t < threads; t++) pthread_join(th[t], NULL);
        free(th);
    }
    pthread_mutex_destroy(&J.lock);
    free(bstart); free(bnodes);
    return J.status != ORC_OK ? J.status : status;
}

/* ------------------------------------------------------------------------ */
/* Exact S(v) = sum_u d(v,u) for every node: one search per node (Eq. (1)).
 * Round-trip when the transpose is given. */
typedef struct {
    int64_t n; const int64_t* rp; const int32_t* col; const int32_t* w;
    const int64_t* rrp; const int32_t* rcol; const int32_t* rw;
    int64_t* S; int64_t next; pthread_mutex_t lock; int status;
} exact_job;

static void* exact_worker(void* arg) {
    exact_job* J = (exact_job*)arg;
    int64_t* a = (int64_t*)malloc(sizeof(int64_t) * (size_t)J->n);
    int64_t* b = J->rrp ? (int64_t*)malloc(sizeof(int64_t) * (size_t)J->n) : NULL;
    for (;;) {
        pthread_mutex_lock(&J->lock);
        int64_t v = J->next++;
        pthread_mutex_unlock(&J->lock);
        if (v >= J->n) break;
        sssp(J->n, J->rp, J->col, J->w, (int32_t)v, a);
        if (b) sssp(J->n, J->rrp, J->rcol, J->rw, (int32_t)v, b);
        int64_t s = 0; int bad = 0;
        for (int64_t u = 0; u < J->n; u++) {
            if (a[u] < 0 || (b && b[u] < 0)) { bad = 1; continue; }
            s += a[u] + (b ? b[u] : 0);
        }
        J->S[v] = bad ? -1 : s;
        if (bad) { pthread_mutex_lock(&J->lock); J->status = ORC_EUNREACHED; pthread_mutex_unlock(&J->lock); }
    }
    free(a); free(b);
    return NULL;
}

int orc_exact_sums(int64_t n, const int64_t* rp, const int32_t* col, const int32_t* w, const int64_t* rrp,
                   const int32_t* rcol, const int32_t* rw, int32_t threads, int64_t* S) {
    exact_job J;
    J.n = n; J.rp = rp; J.col = col; J.w = w; J.rrp = rrp; J.rcol = rcol; J.rw = rw;
    J.S = S; J.next = 0; J.status = ORC_OK;
    pthread_mutex_init(&J.lock, NULL);
    if (threads <= 1) {
        exact_worker(&J);
    } else {
        pthread_t* th = (pthread_t*)malloc(sizeof(pthread_t) * (size_t)threads);
        for (int32_t t = 0; t < threads; t++) pthread_create(&th[t], NULL, exact_worker, &J);
        for (int32_t t = 0; t < threads; t++) pthread_join(th[t], NULL);
        free(th);
    }
    pthread_mutex_destroy(&J.lock);
    return J.status;
}

/* ------------------------------------------------------------------------ */
/* Sec. 6.2 / Algorithm 4, outbound (search on G) or inbound (search on the
 * transpose, passed as rp/col): the bottom-k sample of each node's
 * reachability set under the rank order rank[u] (0-based position of u in a
 * uniformly random order of V), taken from its definition.  For every node v:
 *   count   = min(k, |R(v)|), R(v) = the nodes u != v reached from v;
 *   distsum = the sum of d over the count members of R(v) first in rank order;
 *   T       = when count = k, the number of nodes other than v whose rank is
 *             at most that of the k-th member (its 1-based position among
 *             V \ {v}); 0 otherwise;
 *   B       = distsum / count (0 when count = 0), the average-distance
 *             estimate;
 *   R       = count when count < k, else 1 + (k-1)(n-2) / (T-1), the
 *             reachability estimate (1 when k = 1, whose numerator is 0). */
typedef struct {
    int64_t n; const int64_t* rp; const int32_t* col; const int32_t* w; const int32_t* rank; int32_t k;
    const int32_t* nodes; int64_t nnodes;  /* the nodes to compute (NULL: all, outputs indexed by node) */
    int32_t* count; int64_t* distsum; int64_t* T; double* B; double* R; int64_t next; pthread_mutex_t lock;
} reach_job;

static void* reach_worker(void* arg) {
    reach_job* J = (reach_job*)arg;
    const int64_t n = J->n;
    int64_t* d = (int64_t*)malloc(sizeof(int64_t) * (size_t)n);
    int32_t* by_rank = (int32_t*)malloc(sizeof(int32_t) * (size_t)n);  /* node at each rank */
    for (int64_t u = 0; u < n; u++) by_rank[J->rank[u]] = (int32_t)u;
    for (;;) {
        pthread_mutex_lock(&J->lock);
        int64_t slot = J->next++;
        pthread_mutex_unlock(&J->lock);
        if (slot >= (J->nodes ? J->nnodes : n)) break;
        int64_t v = J->nodes ? J->nodes[slot] : slot;
        sssp(n, J->rp, J->col, J->w, (int32_t)v, d);
        int32_t cnt = 0;
        int64_t sum = 0, T = 0, kth = -1;
        /* walk V in rank order, keep the first k reached nodes other than v */
        for (int64_t r = 0; r < n && cnt < J->k; r++) {
            int32_t u = by_rank[r];
            if (u == v || d[u] < 0) continue;
            cnt++;
            sum += d[u];
            if (cnt == J->k) kth = r;
        }
        if (kth >= 0) T = (kth + 1) - (J->rank[v] < kth ? 1 : 0);
        J->count[slot] = cnt;
        J->distsum[slot] = sum;
        J->T[slot] = T;
        J->B[slot] = cnt > 0 ? (double)sum / (double)cnt : 0.0;
        if (cnt < J->k) J->R[slot] = (double)cnt;
        else if (J->k == 1) J->R[slot] = 1.0;
        else J->R[slot] = 1.0 + (double)((int64_t)(J->k - 1) * (n - 2)) / (double)(T - 1);
    }
    free(d); free(by_rank);
    return NULL;
}

int orc_reach_all(int64_t n, const int64_t* rp, const int32_t* col, const int32_t* w, const int32_t* rank,
                  int32_t k, const int32_t* nodes, int64_t nnodes, int32_t threads, int32_t* count,
                  int64_t* distsum, int64_t* T, double* B, double* R) {
    if (k < 1) return ORC_EINVAL;
    reach_job J;
    J.n = n; J.rp = rp; J.col = col; J.w = w; J.rank = rank; J.k = k; J.nodes = nodes; J.nnodes = nnodes;
    J.count = count; J.distsum = distsum; J.T = T; J.B = B; J.R = R; J.next = 0;
    pthread_mutex_init(&J.lock, NULL);
    if (threads <= 1) {
        reach_worker(&J);
    } else {
        pthread_t* th = (pthread_t*)malloc(sizeof(pthread_t) * (size_t)threads);
        for (int32_t t = 0; t < threads; t++) pthread_create(&th[t], NULL, reach_worker, &J);
        for (int32_t t = 0; t < threads; t++) pthread_join(th[t], NULL);
        free(th);
    }
    pthread_mutex_destroy(&J.lock);
    return ORC_OK;
}

/* ------------------------------------------------------------------------ */
/* Sec. 5 / Algorithm 3: the node-weighted hybrid estimate.  The sample C has
 * adjusted weights beta^(c) = max(tau, beta(c)), tau = R/m: the light samples
 * (light[i] = 1) weigh tau, the heavy ones their own weight.  For v not in C,
 * with the pivot, Delta and the sets L, HC, H of Eq. (6) (u != v, L decided
 * by d(c(v),u) * num <= Delta * den):
 *   S_beta^(v) = sum_H beta(u) d(c(v),u) + sum_HC beta(u) d(v,u) + sum_{L cap C} beta^(u) d(v,u)
 * evaluated exactly as N / m, N = (sum_H + sum_HC + sum_{heavy L cap C}) * m
 * + R * sum_{light L cap C} d(v,u), one division; and the variance estimate
 * of the L term, sum over light L cap C of d^2 (tau - beta(u)) tau, as
 * t * (t * A - B) with t = R/m, A = sum d^2, B = sum beta(u) d^2 over the light
 * members of L cap C.  For v in C: the exact sum_u beta(u) d(v,u), variance 0.
 * D[u*k + i] = d(c_i, u) (symmetric distances). */
typedef struct {
    int64_t n; int32_t k; const int32_t* sidx; const uint8_t* light; const uint32_t* beta; int64_t R; int32_t m;
    const int64_t* D; int64_t num, den; const int32_t* nodes; int64_t nnodes;  /* NULL: all nodes */
    double* S; double* var; double* err; int64_t next; pthread_mutex_t lock; int status;
} beta_job;

static void* beta_worker(void* arg) {
    beta_job* J = (beta_job*)arg;
    const int64_t n = J->n, k = J->k;
    const __int128 LIM = (__int128)1 << 53;
    for (;;) {
        pthread_mutex_lock(&J->lock);
        int64_t slot = J->next++;
        pthread_mutex_unlock(&J->lock);
        if (slot >= (J->nodes ? J->nnodes : n)) break;
        int64_t v = J->nodes ? J->nodes[slot] : slot;
        const int64_t* row = J->D + v * k;
        int ovf = 0;
        if (J->sidx[v] >= 0) {
            int32_t i = J->sidx[v];
            __int128 s = 0;
            for (int64_t u = 0; u < n; u++) s += (__int128)J->beta[u] * J->D[u * k + i];
            ovf = s >= LIM;
            J->S[slot] = (double)(int64_t)s;
            J->var[slot] = 0.0;
            if (J->err) J->err[slot] = 0.0;
        } else {
            int32_t p = orc_pivot((int32_t)k, row);
            int64_t delta = row[p];
            __int128 H = 0, HC = 0, Lb = 0, Ls = 0, A = 0, B = 0, Hb = 0, HCb = 0, HCsq = 0;
            for (int64_t u = 0; u < n; u++) {
                if (u == v) continue;
                int64_t dpu = J->D[u * k + p];
                int32_t j = J->sidx[u];
                if ((__int128)dpu * J->num <= (__int128)delta * J->den) {  /* u in L */
                    if (j < 0) continue;  /* only the sampled members of L are counted */
                    int64_t d = row[j];
                    if (J->light[j]) { Ls += d; A += (__int128)d * d; B += (__int128)J->beta[u] * d * d; }
                    else Lb += (__int128)J->beta[u] * d;
                } else if (j >= 0) {
                    HC += (__int128)J->beta[u] * row[j];
                    HCb += J->beta[u];
                    HCsq += (__int128)J->beta[u] * (row[j] - dpu) * (row[j] - dpu);
                } else {
                    H += (__int128)J->beta[u] * dpu;
                    Hb += J->beta[u];
                }
            }
            __int128 N = (H + HC + Lb) * J->m + Ls * J->R;
            ovf = N >= LIM || A > (__int128)INT64_MAX || B > (__int128)INT64_MAX;
            J->S[slot] = (double)(int64_t)N / (double)J->m;
            double t = (double)J->R / (double)J->m;
            J->var[slot] = t * (t * (double)(int64_t)A - (double)(int64_t)B);
            /* Sec. 4.1 with beta masses (Sec. 5): the L term's variance plus beta(H) times the
             * beta-weighted mean over HC of (d(v,u) - d(c(v),u))^2; without HC weight the mean is
             * over the samples at the largest distance from the pivot (Sec. 4.1's suffix of the
             * farthest samples), 0 if they weigh nothing either */
            if (HCb == 0) {
                int64_t far = -1;
                for (int64_t u = 0; u < n; u++)
                    if (J->sidx[u] >= 0 && J->D[u * k + p] > far) far = J->D[u * k + p];
                for (int64_t u = 0; u < n; u++) {
                    int32_t j = J->sidx[u];
                    if (j < 0 || J->D[u * k + p] != far) continue;
                    HCb += J->beta[u];
                    HCsq += (__int128)J->beta[u] * (row[j] - far) * (row[j] - far);
                }
            }
            ovf = ovf || HCsq > (__int128)INT64_MAX;
            if (J->err)
                J->err[slot] = J->var[slot] +
                               (HCb > 0 ? ((double)(int64_t)HCsq / (double)(int64_t)HCb) * (double)(int64_t)Hb : 0.0);
        }
        if (ovf) { pthread_mutex_lock(&J->lock); J->status = ORC_EOVERFLOW; pthread_mutex_unlock(&J->lock); }
    }
    return NULL;
}

int orc_beta_all(int64_t n, int32_t k, const int32_t* sidx, const uint8_t* light, const uint32_t* beta, int64_t R,
                 int32_t m, const int64_t* D, int64_t num, int64_t den, const int32_t* nodes, int64_t nnodes,
                 int32_t threads, double* S, double* var, double* err) {
    if (k < 1 || m < 1 || num < 1 || den < 1) return ORC_EINVAL;
    beta_job J;
    J.n = n; J.k = k; J.sidx = sidx; J.light = light; J.beta = beta; J.R = R; J.m = m; J.D = D;
    J.nodes = nodes; J.nnodes = nnodes;
    J.num = num; J.den = den; J.S = S; J.var = var; J.err = err; J.next = 0; J.status = ORC_OK;
    pthread_mutex_init(&J.lock, NULL);
    if (threads <= 1) {
        beta_worker(&J);
    } else {
        pthread_t* th = (pthread_t*)malloc(sizeof(pthread_t) * (size_t)threads);
        for (int32_t t = 0; t < threads; t++) pthread_create(&th[t], NULL, beta_worker, &J);
        for (int32_t t = 0; t < threads; t++) pthread_join(th[t], NULL);
        free(th);
    }
    pthread_mutex_destroy(&J.lock);
    return J.status;
}

/* ------------------------------------------------------------------------ */
/* Sec. 6.2 / Algorithm 5, node-weighted reachability sampling.  Nodes with
 * beta > 0 have priority ranks r(u) = U(u) / (2^53 beta(u)), U(u) in
 * [1, 2^53] (compared exactly: r(a) < r(b) iff U(a) beta(b) < U(b) beta(a),
 * ties by id).  For every node v, the sample is the k members of R(v) (nodes
 * u != v with beta > 0 reached from v; the caller passes the transpose for
 * inbound) first in rank order.  With c = the sample size:
 *   c < k : S = sum beta(u) d, R = sum beta(u) over the sample (exact);
 *   c = k : T = r(k-th member), tau = 1/T = 2^53 beta_k / U_k; each of the
 *           first k-1 members weighs max(beta(u), tau) (priority sampling):
 *           heavy (beta(u) U_k >= 2^53 beta_k) its own weight, light tau;
 *           S = (double)sum_heavy beta d + tau * (double)sum_light d,
 *           R = (double)sum_heavy beta + tau * (double)(number light),
 *           tau computed as ldexp(beta_k, 53) / U_k.
 * Outputs count, the k-th member (-1 if none), S and R. */
typedef struct {
    int64_t n; const int64_t* rp; const int32_t* col; const int32_t* w; const uint32_t* beta; const uint64_t* U;
    const int32_t* by_rank; int64_t npos; const int32_t* pos_of; int32_t k; const int32_t* nodes; int64_t nnodes;
    int32_t* count; int32_t* kth; double* S; double* R; int64_t next; pthread_mutex_t lock;
} rbeta_job;

static void* rbeta_worker(void* arg) {
    rbeta_job* J = (rbeta_job*)arg;
    const int64_t n = J->n;
    int64_t* d = (int64_t*)malloc(sizeof(int64_t) * (size_t)n);
    int32_t* mem = (int32_t*)malloc(sizeof(int32_t) * (size_t)(J->k > 0 ? J->k : 1));
    for (;;) {
        pthread_mutex_lock(&J->lock);
        int64_t slot = J->next++;
        pthread_mutex_unlock(&J->lock);
        if (slot >= (J->nodes ? J->nnodes : n)) break;
        int64_t v = J->nodes ? J->nodes[slot] : slot;
        sssp(n, J->rp, J->col, J->w, (int32_t)v, d);
        int32_t c = 0;
        for (int64_t r = 0; r < J->npos && c < J->k; r++) {
            int32_t u = J->by_rank[r];
            if (u == v || d[u] < 0) continue;
            mem[c++] = u;
        }
        J->count[slot] = c;
        if (c < J->k) {
            int64_t s = 0, rr = 0;
            for (int32_t j = 0; j < c; j++) { s += (int64_t)J->beta[mem[j]] * d[mem[j]]; rr += J->beta[mem[j]]; }
            J->kth[slot] = -1;
            J->S[slot] = (double)s;
            J->R[slot] = (double)rr;
        } else {
            int32_t q = mem[J->k - 1];
            uint64_t Uk = J->U[q];
            uint64_t bk = J->beta[q];
            double tau = ldexp((double)bk, 53) / (double)Uk;
            int64_t hs = 0, hr = 0, ls = 0, lc = 0;
            for (int32_t j = 0; j < J->k - 1; j++) {
                int32_t u = mem[j];
                unsigned __int128 lhs = (unsigned __int128)J->beta[u] * Uk;
                unsigned __int128 rhs = (unsigned __int128)bk << 53;
                if (lhs >= rhs) { hs += (int64_t)J->beta[u] * d[u]; hr += J->beta[u]; }
                else { ls += d[u]; lc += 1; }
            }
            J->kth[slot] = q;
            J->S[slot] = (double)hs + tau * (double)ls;
            J->R[slot] = (double)hr + tau * (double)lc;
        }
    }
    free(d); free(mem);
    return NULL;
}

int orc_reach_beta(int64_t n, const int64_t* rp, const int32_t* col, const int32_t* w, const uint32_t* beta,
                   const uint64_t* U, const int32_t* by_rank, int64_t npos, int32_t k, const int32_t* nodes,
                   int64_t nnodes, int32_t threads, int32_t* count, int32_t* kth, double* S, double* R) {
    if (k < 1) return ORC_EINVAL;
    rbeta_job J;
    J.n = n; J.rp = rp; J.col = col; J.w = w; J.beta = beta; J.U = U; J.by_rank = by_rank; J.npos = npos;
    J.k = k; J.nodes = nodes; J.nnodes = nnodes; J.count = count; J.kth = kth; J.S = S; J.R = R; J.next = 0;
    pthread_mutex_init(&J.lock, NULL);
    if (threads <= 1) {
        rbeta_worker(&J);
    } else {
        pthread_t* th = (pthread_t*)malloc(sizeof(pthread_t) * (size_t)threads);
        for (int32_t t = 0; t < threads; t++) pthread_create(&th[t], NULL, rbeta_worker, &J);
        for (int32_t t = 0; t < threads; t++) pthread_join(th[t], NULL);
        free(th);
    }
    pthread_mutex_destroy(&J.lock);
    return ORC_OK;
}
