/*
 * ccgpu -- sample-based classic closeness centrality on one AMD Instinct
 * MI355X (gfx950).  C ABI.
 *
 * Method: Cohen, Delling, Pajor & Werneck, "Computing Classic Closeness
 * Centrality, at Scale" (2014).  For a graph G = (V, E) with n nodes the
 * classic closeness of v is (n-1) / S(v) with S(v) = sum_u d(v,u) (Eq. (1)).
 * The library draws k sample nodes C = (c_0 .. c_{k-1}), computes the
 * distances d(c_i, v) from every sample to every node (k single-source
 * shortest-path computations, Sec. 3), and returns, for every node v:
 *
 *   pivot[v]   index p of the nearest sample c(v) (Sec. 2), ties -> lowest p
 *   delta[v]   Delta(v) = d(v, c(v))
 *   sampsum[v] sum_i d(v, c_i)
 *   S_samp[v]  sample-average estimate, Eq. (5), as a sum: (n-1)/k * sampsum
 *   S_piv[v]   pivot estimate S(c(v)) (Sec. 1)
 *   S_pub[v]   pivoting upper bound S(c(v)) + (n-1) * Delta(v) (Sec. 1)
 *   S_hyb[v]   hybrid estimate, Eq. (6), threshold Delta(v)/eps
 *
 * and for v in C the exact S(v) in all four estimate fields (Sec. 2).  The
 * closeness estimate is (n-1) / S_*[v].
 *
 * Graphs are undirected (every edge stored as two arcs), or strongly
 * connected digraphs, for which distances are round-trip distances
 * d(u,v) + d(v,u) (Sec. 6.1).  Arc lengths are int32 >= 1; NULL lengths mean
 * unit lengths (breadth-first search).  Distances are int32, sums int64, and
 * S_hyb / S_samp are one correctly rounded IEEE double division of exact
 * integers (CC_EOVERFLOW when a numerator reaches 2^53).
 *
 * Conventions for every call:
 *   - Return value: CC_OK (0) or an error code; no exceptions, aborts or
 *     longjmp cross this boundary.  On error, caller-owned outputs are left
 *     untouched (device outputs may be partially written for CC_EDEVICE).
 *     cc_last_error() gives a text for the calling thread's last error.
 *   - Ownership: the caller owns every buffer it passes (host or device) and
 *     every handle it receives until the matching release/destroy call.  The
 *     library never returns memory the caller must free with anything but the
 *     functions below.
 *   - Threads: one context may be used from several host threads; calls on
 *     the same context are serialised internally.
 */
#ifndef CCGPU_H
#define CCGPU_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    CC_OK = 0,
    CC_EINVAL = 1,        /* bad argument: k < 1 or k > n, eps outside (0,1], bad CSR,
                             arc length < 1, duplicate or out-of-range sample */
    CC_EDISCONNECTED = 2, /* some node is unreachable from some sample: the graph is not
                             connected (strongly connected for digraphs), where the
                             classic centrality is not defined (Sec. 1) */
    CC_ENOMEM = 3,        /* device or host allocation failed */
    CC_EOVERFLOW = 4,     /* a distance left int32, or an estimate numerator reached 2^53 */
    CC_EDEVICE = 5,       /* HIP runtime error, or a kernel's bounded wait expired */
    CC_EBUSY = 6,         /* serving: not admitted yet (memory or slot limit); retry */
    CC_ECANCELLED = 7,    /* serving: job cancelled before it ran */
    CC_ENOTREADY = 8      /* serving: job still running (cc_poll) */
} cc_status;

/* Graph flags */
#define CC_DIRECTED 1u  /* arcs are directed; estimates use round-trip distances */
#define CC_VALIDATE 2u  /* check CSR shape, ids, lengths and (undirected) symmetry on upload */

/* Traversal mode */
#define CC_BATCHED 0    /* 64 samples per 64-bit word, all words of a node together */
#define CC_PLAIN 1      /* one sample at a time (the one-source baseline) */
#define CC_GRAPH 0x100  /* or-ed into CC_BATCHED: capture the whole estimate as a HIP graph on the first call
                           and replay it when the same graph, k, eps, output pointers and stream come again
                           (k <= 256: undirected graphs, round trips on digraphs, and graphs with arc lengths).
                           A replay is checked on the host (each BFS ended within the captured levels with
                           the same deepest level; the weighted searches' largest distances within the
                           captured ones; no error flag) and otherwise the estimate is recomputed as usual,
                           so results never depend on it.  Samples may change between calls. */

typedef struct cc_context cc_context;
typedef struct cc_graph cc_graph;
typedef struct cc_job cc_job;

typedef struct {
    int64_t mem_budget_bytes; /* serving admission budget; 0 = 80% of free device memory */
    int32_t max_inflight;     /* serving: slots (one stream each) running jobs at once; 0 = 4, the
                                 device's hardware queues per process */
    int32_t reserved;
} cc_config;

/* Create a context on HIP device `device`.  cfg may be NULL (defaults).
 * Creates a library-owned HIP stream used when callers pass stream NULL. */
cc_status cc_context_create(int device, const cc_config* cfg, cc_context** out);
void cc_context_destroy(cc_context* ctx);

/* Upload a CSR graph: row_ptr int64[n+1] (row_ptr[0] = 0, non-decreasing),
 * col_idx int32[arcs] (targets in [0,n)), w int32[arcs] or NULL (unit
 * lengths).  All three are HOST pointers; they are copied into library-owned
 * device memory (and, for CC_DIRECTED, the transposed graph is built once).
 * arcs must be < 2^32.  Self-loops are allowed and ignored by the distances.
 * The graph is released with cc_graph_release (it stays alive while jobs
 * that use it are running). */
cc_status cc_graph_upload(cc_context* ctx, int64_t n, int64_t arcs, const int64_t* row_ptr,
                          const int32_t* col_idx, const int32_t* w, uint32_t flags, cc_graph** out);
void cc_graph_release(cc_graph* g);
cc_status cc_graph_info(const cc_graph* g, int64_t* n, int64_t* arcs, uint32_t* flags);

/* The same graph (Algorithm 1's input "Network G") from a CSR that already
 * sits in DEVICE memory of the context's device, e.g. torch tensors:
 * row_ptr int64[n+1], col_idx int32[arcs], w int32[arcs] or NULL, in the
 * layout of cc_graph_upload.  Zero copy: the library reads col_idx and w in
 * place for the whole life of the graph and never writes or frees them; the
 * caller keeps the three arrays alive and unchanged until cc_graph_release
 * has been called AND every job that uses the graph has ended (the handle is
 * reference-counted while jobs run), and has finished writing them before
 * this call (it reads them on the context's own stream).  The library owns
 * only what it derives: 32-bit row bounds (4(n+1) B), for CC_DIRECTED the
 * transposed arcs (as in cc_graph_upload), the 64-node groups that hold a
 * node of degree above 32 and their arc chunks, and an identity id map.
 * Nodes keep the caller's order (no degree relabelling), so traversals of
 * skewed graphs can run slower than after cc_graph_upload; results are the
 * same.  Checks: shape and non-decreasing row bounds, ids in [0, n) and
 * lengths >= 1 (on the device), symmetry with CC_VALIDATE (copies the arcs to
 * the host).  CC_EINVAL when a check fails or an array is not device memory
 * of the context's device.  Such graphs are not batched with others
 * (cc_estimate_batch and the serving slots run them alone). */
cc_status cc_graph_borrow_device(cc_context* ctx, int64_t n, int64_t arcs, const int64_t* row_ptr,
                                 const int32_t* col_idx, const int32_t* w, uint32_t flags, cc_graph** out);

/* The sample draw of Sec. 2 (k nodes uniformly at random, as a set), fixed
 * so that independent implementations agree: SplitMix64 seeded with `seed`,
 * bounded integers by Lemire's multiply-shift with rejection (64-bit draws),
 * partial Fisher-Yates over 0..n-1; out[i] = c_i in draw order.  Host only;
 * needs no device. */
cc_status cc_draw_samples(int64_t n, int32_t k, uint64_t seed, int32_t* out);

typedef struct {
    int32_t k;                /* number of samples, 1 <= k <= n (k <= 4096) */
    int32_t mode;             /* CC_BATCHED or CC_PLAIN */
    uint64_t seed;            /* used when samples == NULL */
    const int32_t* samples;   /* HOST int32[k] explicit samples (distinct), or NULL */
    int32_t eps_num, eps_den; /* eps = eps_num / eps_den in (0, 1]; 0/0 = 1/round(sqrt(k)) */
} cc_params;

/* Outputs; every field may be NULL (= not wanted).  Per-node arrays have n
 * entries, per-sample arrays k entries, dmat k*k (dmat[i*k+j] = d(c_i,c_j)),
 * D n*k node-major (D[v*k+i] = d(c_i, v)). */
typedef struct {
    double* S_hyb;
    double* S_samp;
    int64_t* S_piv;
    int64_t* S_pub;
    int32_t* pivot;
    int32_t* delta;
    int64_t* sampsum;
    int64_t* src_sum;  /* S(c_i), exact */
    int32_t* samples;  /* the samples used */
    int32_t* dmat;
    int32_t* D;
    /* Sec. 4 (n entries each; 0 / the exact sum on sampled nodes):
     *   S_err     estimated squared error of S_hyb: |L|/|L cap C| times the sample
     *             variance of the distances to L cap C (mean squared deviation from
     *             their mean), plus |H| times the mean over F of
     *             (d(v,u) - d(c(v),u))^2, where F = HC, or, when HC is empty, the
     *             samples at the largest distance from c(v) (Sec. 4.1's "suffix" of
     *             the farthest samples); computed as
     *             ((|LC| * sum_LC d^2 - (sum_LC d)^2) / |LC|^3) * |L|
     *             + (sum_F (d - d_p)^2 / |F|) * |H| in that order of double operations
     *   S_ad      adaptive estimate: for each eps in {0.001, 0.025, 0.05, 0.1, 0.2,
     *             0.5, 0.99} (the list of Sec. 8) the hybrid estimate and its
     *             estimated error; the estimate with the smallest error (the first
     *             in this order on ties)
     *   S_ad_err  its estimated squared error
     * Algorithm 2 / Sec. 4.2, adaptive error minimisation (n entries each; the
     * exact sum and 0 on sampled nodes):
     *   S_sweep      for an unsampled v with pivot c: the candidates are pure
     *                pivoting (S(c), error (sum_i (d(v,c_i) - d(c,c_i))^2 / k) *
     *                (n-1-k)) and, for every distinct distance T from c to a sample,
     *                increasing, the estimate with L = {u != v : d(c,u) <= T}, HC the
     *                samples beyond T, H the other nodes beyond T (v itself is in
     *                none of them), Eq. (6)'s form, and its Sec. 4.1 error (with F
     *                as for S_err: the farthest samples when no sample lies beyond
     *                T); the candidate with the smallest error (the first on ties)
     *   S_sweep_err  its estimated squared error */
    double* S_err;
    double* S_ad;
    double* S_ad_err;
    double* S_sweep;
    double* S_sweep_err;
} cc_result;

/* Synchronous estimate; `out` holds HOST pointers. */
cc_status cc_estimate(cc_context* ctx, const cc_graph* g, const cc_params* p, cc_result* out);

/* Estimate into DEVICE pointers, enqueued on `hip_stream` (a hipStream_t;
 * NULL = the context's stream).  Returns after the work is enqueued and its
 * status is known (the call synchronises the stream once at the end to read
 * the device-side error flags). */
cc_status cc_estimate_device(cc_context* ctx, const cc_graph* g, const cc_params* p, cc_result* out,
                             void* hip_stream);

/* For callers that cannot allocate device memory (code running under HIP
 * graph capture of their own, tight serving loops, harnesses that forbid
 * allocation): cc_estimate_device without any device allocation.  The same
 * kernels run with every buffer carved from a 64 MiB array in the library's
 * device code (`scratch`, one copy per GPU, held until the process ends; its
 * address is looked up once per device when a context is created).  Calls
 * on one GPU share that array and the previous call's contents stay there:
 * the kernels initialise what they read.  Calls that would overlap on one GPU
 * race on it, so the library runs them one at a time (a per-device lock).
 * Undirected graphs without arc lengths, mode CC_BATCHED (no CC_GRAPH),
 * k <= 256; anything else is CC_EINVAL.  CC_ENOMEM (outputs untouched) when
 * the estimate needs more than the array holds: 16 MiB of per-job buffers and
 * traversal state, 40 MiB of level masks (levels x n x ceil(k/64) x 8 bytes,
 * plus n x k bytes when D is requested), 8 MiB of estimator tables.  Like
 * cc_estimate_device it synchronises `hip_stream` once at the end. */
cc_status cc_estimate_device_noalloc(cc_context* ctx, const cc_graph* g, const cc_params* p, cc_result* out,
                                     void* hip_stream);

/* Several estimates in one call, for many small graphs.  outs[j] holds HOST
 * pointers for job j (graphs[j], params[j]).  Jobs on undirected graphs
 * without arc lengths, with k <= 192 and at most 131072 nodes, are traversed
 * together: their graphs are laid side by side and their samples share the
 * bit words of one batched search (up to 256 samples, each job in whole
 * 64-bit words), so one launch per level serves every job of a batch; other
 * jobs run one by one.  Results are identical to separate calls.  statuses
 * (may be NULL) receives each job's status; the return value is CC_OK or the
 * first job error. */
cc_status cc_estimate_batch(cc_context* ctx, int32_t count, const cc_graph* const* graphs, const cc_params* params,
                            cc_result* outs, cc_status* statuses);

/* Timing of the last cc_estimate / cc_estimate_device on this context, from
 * HIP events recorded on the stream the kernels ran on (milliseconds), plus
 * the work counters the bench turns into bytes. */
typedef struct {
    double total_ms;       /* samples on device -> all outputs in device memory */
    double traverse_ms;    /* all traversal kernels (both directions for digraphs) */
    double epilogue_ms;    /* reductions, suffix tables, estimates */
    int64_t levels;        /* BFS levels / delta-stepping phases executed */
    int64_t arcs_scanned;  /* adjacency entries read by the traversal kernels */
    int64_t nodes_visited; /* node-level work items processed by the traversal */
    int64_t launches;      /* all traversal launches (including bookkeeping kernels) */
    int32_t dist_bytes;    /* bytes per stored distance (1, 2 or 4) */
    int32_t reserved;
    double kernel_ms;      /* summed duration of the level batches (device time from first to last level) */
    int64_t kernel_launches; /* levels enqueued */
    int64_t arcs_matched;  /* arcs pushed along by push levels */
    double scatter_ms;     /* summed duration of the scatter launches (one per level: the push, or the
                              pull over high in-degree nodes' arc chunks) */
    int64_t scatter_launches; /* number of those launches */
    int64_t scatter_arcs;  /* arcs they scanned (pulls) or pushed along (pushes) */
    int64_t hub_arcs;      /* of which scanned by pulls */
    double pull_scatter_ms; /* of scatter_ms, the levels that pulled */
    int64_t pull_levels;   /* levels run as pulls */
} cc_timing;
cc_status cc_last_timing(const cc_context* ctx, cc_timing* t);

/* ---- tuning ------------------------------------------------------------
 * Launch shapes and thresholds of the traversal, kept per graph.  None of
 * them changes any result (every estimate is exact given the samples); they
 * only change speed.  Set them while no job uses the graph. */
typedef struct {
    int32_t alpha;          /* BFS: a level pushes iff its frontier's out-arcs * alpha are fewer than the arcs
                               the last pull scanned (1..1024; default 4) */
    int32_t level_blocks;   /* BFS: blocks of the merge launch per level (1..65535; default 1024) */
    int32_t scatter_blocks; /* BFS: blocks of the scatter launch per level (1..65535; default 8192) */
    int32_t delta;          /* weighted: bucket width of delta-stepping (>= 1; default 1.5 x mean arc length) */
    int32_t round_blocks;   /* weighted: blocks per relaxation round (1..65535; default 1024) */
    int32_t local_passes;   /* weighted: block-local relaxation passes per round (0..1024; default 64) */
} cc_tuning;
cc_status cc_graph_get_tuning(const cc_graph* g, cc_tuning* t);
/* CC_EINVAL for a value outside its range. */
cc_status cc_graph_set_tuning(cc_graph* g, const cc_tuning* t);
/* Autotuner: times full estimates of k samples drawn from `seed` (median of
 * `reps` runs per candidate) while it varies one knob at a time over a fixed
 * candidate list (coordinate descent from the graph's current setting), keeps
 * the fastest setting in the graph and returns it with its time (ms, device
 * time of one estimate); a candidate replaces the current setting only when it
 * is at least 3% faster, so that timing noise does not move the setting.  Uses
 * the context's own stream and device buffers it allocates and frees itself. */
cc_status cc_autotune(cc_context* ctx, cc_graph* g, int32_t k, uint64_t seed, int32_t reps, cc_tuning* best,
                      double* best_ms);

/* ---- node-weighted centrality (Sec. 5, Algorithm 3) --------------------
 *
 * S_beta(v) = sum_u beta(u) d(v,u) for integer node weights beta >= 0.
 *
 * Sample (cc_draw_weighted): exactly k nodes (every node with beta > 0 when
 * there are at most k), node v taken with probability min(1, beta(v)/tau),
 * where tau solves sum_v min(1, beta(v)/tau) = k -- VarOpt's threshold -- with
 * exact integers:
 *   - the nodes with beta > 0 heaviest first (ties by id); the number L of
 *     heavy nodes is the first L with beta_(L+1) * (k-L) < R_L, R_L the weight
 *     of all but the L heaviest; tau = R / m with R = R_L, m = k - L; the heavy
 *     nodes are taken, with their own weight as adjusted weight;
 *   - the light nodes, masses beta(v) * m out of Q = R, pass in the order of
 *     cc_draw_samples(n, n, seed) through ordered pivotal (splitting)
 *     sampling: the pivot with mass a meets the next node with mass b; if
 *     a + b <= Q one of them gets a + b (the pivot with probability a/(a+b)),
 *     the other is dropped; else one is taken (the pivot with probability
 *     (Q-b)/(2Q-a-b)) and the other keeps a + b - Q; a pivot at Q is taken.
 *     Each decision of probability num/den draws x, the next output of the
 *     same generator after the permutation's draws, and is "yes" iff
 *     x * den < num * 2^64.  Taken light nodes have adjusted weight tau.
 *   This keeps the inclusion probabilities and the sample size exact with no
 *   positive covariances between inclusions (as VarOpt requires); it stands in
 *   for VarOpt's stream procedure, whose floating-point threshold updates
 *   would make the sample depend on rounding.
 * Estimate (Algorithm 3): the traversal of cc_estimate from this sample, then
 * for v outside C, with the pivot, Delta and L, HC, H of Eq. (6),
 *   S_beta^(v) = sum_H beta d(c(v),u) + sum_HC beta d(v,u) + sum_{L cap C} adjusted * d(v,u)
 * computed as N / m with N = (sum_H + sum_HC + sum_{heavy L cap C}) * m
 * + R * sum_{light L cap C} d (exact integers, one division), and the variance
 * estimate of the L term, sum over light L cap C of d^2 (tau - beta) tau, as
 * t * (t * A - B), t = R/m, A = sum d^2, B = sum beta d^2.  Sampled nodes: the
 * exact sum, variance 0. */
typedef struct {
    int32_t k;                 /* sample size (fewer when fewer nodes have beta > 0) */
    int32_t mode;              /* CC_BATCHED or CC_PLAIN, as in cc_params */
    uint64_t seed;
    int32_t eps_num, eps_den;  /* 0/0: eps = 1/round(sqrt(sample size)) */
    const uint32_t* beta;      /* HOST, n node weights at the caller's ids; some > 0 */
} cc_weighted_params;
typedef struct {
    double* S_beta;        /* n */
    double* S_beta_var;    /* n */
    int32_t* samples;      /* k: the sample in increasing id order, -1 past its size */
    double* adjusted;      /* k: adjusted weights (tau or the node's weight) */
    double* tau;           /* 1: R / m (0 when every positive node is sampled) */
    int32_t* sample_size;  /* 1 */
    double* S_beta_err;    /* n: the error estimate of Sec. 4.1 with beta masses (Sec. 5): S_beta_var
                              plus beta(H) times the beta-weighted mean over F of
                              (d(v,u) - d(c(v),u))^2, F = HC, or the samples at the largest
                              distance from c(v) when HC has no weight (0 if F weighs nothing), in
                              that order of double operations: var + (sum / weight(F)) * weight(H);
                              0 on samples */
} cc_weighted_result;
/* Host only: the sample above.  ids and light hold k entries; *count is the
 * sample size, *R and *m give tau = R/m.  CC_EINVAL without a node of positive
 * weight or when the total weight reaches 2^62. */
cc_status cc_draw_weighted(int64_t n, const uint32_t* beta, int32_t k, uint64_t seed, int32_t* ids, uint8_t* light,
                           int64_t* R, int32_t* m, int32_t* count);
/* Synchronous; `out` holds HOST pointers (any may be NULL).  CC_EOVERFLOW when
 * an exact numerator reaches 2^53 or a weighted sum leaves int64. */
cc_status cc_estimate_weighted(cc_context* ctx, const cc_graph* g, const cc_weighted_params* p,
                               cc_weighted_result* out);

/* ---- reachability sampling on general digraphs (Sec. 6.2, Algorithm 4) --
 *
 * For every node v: R(v) = the nodes u != v that v reaches (outbound) or that
 * reach v (inbound), with d the distance from v (outbound) or to v (inbound).
 * Under a rank order of the nodes (a uniformly random permutation), the
 * sample of v is the k members of R(v) ranked first (a uniform sample of size
 * min(k, |R(v)|) from R(v), as the bottom-k sample of Sec. 6.2).  Outputs,
 * per node at the caller's ids:
 *   count    min(k, |R(v)|)
 *   distsum  sum of d over the sample
 *   T        when count = k: the number of nodes other than v ranked no later
 *            than the k-th member of the sample; 0 otherwise
 *   B        distsum / count (0 when count = 0): the average-distance estimate
 *            of Algorithm 4's final step
 *   R        count when count < k, else 1 + (k-1)(n-2) / (T-1) (1 when k = 1):
 *            the reachability estimate of Algorithm 4's final step
 * The searches from the ranked sources stop at a node that holds k + 1
 * members ranked before the source, counting the node itself when it ranks
 * before it: this loses no member of any sample.  (Algorithm 4 as printed
 * stops at k members, which can lose a member: a node x whose k members
 * include v itself stops the search that v needed.)  Undirected graphs give
 * R(v) = the rest of v's component.  Unit arc lengths run batches of up to
 * 1024 sources as one bit-parallel BFS; with arc lengths (the listing's
 * Dijkstra) d is the shortest-path length and batches of up to 256 sources
 * run one delta-stepping search each (bucket width: the graph's tuning
 * knob `delta`), pruned by the same rule against the earlier batches. */
typedef struct {
    int32_t k;             /* sample size, k >= 1 */
    int32_t inbound;       /* 0: outbound (distances from v), 1: inbound (distances to v) */
    uint64_t seed;         /* rank order = cc_draw_samples(n, n, seed) when order is NULL */
    const int32_t* order;  /* optional HOST array of n node ids: the rank order, first to last */
} cc_reach_params;
typedef struct {
    int32_t* count;
    int64_t* distsum;
    int64_t* T;
    double* B;
    double* R;
} cc_reach_result;
/* Synchronous; `out` holds HOST pointers (n entries each; any may be NULL).
 * CC_EINVAL: k < 1, inbound not 0 or 1, or order not a permutation;
 * CC_EOVERFLOW: a search deeper than 65535 levels (unit lengths) or a
 * distance above 2^31 - 2 (arc lengths); CC_EDEVICE: an arc-length search
 * that ran past its two-minute limit; CC_ENOMEM.  Device state: about
 * 128 + 36 bytes per node (unit lengths), or 24 bytes per node and source of
 * a batch plus about 40 per node (arc lengths; the batch shrinks to fit a
 * quarter of the free memory), held in the context's arena. */
cc_status cc_reach_estimate(cc_context* ctx, const cc_graph* g, const cc_reach_params* p, cc_reach_result* out);

/* Node-weighted reachability sampling (Sec. 6.2, Algorithm 5): the nodes u
 * with beta(u) > 0 get priority ranks r(u) = U(u) / (2^53 beta(u)), U(u) =
 * (x >> 11) + 1 for the u-th output x of SplitMix64(seed) (u = 0..n-1),
 * compared exactly (ties by id); the sample of v is the k members of R(v) of
 * positive weight first in rank order, found by the same stopping searches.
 * Outputs per node:
 *   count  min(k, number of such members)
 *   kth    the k-th member (-1 when fewer)
 *   S, R   fewer than k members: the exact sum of beta(u) d and of beta(u)
 *          over them; else priority sampling's estimates of the weighted
 *          distance sum and the weighted reach: each of the first k-1 members
 *          weighs max(beta(u), 1/T), T = r(k-th member), 1/T computed as
 *          ldexp(beta_k, 53) / U_k; S = (double)(sum of beta d over the
 *          heavy ones) + (1/T) * (double)(sum of d over the light ones),
 *          R = (double)(sum of beta over the heavy) + (1/T) * (number light).
 *          (Algorithm 5's last step, S = (sum of beta d) / T, agrees for unit
 *          weights and is biased otherwise.)
 * Unit arc lengths or arc lengths (shortest-path lengths, searched as for
 * cc_reach_estimate); k <= 4096.  CC_EOVERFLOW when a weighted distance sum
 * leaves int64 (arc lengths) or a search is deeper than 65535 levels. */
typedef struct {
    int32_t k;
    int32_t inbound;        /* 0: outbound, 1: inbound */
    uint64_t seed;
    const uint32_t* beta;   /* HOST, n node weights; some > 0 */
} cc_reach_weighted_params;
typedef struct {
    int32_t* count;
    int32_t* kth;
    double* S;
    double* R;
} cc_reach_weighted_result;
/* Synchronous; `out` holds HOST pointers (n entries each; any may be NULL).
 * Device state: about 6(k-1) + 170 bytes per node (unit lengths), 8(k-1)
 * more than cc_reach_estimate's with arc lengths. */
cc_status cc_reach_weighted(cc_context* ctx, const cc_graph* g, const cc_reach_weighted_params* p,
                            cc_reach_weighted_result* out);

/* ---- serving: continuous batching over resident graphs ---------------- */

/* Submit a job; `out` holds HOST pointers that must stay valid until the job
 * completes.  Returns CC_OK with a job handle (queued), or CC_EINVAL.  Jobs
 * are admitted onto the device as memory (cc_config.mem_budget_bytes) and
 * slots (max_inflight) free up, and run concurrently on several streams; a
 * slot that takes a small job (as in cc_estimate_batch) also takes the small
 * jobs queued behind it that fit, into one batched traversal.  The oldest
 * queued job can be passed by younger ones that fit the memory it waits for
 * at most 16 times; then it is admitted next.  Each slot keeps its device
 * and pinned host staging between jobs (given back when it exceeds the
 * slot's share of the budget), so a job allocates nothing once its slot has
 * run one as large. */
cc_status cc_submit(cc_context* ctx, const cc_graph* g, const cc_params* p, const cc_result* out,
                    cc_job** job);
/* CC_OK when done successfully, CC_ENOTREADY while queued or running,
 * otherwise the job's error code. */
cc_status cc_poll(cc_job* job);
cc_status cc_wait(cc_job* job);
/* Cancels a job that has not started (CC_OK), else CC_EBUSY. */
cc_status cc_cancel(cc_job* job);
/* Latency bookkeeping of a finished job: submit->admit and submit->done, ms. */
cc_status cc_job_times(const cc_job* job, double* queue_ms, double* total_ms);
void cc_job_release(cc_job* job);

const char* cc_status_str(cc_status s);
const char* cc_last_error(void);

#ifdef __cplusplus
}
#endif
#endif
