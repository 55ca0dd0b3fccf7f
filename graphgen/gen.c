/*
 * Seeded synthetic graph generators and graph preparation (component
 * extraction, relabelling, CSR construction, transposition).
 *
 * This module produces the INPUTS shared by the CPU oracle and the GPU
 * library.  It contains none of the estimator's arithmetic: no shortest-path
 * distances, no sampling of centrality sources, no estimates.  Connected
 * components use plain label propagation over an explicit stack, which is
 * graph preparation, not a distance computation.
 *
 * Random numbers: SplitMix64 (Steele, Lea & Flood, OOPSLA 2014) seeded per
 * graph, bounded integers by Lemire's multiply-shift with rejection (ACM TOMACS
 * 2019).  This stream is private to the generators.
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

typedef struct { uint64_t s; } gg_rng;

static inline uint64_t gg_next(gg_rng* r) {
    uint64_t z = (r->s += 0x9E3779B97F4A7C15ULL);
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ULL;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBULL;
    return z ^ (z >> 31);
}

/* uniform integer in [0, s), s >= 1 */
static inline uint64_t gg_below(gg_rng* r, uint64_t s) {
    uint64_t x = gg_next(r);
    unsigned __int128 m = (unsigned __int128)x * s;
    uint64_t l = (uint64_t)m;
    if (l < s) {
        uint64_t t = (0 - s) % s;
        while (l < t) {
            x = gg_next(r);
            m = (unsigned __int128)x * s;
            l = (uint64_t)m;
        }
    }
    return (uint64_t)(m >> 64);
}

/* uniform double in [0, 1) with 53 random bits */
static inline double gg_unit(gg_rng* r) { return (double)(gg_next(r) >> 11) * (1.0 / 9007199254740992.0); }

/* ------------------------------------------------------------------------ */
/* Barabasi-Albert preferential attachment.  A seed clique on m+1 nodes, then
 * each new node t attaches to m DISTINCT existing nodes chosen with
 * probability proportional to degree (endpoint-list method: a uniform entry of
 * the list of all edge endpoints so far).  Edges are emitted once each.
 * Capacity needed: m(m+1)/2 + (n-m-1)m. Returns the edge count, or -1. */
int64_t gg_ba(int64_t n, int32_t m, uint64_t seed, int32_t* src, int32_t* dst) {
    if (m < 1 || n < m + 1) return -1;
    gg_rng r = {seed};
    int64_t cap_end = 2 * ((int64_t)m * (m + 1) / 2 + (n - m - 1) * (int64_t)m);
    int32_t* ends = (int32_t*)malloc(sizeof(int32_t) * (size_t)cap_end);
    int32_t* pick = (int32_t*)malloc(sizeof(int32_t) * (size_t)m);
    if (!ends || !pick) { free(ends); free(pick); return -1; }
    int64_t ne = 0, e = 0;
    for (int32_t i = 0; i <= m; i++)
        for (int32_t j = i + 1; j <= m; j++) {
            src[e] = i; dst[e] = j; e++;
            ends[ne++] = i; ends[ne++] = j;
        }
    for (int64_t t = m + 1; t < n; t++) {
        int32_t got = 0;
        while (got < m) {
            int32_t c = ends[gg_below(&r, (uint64_t)ne)];
            int dup = 0;
            for (int32_t q = 0; q < got; q++) if (pick[q] == c) { dup = 1; break; }
            if (!dup) pick[got++] = c;
        }
        for (int32_t q = 0; q < m; q++) {
            src[e] = (int32_t)t; dst[e] = pick[q]; e++;
            ends[ne++] = (int32_t)t; ends[ne++] = pick[q];
        }
    }
    free(ends); free(pick);
    return e;
}

/* ------------------------------------------------------------------------ */
/* R-MAT (Chakrabarti, Zhan & Faloutsos, SDM 2004): each of `nedges` arcs picks
 * one of four quadrants per bit of the node id with probabilities a, b, c,
 * d = 1-a-b-c.  Node ids are then relabelled by a uniform random permutation
 * (so that id order carries no degree information).  Arcs may contain
 * duplicates and self-loops; the CSR builder removes them. */
void gg_rmat(int32_t scale, int64_t nedges, double a, double b, double c, uint64_t seed,
             int32_t* src, int32_t* dst) {
    gg_rng r = {seed};
    int64_t n = (int64_t)1 << scale;
    /* 32-bit thresholds; each 64-bit draw serves two levels (high, low half) */
    const uint64_t A = (uint64_t)(a * 4294967296.0);
    const uint64_t AB = (uint64_t)((a + b) * 4294967296.0);
    const uint64_t ABC = (uint64_t)((a + b + c) * 4294967296.0);
    for (int64_t e = 0; e < nedges; e++) {
        uint64_t u = 0, v = 0, x = 0;
        for (int32_t lvl = 0; lvl < scale; lvl++) {
            uint64_t h;
            if ((lvl & 1) == 0) { x = gg_next(&r); h = x >> 32; } else { h = x & 0xffffffffULL; }
            /* quadrant a: (0,0)  b: (0,1)  c: (1,0)  d: (1,1) */
            uint64_t ub = (uint64_t)(h >= AB);
            uint64_t vb = (uint64_t)(h >= A) ^ (uint64_t)(h >= AB) ^ (uint64_t)(h >= ABC);
            u = (u << 1) | ub;
            v = (v << 1) | vb;
        }
        src[e] = (int32_t)u; dst[e] = (int32_t)v;
    }
    int32_t* perm = (int32_t*)malloc(sizeof(int32_t) * (size_t)n);
    if (!perm) return;
    for (int64_t i = 0; i < n; i++) perm[i] = (int32_t)i;
    for (int64_t i = n - 1; i > 0; i--) {
        int64_t j = (int64_t)gg_below(&r, (uint64_t)(i + 1));
        int32_t t = perm[i]; perm[i] = perm[j]; perm[j] = t;
    }
    for (int64_t e = 0; e < nedges; e++) { src[e] = perm[src[e]]; dst[e] = perm[dst[e]]; }
    free(perm);
}

/* ------------------------------------------------------------------------ */
/* rows x cols grid, node id = y*cols + x.  nbr = 4 (axis moves) or 8 (axis +
 * diagonal moves).  Each edge is kept with probability 1-pdel and gets an
 * integer weight uniform in [wlo, whi] (wlo == whi == 1: unit grid).
 * Capacity: 2*rows*cols*... use gg_grid_capacity.  Returns the edge count. */
int64_t gg_grid_capacity(int32_t rows, int32_t cols, int32_t nbr) {
    int64_t R = rows, C = cols;
    int64_t e = R * (C - 1) + (R - 1) * C;
    if (nbr == 8) e += 2 * (R - 1) * (C - 1);
    return e;
}

int64_t gg_grid(int32_t rows, int32_t cols, int32_t nbr, double pdel, int32_t wlo, int32_t whi,
                uint64_t seed, int32_t* src, int32_t* dst, int32_t* w) {
    gg_rng r = {seed};
    int64_t e = 0;
    uint64_t span = (uint64_t)(whi - wlo + 1);
    for (int32_t y = 0; y < rows; y++)
        for (int32_t x = 0; x < cols; x++) {
            int32_t u = y * cols + x;
            int32_t cand[4]; int nc = 0;
            if (x + 1 < cols) cand[nc++] = u + 1;
            if (y + 1 < rows) cand[nc++] = u + cols;
            if (nbr == 8 && y + 1 < rows) {
                if (x + 1 < cols) cand[nc++] = u + cols + 1;
                if (x > 0) cand[nc++] = u + cols - 1;
            }
            for (int q = 0; q < nc; q++) {
                /* draw both numbers for every candidate edge so the weight
                 * stream does not depend on deletions */
                double keep = gg_unit(&r);
                int32_t wt = wlo + (int32_t)gg_below(&r, span);
                if (pdel > 0.0 && keep < pdel) continue;
                src[e] = u; dst[e] = cand[q];
                if (w) w[e] = wt;
                e++;
            }
        }
    return e;
}

/* ------------------------------------------------------------------------ */
/* CSR from an arc list.  symmetrize != 0 adds the reverse of every arc.
 * Self-loops are dropped; parallel arcs are merged keeping the minimum weight.
 * Adjacency lists come out sorted by target id.  `w`/`wout` may be NULL.
 * Output capacity for col/wout: m (or 2m when symmetrizing).
 * Returns the arc count. */
int64_t gg_csr_build(int64_t n, int64_t m, const int32_t* src, const int32_t* dst, const int32_t* w,
                     int32_t symmetrize, int64_t* row_ptr, int32_t* col, int32_t* wout) {
    /* expand to the full arc list (self-loops dropped), then two stable
     * counting sorts: by target, then by source, which leaves every row
     * ordered by target; duplicates are then adjacent. */
    int64_t total = 0;
    for (int64_t e = 0; e < m; e++)
        if (src[e] != dst[e]) total += symmetrize ? 2 : 1;
    size_t T = (size_t)(total > 0 ? total : 1);
    int32_t* as = (int32_t*)malloc(sizeof(int32_t) * T);
    int32_t* ad = (int32_t*)malloc(sizeof(int32_t) * T);
    int32_t* aw = (int32_t*)malloc(sizeof(int32_t) * T);
    int32_t* bs = (int32_t*)malloc(sizeof(int32_t) * T);
    int32_t* bd = (int32_t*)malloc(sizeof(int32_t) * T);
    int32_t* bw = (int32_t*)malloc(sizeof(int32_t) * T);
    int64_t* cnt = (int64_t*)malloc(sizeof(int64_t) * (size_t)(n + 1));
    if (!as || !ad || !aw || !bs || !bd || !bw || !cnt) {
        free(as); free(ad); free(aw); free(bs); free(bd); free(bw); free(cnt);
        return -1;
    }
    int64_t q = 0;
    for (int64_t e = 0; e < m; e++) {
        int32_t s = src[e], d = dst[e];
        if (s == d) continue;
        int32_t wt = w ? w[e] : 1;
        as[q] = s; ad[q] = d; aw[q] = wt; q++;
        if (symmetrize) { as[q] = d; ad[q] = s; aw[q] = wt; q++; }
    }
    /* pass 1: stable by target */
    memset(cnt, 0, sizeof(int64_t) * (size_t)(n + 1));
    for (int64_t e = 0; e < total; e++) cnt[ad[e] + 1]++;
    for (int64_t i = 0; i < n; i++) cnt[i + 1] += cnt[i];
    for (int64_t e = 0; e < total; e++) {
        int64_t p = cnt[ad[e]]++;
        bs[p] = as[e]; bd[p] = ad[e]; bw[p] = aw[e];
    }
    /* pass 2: stable by source */
    memset(cnt, 0, sizeof(int64_t) * (size_t)(n + 1));
    for (int64_t e = 0; e < total; e++) cnt[bs[e] + 1]++;
    for (int64_t i = 0; i < n; i++) cnt[i + 1] += cnt[i];
    for (int64_t e = 0; e < total; e++) {
        int64_t p = cnt[bs[e]]++;
        as[p] = bs[e]; ad[p] = bd[e]; aw[p] = bw[e];
    }
    /* rows are contiguous and target-sorted; merge parallel arcs (min weight) */
    int64_t out = 0, e = 0;
    row_ptr[0] = 0;
    for (int64_t v = 0; v < n; v++) {
        while (e < total && as[e] == v) {
            int32_t t = ad[e], wt = aw[e];
            e++;
            while (e < total && as[e] == v && ad[e] == t) {
                if (aw[e] < wt) wt = aw[e];
                e++;
            }
            col[out] = t;
            if (wout) wout[out] = wt;
            out++;
        }
        row_ptr[v + 1] = out;
    }
    free(as); free(ad); free(aw); free(bs); free(bd); free(bw); free(cnt);
    return out;
}

/* ------------------------------------------------------------------------ */
/* Largest connected component of a symmetric CSR.  newid[v] = new id (order
 * preserving) for v in the component, -1 otherwise.  Ties between equally
 * large components go to the one containing the smallest node id.
 * Returns the component size. */
int64_t gg_lcc(int64_t n, const int64_t* rp, const int32_t* col, int32_t* newid) {
    int32_t* comp = (int32_t*)malloc(sizeof(int32_t) * (size_t)(n > 0 ? n : 1));
    int32_t* stack = (int32_t*)malloc(sizeof(int32_t) * (size_t)(n > 0 ? n : 1));
    if (!comp || !stack) { free(comp); free(stack); return -1; }
    for (int64_t v = 0; v < n; v++) comp[v] = -1;
    int32_t best = -1; int64_t best_size = 0; int32_t nc = 0;
    for (int64_t s = 0; s < n; s++) {
        if (comp[s] >= 0) continue;
        int64_t top = 0, size = 0;
        stack[top++] = (int32_t)s; comp[s] = nc;
        while (top > 0) {
            int32_t v = stack[--top]; size++;
            for (int64_t e = rp[v]; e < rp[v + 1]; e++) {
                int32_t u = col[e];
                if (comp[u] < 0) { comp[u] = nc; stack[top++] = u; }
            }
        }
        if (size > best_size) { best_size = size; best = nc; }
        nc++;
    }
    int32_t next = 0;
    for (int64_t v = 0; v < n; v++) newid[v] = (comp[v] == best) ? next++ : -1;
    free(comp); free(stack);
    return best_size;
}

/* Largest strongly connected component of a directed CSR (Tarjan's algorithm
 * with an explicit call stack).  Same output convention as gg_lcc. */
int64_t gg_lscc(int64_t n, const int64_t* rp, const int32_t* col, int32_t* newid) {
    size_t N = (size_t)(n > 0 ? n : 1);
    int64_t* index = (int64_t*)malloc(sizeof(int64_t) * N);
    int64_t* low = (int64_t*)malloc(sizeof(int64_t) * N);
    int32_t* comp = (int32_t*)malloc(sizeof(int32_t) * N);
    char* onstk = (char*)calloc(N, 1);
    int32_t* stk = (int32_t*)malloc(sizeof(int32_t) * N);
    int32_t* cs_v = (int32_t*)malloc(sizeof(int32_t) * N);
    int64_t* cs_e = (int64_t*)malloc(sizeof(int64_t) * N);
    if (!index || !low || !comp || !onstk || !stk || !cs_v || !cs_e) {
        free(index); free(low); free(comp); free(onstk); free(stk); free(cs_v); free(cs_e);
        return -1;
    }
    for (int64_t v = 0; v < n; v++) { index[v] = -1; comp[v] = -1; }
    int64_t idx = 0, sp = 0, csp = 0;
    int32_t nc = 0, best = -1; int64_t best_size = 0, best_min = INT64_MAX;
    for (int64_t s = 0; s < n; s++) {
        if (index[s] >= 0) continue;
        cs_v[csp] = (int32_t)s; cs_e[csp] = rp[s]; csp++;
        index[s] = low[s] = idx++; stk[sp++] = (int32_t)s; onstk[s] = 1;
        while (csp > 0) {
            int32_t v = cs_v[csp - 1];
            int64_t e = cs_e[csp - 1];
            if (e < rp[v + 1]) {
                cs_e[csp - 1] = e + 1;
                int32_t u = col[e];
                if (index[u] < 0) {
                    index[u] = low[u] = idx++; stk[sp++] = u; onstk[u] = 1;
                    cs_v[csp] = u; cs_e[csp] = rp[u]; csp++;
                } else if (onstk[u] && index[u] < low[v]) {
                    low[v] = index[u];
                }
            } else {
                csp--;
                if (csp > 0) {
                    int32_t p = cs_v[csp - 1];
                    if (low[v] < low[p]) low[p] = low[v];
                }
                if (low[v] == index[v]) {
                    int64_t size = 0, mn = INT64_MAX;
                    int32_t x;
                    do {
                        x = stk[--sp]; onstk[x] = 0; comp[x] = nc; size++;
                        if (x < mn) mn = x;
                    } while (x != v);
                    if (size > best_size || (size == best_size && mn < best_min)) {
                        best_size = size; best = nc; best_min = mn;
                    }
                    nc++;
                }
            }
        }
    }
    int32_t next = 0;
    for (int64_t v = 0; v < n; v++) newid[v] = (comp[v] == best) ? next++ : -1;
    free(index); free(low); free(comp); free(onstk); free(stk); free(cs_v); free(cs_e);
    return best_size;
}

/* Induced subgraph on the nodes with newid >= 0, relabelled.  Adjacency order
 * is preserved (sorted input stays sorted: relabelling is monotone).
 * Returns the arc count. */
int64_t gg_induce(int64_t n, const int64_t* rp, const int32_t* col, const int32_t* w,
                  const int32_t* newid, int64_t* rp2, int32_t* col2, int32_t* w2) {
    int64_t out = 0, nv = 0;
    rp2[0] = 0;
    for (int64_t v = 0; v < n; v++) {
        if (newid[v] < 0) continue;
        for (int64_t e = rp[v]; e < rp[v + 1]; e++) {
            int32_t u = newid[col[e]];
            if (u < 0) continue;
            col2[out] = u;
            if (w && w2) w2[out] = w[e];
            out++;
        }
        rp2[++nv] = out;
    }
    return out;
}

/* Transpose of a CSR (arc u->v becomes v->u); lists come out sorted. */
void gg_transpose(int64_t n, const int64_t* rp, const int32_t* col, const int32_t* w,
                  int64_t* rp2, int32_t* col2, int32_t* w2) {
    memset(rp2, 0, sizeof(int64_t) * (size_t)(n + 1));
    for (int64_t e = 0; e < rp[n]; e++) rp2[col[e] + 1]++;
    for (int64_t i = 0; i < n; i++) rp2[i + 1] += rp2[i];
    int64_t* pos = (int64_t*)malloc(sizeof(int64_t) * (size_t)(n + 1));
    if (!pos) return;
    memcpy(pos, rp2, sizeof(int64_t) * (size_t)(n + 1));
    for (int64_t u = 0; u < n; u++)
        for (int64_t e = rp[u]; e < rp[u + 1]; e++) {
            int64_t q = pos[col[e]]++;
            col2[q] = (int32_t)u;
            if (w && w2) w2[q] = w[e];
        }
    free(pos);
}
