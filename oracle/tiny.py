"""Set-level brute force for tiny graphs (test infrastructure only).

Distances by Floyd-Warshall over an adjacency matrix (all pairs, no search
order at all), then every estimator of Sec. 2 evaluated with explicit Python
sets and exact rationals (fractions.Fraction): L(j), HC(j) and H(j) are built
as sets and Eq. (6) is evaluated as written.  Used to cross-check the C oracle
on many random tiny graphs; O(n^3) time.
"""
from __future__ import annotations

from fractions import Fraction

INF = float("inf")


def floyd_warshall(n, row_ptr, col_idx, w=None):
    d = [[INF] * n for _ in range(n)]
    for v in range(n):
        d[v][v] = 0
        for e in range(int(row_ptr[v]), int(row_ptr[v + 1])):
            u = int(col_idx[e])
            c = 1 if w is None else int(w[e])
            if u != v and c < d[v][u]:
                d[v][u] = c
    for m in range(n):
        dm = d[m]
        for a in range(n):
            dam = d[a][m]
            if dam == INF:
                continue
            da = d[a]
            for b in range(n):
                x = dam + dm[b]
                if x < da[b]:
                    da[b] = x
    return d


def round_trip(d):
    n = len(d)
    return [[d[a][b] + d[b][a] for b in range(n)] for a in range(n)]


def pivot_sq_err(dist, samples, j, cp, HC):
    """Sec. 4.1's estimate of the mean squared pivoting error of node j with
    pivot cp: the mean of (d(j,u) - d(cp,u))^2 over HC, and when HC is empty
    over the "suffix" of the farthest samples, read as the samples at the
    largest distance from the pivot (Fraction)."""
    if HC:
        return sum(Fraction(dist[j][i] - dist[cp][i]) ** 2 for i in HC) / len(HC)
    far = max(dist[cp][c] for c in samples)
    F = [c for c in samples if dist[cp][c] == far]
    return sum(Fraction(dist[j][i] - dist[cp][i]) ** 2 for i in F) / len(F)


def estimates(dist, samples, eps: Fraction):
    """dist: full n x n metric (list of lists); samples: ordered list C.
    Returns dict of per-node lists: pivot, delta, S_exact, S_samp, S_piv, S_pub, S_hyb
    (Fractions for the fractional ones)."""
    n = len(dist)
    k = len(samples)
    C = set(samples)
    S = [sum(dist[v]) for v in range(n)]
    out = {key: [] for key in ("pivot", "delta", "S_exact", "S_samp", "S_piv", "S_pub", "S_hyb", "S_err")}
    for j in range(n):
        out["S_exact"].append(S[j])
        dists = [dist[j][c] for c in samples]
        m = min(dists)
        p = dists.index(m)              # first (lowest) index among ties
        cp = samples[p]
        out["pivot"].append(p)
        out["delta"].append(m)
        if j in C:
            for key in ("S_samp", "S_piv", "S_pub", "S_hyb"):
                out[key].append(Fraction(S[j]))
            out["S_err"].append(Fraction(0))
            continue
        T = Fraction(m) / eps
        others = set(range(n)) - {j}
        L = {i for i in others if dist[cp][i] <= T}
        HC = {i for i in others if i in C and dist[cp][i] > T}
        H = {i for i in others if i not in C and dist[cp][i] > T}
        assert L | HC | H == others and not (L & HC) and not (L & H) and not (HC & H)
        LC = L & C
        s_hyb = (sum(Fraction(dist[cp][i]) for i in H) + sum(Fraction(dist[j][i]) for i in HC)
                 + Fraction(len(L), len(LC)) * sum(Fraction(dist[j][i]) for i in LC))
        out["S_hyb"].append(s_hyb)
        # Sec. 4.1: sample variance over L cap C (population form, mean of the
        # squared deviations from the sample mean), over |L cap C|, times |L|;
        # plus |H| times the mean squared pivot error over HC (no HC: over the
        # farthest samples)
        mean = sum(Fraction(dist[j][i]) for i in LC) / len(LC)
        var = sum((Fraction(dist[j][i]) - mean) ** 2 for i in LC) / len(LC)
        piv_err = pivot_sq_err(dist, samples, j, cp, HC)
        out["S_err"].append(var / len(LC) * len(L) + piv_err * len(H))
        out["S_samp"].append(Fraction(n - 1, k) * sum(dists))
        out["S_piv"].append(Fraction(S[cp]))
        out["S_pub"].append(Fraction(S[cp] + (n - 1) * m))
    return out


def adaptive(dist, samples, eps_list):
    """Per node, the hybrid estimate for the eps of eps_list (Fractions) with
    the smallest estimated squared error, the first on ties (exact
    rationals).  Returns (S_ad list, S_ad_err list, chosen index list)."""
    per = [estimates(dist, samples, e) for e in eps_list]
    n = len(dist)
    S_ad, S_err, which = [], [], []
    for j in range(n):
        best = 0
        for e in range(1, len(eps_list)):
            if per[e]["S_err"][j] < per[best]["S_err"][j]:
                best = e
        S_ad.append(per[best]["S_hyb"][j])
        S_err.append(per[best]["S_err"][j])
        which.append(best)
    return S_ad, S_err, which


def sweep_candidates(dist, samples, j):
    """The candidates of Algorithm 2 / Sec. 4.2 for an unsampled node j, in
    the order they are compared: pure pivoting (S(c(j)), mean squared pivot
    error over all samples times the other unsampled nodes), then, for each
    distinct distance T from the pivot to a sample in increasing order, the
    threshold estimate over the partition of V minus j into L, HC and H, with
    its estimated error as in Sec. 4.1.  Exact rationals, explicit sets."""
    n = len(dist)
    k = len(samples)
    C = set(samples)
    dists = [dist[j][c] for c in samples]
    cp = samples[dists.index(min(dists))]
    sq_all = sum(Fraction(dist[j][c] - dist[cp][c]) ** 2 for c in samples)
    out = [(Fraction(sum(dist[cp])), sq_all / k * (n - 1 - k))]
    others = set(range(n)) - {j}
    for T in sorted({dist[cp][c] for c in samples}):
        L = {i for i in others if dist[cp][i] <= T}
        HC = {i for i in others if i in C and dist[cp][i] > T}
        H = {i for i in others if i not in C and dist[cp][i] > T}
        LC = L & C
        s_T = (sum(Fraction(dist[cp][i]) for i in H) + sum(Fraction(dist[j][i]) for i in HC)
               + Fraction(len(L), len(LC)) * sum(Fraction(dist[j][i]) for i in LC))
        mean = sum(Fraction(dist[j][i]) for i in LC) / len(LC)
        var = sum((Fraction(dist[j][i]) - mean) ** 2 for i in LC) / len(LC)
        piv = pivot_sq_err(dist, samples, j, cp, HC)
        out.append((s_T, var / len(LC) * len(L) + piv * len(H)))
    return out


def sweep(dist, samples):
    """Algorithm 2 / Sec. 4.2 with exact rationals: per node the candidate of
    sweep_candidates with the smallest estimated error (the first on ties);
    sampled nodes get their exact sum and error 0.  Returns (estimates,
    errors)."""
    C = set(samples)
    est, errs = [], []
    for j in range(len(dist)):
        if j in C:
            est.append(Fraction(sum(dist[j])))
            errs.append(Fraction(0))
            continue
        cand = sweep_candidates(dist, samples, j)
        best = min(range(len(cand)), key=lambda t: (cand[t][1], t))
        est.append(cand[best][0])
        errs.append(cand[best][1])
    return est, errs


def reach_definition(dist, order, k):
    """Sec. 6.2 from the definitions, exact rationals: for each node v the
    first k nodes u != v in `order` with dist[v][u] finite (dist[v][u] is the
    distance the estimate averages: from v for outbound, to v for inbound --
    pass the transposed matrix), and
    (count, distsum, T, B, R) with T the 1-based position of the k-th among
    V minus v, B = distsum/count (0 if none), R = count if count < k else
    1 + (k-1)(n-2)/(T-1)."""
    n = len(dist)
    pos = {u: i for i, u in enumerate(order)}
    out = []
    for v in range(n):
        reach = sorted((u for u in range(n) if u != v and dist[v][u] != INF), key=lambda u: pos[u])
        chosen = reach[:k]
        cnt = len(chosen)
        ds = sum(dist[v][u] for u in chosen)
        T = 0
        if cnt == k:
            T = sum(1 for u in range(n) if u != v and pos[u] <= pos[chosen[-1]])
        B = Fraction(ds, cnt) if cnt else Fraction(0)
        R = Fraction(cnt) if cnt < k else (Fraction(1) if k == 1 else 1 + Fraction((k - 1) * (n - 2), T - 1))
        out.append((cnt, ds, T, B, R))
    return out


def reach_algorithm4(n, arcs, order, k, corrected=False):
    """Algorithm 4 on a tiny graph given as a list of (tail, head, length)
    arcs: sources u in `order`; from each, a Dijkstra on the transposed graph
    (outbound: it reaches the nodes v that reach u, at distance d(v,u)); every
    scanned v != u counts u, adds d(v,u) while its count is at most k, and
    records T when its count reaches k (the number of processed sources, less
    one if v itself was processed earlier).  Pass reversed arcs for inbound.
    The search stops expanding at a node x when
      * as printed (corrected=False): x's count is already k;
      * corrected: x's count plus one if x was processed before u is at least
        k + 1 -- then every node reaching x has k members ranked before u
        other than itself, so u is in none of their samples.  The printed
        rule also stops when x's k members include a node w that reaches x,
        and w, which cannot count itself, loses u.
    Returns the same tuples as reach_definition."""
    import heapq
    radj = [[] for _ in range(n)]
    for a, b, w in arcs:
        radj[b].append((a, w))
    mark = [False] * n
    count = [0] * n
    T = [0] * n
    distsum = [0] * n
    for t, u in enumerate(order, start=1):
        mark[u] = True
        best = {u: 0}
        heap = [(0, u)]
        done = set()
        while heap:
            d, v = heapq.heappop(heap)
            if v in done or d > best[v]:
                continue
            done.add(v)
            if corrected:
                if count[v] + (1 if (mark[v] and v != u) else 0) >= k + 1:
                    continue  # pruned: not expanded
            elif count[v] >= k:
                continue  # pruned: not expanded
            if v != u:
                count[v] += 1
                if count[v] <= k:
                    distsum[v] += d
                if count[v] == k:
                    T[v] = t - 1 if mark[v] else t
            for x, w in radj[v]:
                nd = d + w
                if x not in best or nd < best[x]:
                    best[x] = nd
                    heapq.heappush(heap, (nd, x))
    out = []
    for v in range(n):
        cnt = min(count[v], k)
        B = Fraction(distsum[v], cnt) if cnt else Fraction(0)
        R = Fraction(cnt) if cnt < k else (Fraction(1) if k == 1 else 1 + Fraction((k - 1) * (n - 2), T[v] - 1))
        out.append((cnt, distsum[v], T[v] if cnt == k else 0, B, R))
    return out


def weighted_estimates(dist, beta, samples, light, tau, eps):
    """Sec. 5 / Algorithm 3 with exact rationals and explicit sets: for v
    not in C, with the pivot, Delta and L, HC, H of Eq. (6) over V minus v,
    S^ = sum_H beta d(c,u) + sum_HC beta d(v,u) + sum_{L cap C} beta^ d(v,u)
    (beta^ = tau for light samples, beta for heavy ones) and the variance
    estimate sum over light L cap C of d^2 (tau - beta) tau; sampled nodes
    their exact weighted sum and 0.  tau and eps are Fractions."""
    n = len(dist)
    C = list(samples)
    Cset = set(C)
    adj = {c: (tau if lt else Fraction(beta[c])) for c, lt in zip(C, light)}
    lightset = {c for c, lt in zip(C, light) if lt}
    est, var = [], []
    for v in range(n):
        if v in Cset:
            est.append(Fraction(sum(beta[u] * dist[v][u] for u in range(n))))
            var.append(Fraction(0))
            continue
        dists = [dist[v][c] for c in C]
        cp = C[dists.index(min(dists))]
        delta = dist[v][cp]
        others = [u for u in range(n) if u != v]
        L = {u for u in others if dist[cp][u] <= Fraction(delta) / eps}
        HC = {u for u in others if u in Cset and u not in L}
        H = {u for u in others if u not in Cset and u not in L}
        s = (sum(Fraction(beta[u] * dist[cp][u]) for u in H) + sum(Fraction(beta[u] * dist[v][u]) for u in HC)
             + sum(adj[u] * dist[v][u] for u in L & Cset))
        w = sum(Fraction(dist[v][u]) ** 2 * (tau - beta[u]) * tau for u in L & lightset)
        est.append(s)
        var.append(w)
    return est, var


def weighted_errors(dist, beta, samples, light, tau, eps):
    """Sec. 5's error estimate: Sec. 4.1 with beta masses -- the variance
    estimate of the L term plus beta(H) times the beta-weighted mean over HC
    of (d(v,u) - d(c(v),u))^2; without HC weight the mean is taken over the
    samples at the largest distance from the pivot (Sec. 4.1's suffix of the
    farthest samples; 0 if they weigh nothing either); sampled nodes 0."""
    n = len(dist)
    C = list(samples)
    Cset = set(C)
    _, var = weighted_estimates(dist, beta, samples, light, tau, eps)
    out = []
    for v in range(n):
        if v in Cset:
            out.append(Fraction(0))
            continue
        dists = [dist[v][c] for c in C]
        cp = C[dists.index(min(dists))]
        delta = dist[v][cp]
        others = [u for u in range(n) if u != v]
        far = [u for u in others if dist[cp][u] > Fraction(delta) / eps]
        HC = [u for u in far if u in Cset]
        Hb = sum(beta[u] for u in far if u not in Cset)
        HCb = sum(beta[u] for u in HC)
        if not HCb:
            top = max(dist[cp][c] for c in C)
            HC = [c for c in C if dist[cp][c] == top]
            HCb = sum(beta[u] for u in HC)
        sq = (sum(beta[u] * Fraction(dist[v][u] - dist[cp][u]) ** 2 for u in HC) / HCb) if HCb else Fraction(0)
        out.append(var[v] + sq * Hb)
    return out


def reach_weighted_definition(dist, beta, U, k):
    """Sec. 6.2 / Algorithm 5 with exact rationals: ranks r(u) = U(u) /
    (2^53 beta(u)) for beta(u) > 0 (ties by id); per node v the k members of
    R(v) (u != v, beta(u) > 0, dist[v][u] finite) of lowest rank; fewer than
    k: exact S = sum beta d, R = sum beta; else with T the k-th member's rank,
    each of the first k-1 members weighs max(beta, 1/T) (priority sampling).
    Returns (count, kth member or -1, S, R) per node, S and R as Fractions."""
    n = len(dist)
    rank = {u: (Fraction(int(U[u]), (1 << 53) * int(beta[u])), u) for u in range(n) if beta[u] > 0}
    out = []
    for v in range(n):
        mem = sorted((u for u in rank if u != v and dist[v][u] != INF), key=lambda u: rank[u])[:k]
        if len(mem) < k:
            out.append((len(mem), -1, Fraction(sum(beta[u] * dist[v][u] for u in mem)),
                        Fraction(sum(beta[u] for u in mem))))
            continue
        tau = 1 / rank[mem[-1]][0]
        wts = [max(Fraction(int(beta[u])), tau) for u in mem[:-1]]
        out.append((k, mem[-1], sum(w * dist[v][u] for w, u in zip(wts, mem[:-1])), sum(wts)))
    return out


def reach_weighted_algorithm5(n, arcs, beta, U, k):
    """Algorithm 5's searches run literally on a tiny graph (arcs (tail, head,
    length); pass reversed arcs for inbound): sources with beta > 0 in rank
    order, a Dijkstra from each on the transpose counting the source at every
    scanned node v != u, stopping (as for Algorithm 4) at a node holding k + 1
    members ranked before the source, counting itself when it ranks before
    it.  Returns each node's members in order (the first k)."""
    import heapq
    radj = [[] for _ in range(n)]
    for a, b, w in arcs:
        radj[b].append((a, w))
    order = sorted((u for u in range(n) if beta[u] > 0),
                   key=lambda u: (Fraction(int(U[u]), (1 << 53) * int(beta[u])), u))
    processed = set()
    members = [[] for _ in range(n)]
    for u in order:
        best = {u: 0}
        heap = [(0, u)]
        done = set()
        while heap:
            d, v = heapq.heappop(heap)
            if v in done or d > best[v]:
                continue
            done.add(v)
            if len(members[v]) + (1 if (v in processed and v != u) else 0) >= k + 1:
                continue
            if v != u:
                members[v].append((u, d))
            for x, w in radj[v]:
                nd = d + w
                if x not in best or nd < best[x]:
                    best[x] = nd
                    heapq.heappush(heap, (nd, x))
        processed.add(u)
    return [m[:k] for m in members]
