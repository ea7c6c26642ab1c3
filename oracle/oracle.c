/*
 * CPU oracle for group-closeness maximisation (Bergamini, Gonser, Meyerhenke,
 * "Scaling up Group Closeness Maximization").
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product library calls, links or
 * loads this file; it shares no code, header or table with the GPU path.
 * Only the tests, the smoke check and the benchmark's CPU baseline use it.
 *
 * Everything is integer.  F(S) denotes the integer group farness
 * sum_{w in V} d(S,w); it is n times the paper's f(S) = 1/c(S) with
 * c(S) = n / sum_{v notin S} d(S,v) (Section 2), and it is the objective of
 * the ILP form in Section 5.  The marginal gain of v is
 * g(v,S) = F(S) - F(S u {v}) >= 0, i.e. minus n times the paper's
 * Delta(v,S) of Section 4.2.
 *
 * Tier A  (or_greedy): the plain greedy of Section 3.2, computed from the
 *   definition (after checking the input contract, or_validate): every round recomputes F(S u {v}) for every v not in S with a
 *   full BFS from v (Section 2: SSSP is BFS on unweighted graphs), then picks
 *   the minimum.  Ties go to the smallest node id.
 * Tier B  (or_greedypp): Greedy++ of Section 4, i.e. the memory-efficient
 *   greedy (Algorithm "mem-greedy") with the pruned SSSP of Section 4.1 and
 *   the supermodularity skip of Section 4.2; the first node comes from
 *   top-k closeness with BFScut (Section 3.1, Algorithm "topk"), k = 1.
 *   It is a second, independent route used where tier A is too slow, and the
 *   tests show it equal to tier A.
 *
 * Readings of the paper taken here (all also listed in the design notes):
 *   - ties between equal gains go to the smallest node id;
 *   - the skip test of Section 4.2 compares (stale gain, -id) lexicographically
 *     with the best (gain, -id) found so far in the round, so the result equals
 *     tier A for any candidate order;
 *   - the candidate scan order of the while-loop is ascending node id;
 *   - candidates are skip-tested a batch at a time against the best of the
 *     batches already evaluated in the round (a batch of one is the paper's
 *     sequential loop); batch sizes change the evaluation counts, never the
 *     picks.
 *
 * Build: gcc -O2 -fopenmp -shared -fPIC oracle.c -o liboracle.so
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define OR_OK 0
#define OR_EDISCONNECTED -3
#define OR_EINVAL -1
#define OR_ENOTSYM -2
#define OR_EINVARIANT -100

/* ------------------------------------------------------------------ BFS --- */

/*
 * Plain FIFO breadth-first search from `src` (Section 2: on unweighted graphs
 * the shortest-path distance d(src, w) is the BFS level of w).
 * dist[w] = d(src,w), or -1 when w is unreachable.  Returns #reached.
 */
int64_t or_bfs(int64_t n, const int32_t *rp, const int32_t *ci, int32_t src, int32_t *dist,
               int32_t *queue) {
    for (int64_t w = 0; w < n; ++w) dist[w] = -1;
    int64_t head = 0, tail = 0;
    dist[src] = 0;
    queue[tail++] = src;
    while (head < tail) {
        int32_t x = queue[head++];
        for (int32_t e = rp[x]; e < rp[x + 1]; ++e) {
            int32_t y = ci[e];
            if (dist[y] < 0) {
                dist[y] = dist[x] + 1;
                queue[tail++] = y;
            }
        }
    }
    return tail;
}

/* d(w,S) = min_{s in S} d(w,s)  (Section 2), one BFS per member of S. */
int or_group_dist(int64_t n, const int32_t *rp, const int32_t *ci, const int32_t *S, int32_t ns,
                  int32_t *dS) {
    if (ns < 1) return OR_EINVAL;
    int32_t *d = (int32_t *)malloc(sizeof(int32_t) * (size_t)n);
    int32_t *q = (int32_t *)malloc(sizeof(int32_t) * (size_t)n);
    int rc = OR_OK;
    for (int32_t i = 0; i < ns && rc == OR_OK; ++i) {
        if (S[i] < 0 || S[i] >= n) { rc = OR_EINVAL; break; }
        if (or_bfs(n, rp, ci, S[i], d, q) != n) { rc = OR_EDISCONNECTED; break; }
        for (int64_t w = 0; w < n; ++w)
            if (i == 0 || d[w] < dS[w]) dS[w] = d[w];
    }
    free(d); free(q);
    return rc;
}

/* F(S) = sum_w d(S,w); returns -1 on error. */
int64_t or_farness(int64_t n, const int32_t *rp, const int32_t *ci, const int32_t *S, int32_t ns) {
    int32_t *dS = (int32_t *)malloc(sizeof(int32_t) * (size_t)n);
    int64_t F = -1;
    if (or_group_dist(n, rp, ci, S, ns, dS) == OR_OK) {
        F = 0;
        for (int64_t w = 0; w < n; ++w) F += dS[w];
    }
    free(dS);
    return F;
}

/* F({v}) for every v: n full BFS (the numerator-free farness behind c(v), Section 2). */
int or_farness_all(int64_t n, const int32_t *rp, const int32_t *ci, int64_t *F) {
    int rc = OR_OK;
#pragma omp parallel
    {
        int32_t *d = (int32_t *)malloc(sizeof(int32_t) * (size_t)n);
        int32_t *q = (int32_t *)malloc(sizeof(int32_t) * (size_t)n);
#pragma omp for schedule(dynamic, 16)
        for (int64_t v = 0; v < n; ++v) {
            int64_t r = or_bfs(n, rp, ci, (int32_t)v, d, q);
            int64_t s = 0;
            for (int64_t w = 0; w < n; ++w) s += d[w];
            F[v] = s;
            if (r != n) {
#pragma omp atomic write
                rc = OR_EDISCONNECTED;
            }
        }
        free(d); free(q);
    }
    return rc;
}

/*
 * g(v,S) = F(S) - F(S u {v}) = sum_w (d_S[w] - min(d_S[w], d(v,w)))
 * with a full BFS from v (the sum that Algorithm "mem-greedy" forms after its
 * SSSP from u, written as a difference).
 */
int64_t or_gain(int64_t n, const int32_t *rp, const int32_t *ci, const int32_t *dS, int32_t v) {
    int32_t *d = (int32_t *)malloc(sizeof(int32_t) * (size_t)n);
    int32_t *q = (int32_t *)malloc(sizeof(int32_t) * (size_t)n);
    or_bfs(n, rp, ci, v, d, q);
    int64_t g = 0;
    for (int64_t w = 0; w < n; ++w) {
        int32_t m = d[w] < dS[w] ? d[w] : dS[w];
        g += (int64_t)(dS[w] - m);
    }
    free(d); free(q);
    return g;
}

/* gains for a list of candidates (parallel over candidates), full BFS each */
int or_gains(int64_t n, const int32_t *rp, const int32_t *ci, const int32_t *dS, const int32_t *cand,
             int64_t count, int64_t *gain) {
#pragma omp parallel
    {
        int32_t *d = (int32_t *)malloc(sizeof(int32_t) * (size_t)n);
        int32_t *q = (int32_t *)malloc(sizeof(int32_t) * (size_t)n);
#pragma omp for schedule(dynamic, 4)
        for (int64_t i = 0; i < count; ++i) {
            or_bfs(n, rp, ci, cand[i], d, q);
            int64_t g = 0;
            for (int64_t w = 0; w < n; ++w) {
                int32_t m = d[w] < dS[w] ? d[w] : dS[w];
                g += (int64_t)(dS[w] - m);
            }
            gain[i] = g;
        }
        free(d); free(q);
    }
    return OR_OK;
}

/* --------------------------------------------------------- input check --- */

/*
 * The input contract of the method (Section 2: a connected, undirected,
 * unweighted graph), checked in full: row_ptr starts at 0 and never
 * decreases, ids lie in [0, n), every row is strictly ascending (so no
 * duplicate edges), no self-loops, every edge (u, v) has its reverse (v, u),
 * and one BFS from node 0 reaches every node.  Returns OR_OK, OR_EINVAL,
 * OR_ENOTSYM or OR_EDISCONNECTED.
 */
int or_validate_graph(int64_t n, const int32_t *rp, const int32_t *ci, int32_t directed);

int or_validate(int64_t n, const int32_t *rp, const int32_t *ci) { return or_validate_graph(n, rp, ci, 0); }

/*
 * directed = 1: the rows are out-neighbour lists of a directed graph (the
 * strongly connected directed graphs Section 2 also admits): the same range,
 * order, self-loop and duplicate checks, no symmetry, and instead of one
 * component, strong connectivity -- a BFS from node 0 over the arcs and one
 * over the reversed arcs both reach every node.
 */
int or_validate_graph(int64_t n, const int32_t *rp, const int32_t *ci, int32_t directed) {
    if (n < 1 || rp[0] != 0) return OR_EINVAL;
    for (int64_t u = 0; u < n; ++u) {
        if (rp[u + 1] < rp[u]) return OR_EINVAL;
        for (int32_t e = rp[u]; e < rp[u + 1]; ++e) {
            int32_t v = ci[e];
            if (v < 0 || v >= n || v == u) return OR_EINVAL;
            if (e > rp[u] && ci[e - 1] >= v) return OR_EINVAL;
        }
    }
    if (directed) {
        /* reach from node 0 along the arcs, then along the reversed arcs */
        int32_t *d = (int32_t *)malloc(sizeof(int32_t) * (size_t)n);
        int32_t *q = (int32_t *)malloc(sizeof(int32_t) * (size_t)n);
        int64_t r = or_bfs(n, rp, ci, 0, d, q);
        int64_t nnz = rp[n];
        int32_t *trp = (int32_t *)calloc((size_t)n + 1, sizeof(int32_t));
        int32_t *tci = (int32_t *)malloc(sizeof(int32_t) * (size_t)(nnz > 0 ? nnz : 1));
        for (int64_t e = 0; e < nnz; ++e) trp[ci[e] + 1]++;
        for (int64_t v = 0; v < n; ++v) trp[v + 1] += trp[v];
        int32_t *fill = (int32_t *)malloc(sizeof(int32_t) * (size_t)n);
        memcpy(fill, trp, sizeof(int32_t) * (size_t)n);
        for (int64_t u = 0; u < n; ++u)
            for (int32_t e = rp[u]; e < rp[u + 1]; ++e) tci[fill[ci[e]]++] = (int32_t)u;
        int64_t rr = or_bfs(n, trp, tci, 0, d, q);
        free(d); free(q); free(trp); free(tci); free(fill);
        return (r == n && rr == n) ? OR_OK : OR_EDISCONNECTED;
    }
    for (int64_t u = 0; u < n; ++u)
        for (int32_t e = rp[u]; e < rp[u + 1]; ++e) {
            int32_t v = ci[e], lo = rp[v], hi = rp[v + 1];
            while (lo < hi) { /* first entry of row v that is >= u */
                int32_t mid = lo + (hi - lo) / 2;
                if (ci[mid] < u) lo = mid + 1; else hi = mid;
            }
            if (lo == rp[v + 1] || ci[lo] != u) return OR_ENOTSYM;
        }
    int32_t *d = (int32_t *)malloc(sizeof(int32_t) * (size_t)n);
    int32_t *q = (int32_t *)malloc(sizeof(int32_t) * (size_t)n);
    int64_t r = or_bfs(n, rp, ci, 0, d, q);
    free(d); free(q);
    return r == n ? OR_OK : OR_EDISCONNECTED;
}

/* --------------------------------------------------------------- tier A --- */

/*
 * Plain greedy (Section 3.2, with the memory-efficient d_S vector of Section 4
 * but no pruning and no skipping):
 *   s_1 = argmin_v F({v});
 *   s_{i+1} = argmin_{v notin S_i} F(S_i u {v});  ties -> smallest id.
 * Outputs group[0..k-1] in pick order and Fout[i] = F(S_{i+1}).
 * gains, when not NULL, receives (k-1) rows of n entries: row r holds
 * g(v, S_{r+1}) for v notin S_{r+1} and -1 for members.
 * The loop asserts the invariants that follow from the definitions and from
 * the supermodularity lemma of Section 3.2; a violation returns OR_EINVARIANT.
 */
int or_greedy(int64_t n, const int32_t *rp, const int32_t *ci, int32_t k, int32_t *group,
              int64_t *Fout, int64_t *gains, int32_t directed) {
    if (k < 1 || k > n) return OR_EINVAL;
    {
        int vrc = or_validate_graph(n, rp, ci, directed);
        if (vrc != OR_OK) return vrc;
    }
    int64_t *Fv = (int64_t *)malloc(sizeof(int64_t) * (size_t)n);
    int64_t *prev = (int64_t *)malloc(sizeof(int64_t) * (size_t)n);
    int32_t *dS = (int32_t *)malloc(sizeof(int32_t) * (size_t)n);
    int32_t *dsnew = (int32_t *)malloc(sizeof(int32_t) * (size_t)n);
    int32_t *q = (int32_t *)malloc(sizeof(int32_t) * (size_t)n);
    uint8_t *inS = (uint8_t *)calloc((size_t)n, 1);
    int rc = or_farness_all(n, rp, ci, Fv);
    if (rc != OR_OK) goto done;
    {
        int32_t s = 0;
        for (int64_t v = 1; v < n; ++v)
            if (Fv[v] < Fv[s]) s = (int32_t)v;
        group[0] = s;
        inS[s] = 1;
        or_bfs(n, rp, ci, s, dS, q);
        int64_t F = Fv[s];
        Fout[0] = F;
        for (int64_t v = 0; v < n; ++v) prev[v] = INT64_MAX;
        for (int32_t i = 1; i < k; ++i) {
            int bad = 0;
#pragma omp parallel
            {
                int32_t *d = (int32_t *)malloc(sizeof(int32_t) * (size_t)n);
                int32_t *qq = (int32_t *)malloc(sizeof(int32_t) * (size_t)n);
#pragma omp for schedule(dynamic, 4)
                for (int64_t v = 0; v < n; ++v) {
                    if (inS[v]) { Fv[v] = INT64_MAX; continue; }
                    or_bfs(n, rp, ci, (int32_t)v, d, qq);
                    int64_t t = 0;
                    for (int64_t w = 0; w < n; ++w) t += (d[w] < dS[w] ? d[w] : dS[w]);
                    Fv[v] = t;
                }
                free(d); free(qq);
            }
            int32_t best = -1;
            for (int64_t v = 0; v < n; ++v) {
                if (inS[v]) continue;
                int64_t g = F - Fv[v];
                /* gains never increase between rounds (supermodularity lemma) */
                if (g > prev[v]) bad = 1;
                /* v itself moves from d_S[v] >= 1 to 0 */
                if (g < dS[v] || dS[v] < 1) bad = 1;
                prev[v] = g;
                if (best < 0 || Fv[v] < Fv[best]) best = (int32_t)v;
            }
            if (gains) {
                int64_t *row = gains + (int64_t)(i - 1) * n;
                for (int64_t v = 0; v < n; ++v) row[v] = inS[v] ? -1 : F - Fv[v];
            }
            /* add the pick; d_S <- min(d_S, d(s,.)) (the update of Algorithm "mem-greedy") */
            or_bfs(n, rp, ci, best, dsnew, q);
            int64_t sum = 0;
            for (int64_t w = 0; w < n; ++w) {
                int32_t m = dsnew[w] < dS[w] ? dsnew[w] : dS[w];
                if (m > dS[w]) bad = 1; /* d_S never increases */
                dS[w] = m;
                sum += m;
            }
            if (sum != Fv[best]) bad = 1;            /* F(S) == sum_w d_S[w] */
            if (!(Fv[best] < F)) bad = 1;            /* strictly decreasing while |S| < n */
            F = Fv[best];
            group[i] = best;
            inS[best] = 1;
            Fout[i] = F;
            if (bad) { rc = OR_EINVARIANT; goto done; }
        }
    }
done:
    free(Fv); free(prev); free(dS); free(dsnew); free(q); free(inS);
    return rc;
}

/* --------------------------------------------------------------- tier B --- */

/*
 * Pruned BFS from u (Section 4.1): a node w reached at level l is counted and
 * expanded only if l < d_S[w]; otherwise its whole BFS subtree cannot improve
 * on S and is not entered.  Returns g(u,S) = sum over the counted w of
 * (d_S[w] - l).  `mark` holds per-thread visit stamps.
 * *edges receives sum of deg(w) over counted w (the adjacency entries this
 * search scans), *visited the number of counted nodes.
 */
static int64_t pruned_gain(const int32_t *rp, const int32_t *ci, const int32_t *dS, int32_t u,
                           int32_t *lvl, int32_t *mark, int32_t stamp, int32_t *q, int64_t *edges,
                           int64_t *visited) {
    int64_t g = 0, e_cnt = 0, v_cnt = 0;
    if (!(0 < dS[u])) { *edges = 0; *visited = 0; return 0; } /* u in S */
    int64_t head = 0, tail = 0;
    mark[u] = stamp; lvl[u] = 0; q[tail++] = u;
    while (head < tail) {
        int32_t x = q[head++];
        g += dS[x] - lvl[x];
        v_cnt += 1;
        e_cnt += rp[x + 1] - rp[x];
        for (int32_t e = rp[x]; e < rp[x + 1]; ++e) {
            int32_t y = ci[e];
            if (mark[y] == stamp) continue;
            mark[y] = stamp;
            int32_t l = lvl[x] + 1;
            if (l < dS[y]) { lvl[y] = l; q[tail++] = y; }
        }
    }
    *edges = e_cnt; *visited = v_cnt;
    return g;
}

/*
 * Early exit inside a candidate's pruned BFS: a BFScut-style bound (Section
 * 3.1) on the pruned BFS of Section 4.1.  After the nodes at distance l from
 * u are claimed (gain so far g, e_l the adjacency entries of the nodes
 * claimed at distance l), every node u can still claim lies at distance
 * >= l+1 with d_S >= l+2: at most e_l of them at distance l+1 (each is a
 * neighbour of a node claimed at distance l), each worth 1 + (d_S - l - 2),
 * and the others worth at most d_S - l - 2.  Hence
 *     g(u,S) <= g + e_l + T[l+1],   T[j] = sum_w max(0, d_S[w] - j - 1).
 * The test is made after every level that claimed a node while a deeper
 * level can still claim one (l + 1 < max d_S).  When the bound cannot beat
 * (thr, thr_id) -- bound < thr, or bound == thr and u > thr_id -- the search
 * stops, *cut = 1, and the bound is returned (an upper bound on the gain,
 * kept as the candidate's stale gain).  thr_id < 0: no threshold.
 * *edges and *visited count the nodes claimed until the stop.
 */
static int64_t pruned_gain_cut(const int32_t *rp, const int32_t *ci, const int32_t *dS, int32_t u,
                               int32_t *lvl, int32_t *mark, int32_t stamp, int32_t *q, const int64_t *T,
                               int32_t maxd, int64_t thr, int32_t thr_id, int64_t *edges, int64_t *visited,
                               int *cut) {
    *cut = 0;
    if (!(0 < dS[u])) { *edges = 0; *visited = 0; return 0; } /* u in S */
    int64_t g = dS[u], e_cnt = rp[u + 1] - rp[u], v_cnt = 1;
    int64_t lo = 0, hi = 1;
    mark[u] = stamp; lvl[u] = 0; q[0] = u;
    for (int32_t l = 0; lo < hi; ++l) {
        if (thr_id >= 0 && l + 1 < maxd) {
            int64_t el = 0;
            for (int64_t i = lo; i < hi; ++i) el += rp[q[i] + 1] - rp[q[i]];
            const int64_t bound = g + el + T[l + 1];
            if (bound < thr || (bound == thr && u > thr_id)) {
                *cut = 1; *edges = e_cnt; *visited = v_cnt;
                return bound;
            }
        }
        int64_t tail = hi;
        for (int64_t i = lo; i < hi; ++i) {
            int32_t x = q[i];
            for (int32_t e = rp[x]; e < rp[x + 1]; ++e) {
                int32_t y = ci[e];
                if (mark[y] == stamp) continue;
                mark[y] = stamp;
                if (l + 1 < dS[y]) {
                    lvl[y] = l + 1;
                    q[tail++] = y;
                    g += dS[y] - (l + 1);
                    e_cnt += rp[y + 1] - rp[y];
                    v_cnt += 1;
                }
            }
        }
        lo = hi; hi = tail;
    }
    *edges = e_cnt; *visited = v_cnt;
    return g;
}

/* T[j] = sum_w max(0, d_S[w] - j - 1) for j = 0..maxd (T[maxd] = 0), and max d_S. */
static int32_t tail_sums(int64_t n, const int32_t *dS, int64_t **T_out) {
    int32_t maxd = 0;
    for (int64_t w = 0; w < n; ++w) if (dS[w] > maxd) maxd = dS[w];
    int64_t *cnt = (int64_t *)calloc((size_t)maxd + 2, sizeof(int64_t));
    int64_t *T = (int64_t *)calloc((size_t)maxd + 2, sizeof(int64_t));
    for (int64_t w = 0; w < n; ++w) cnt[dS[w]]++;
    for (int32_t j = 0; j <= maxd; ++j)
        for (int32_t d = j + 2; d <= maxd; ++d) T[j] += (int64_t)(d - j - 1) * cnt[d];
    free(cnt);
    *T_out = T;
    return maxd;
}

/* Full BFS from v with the BFScut lower bound of Section 3.1; returns F({v})
 * or -1 when the bound proves (F({v}), v) cannot beat (bestF, bestId). */
static int64_t bfscut(int64_t n, const int32_t *rp, const int32_t *ci, int32_t v, int64_t bestF,
                      int32_t bestId, int32_t *lvl, int32_t *mark, int32_t stamp, int32_t *q) {
    (void)lvl;
    int64_t lo = 0, hi = 1, sum = 0;
    mark[v] = stamp; q[0] = v;
    for (int64_t d = 0; lo < hi; ++d) {
        /* every node at distance <= d is in q[0..hi); the others are at >= d+1 */
        int64_t lb = sum + (d + 1) * (n - hi);
        if (bestId >= 0 && (lb > bestF || (lb == bestF && v > bestId))) return -1;
        int64_t tail = hi;
        for (int64_t i = lo; i < hi; ++i) {
            int32_t x = q[i];
            for (int32_t e = rp[x]; e < rp[x + 1]; ++e) {
                int32_t y = ci[e];
                if (mark[y] == stamp) continue;
                mark[y] = stamp;
                q[tail++] = y;
            }
        }
        sum += (d + 1) * (tail - hi);
        lo = hi; hi = tail;
    }
    if (hi != n) return -2;
    return sum;
}

/*
 * Greedy++ (Section 4): first node by top-k closeness (k = 1) visiting nodes
 * by decreasing degree (ties: ascending id) with BFScut; then rounds of the
 * lazy scan.  In each round candidates are taken in ascending id order;
 * a candidate u is skipped when its gain from an earlier round (an upper
 * bound by supermodularity) satisfies
 *     ub[u] < best_gain  or  (ub[u] == best_gain and u > best_id).
 * Non-skipped candidates are evaluated with pruned BFS in blocks of `block`
 * (parallel inside a block); the best is updated between blocks, so the
 * evaluation counts do not depend on thread timing.  In the first round
 * after s_1 no bound exists and every candidate is evaluated.
 * evals[i] (i = 1..k-1) receives the number of evaluations in round i;
 * edges (nullable) receives, per round, the summed adjacency entries scanned.
 *
 * cut_mode 1 adds the early exit of pruned_gain_cut to the first round, 2 to
 * every round (0: none).  In the first round the cut_seed candidates of
 * largest degree are evaluated first, exactly, and every other candidate of
 * the round against their best (fixed for the round); in later rounds a
 * batch is cut against the best of the batches before it.  A cut candidate
 * keeps its bound as stale gain; it counts as an evaluation, and cuts
 * (nullable) receives the cut candidates per round.  The picks never change.
 */
int or_greedypp(int64_t n, const int32_t *rp, const int32_t *ci, int32_t k, int32_t block,
                int32_t growth, int32_t *group, int64_t *Fout, int64_t *evals, int64_t *edges,
                int32_t cut_mode, int32_t cut_seed, int64_t *cuts, int32_t directed) {
    if (k < 1 || k > n || block < 1 || growth < 1 || growth > 8) return OR_EINVAL;
    if (cut_mode < 0 || cut_mode > 2 || (cut_mode > 0 && cut_seed < 1)) return OR_EINVAL;
    {
        int vrc = or_validate_graph(n, rp, ci, directed);
        if (vrc != OR_OK) return vrc;
    }
    /* the largest batch: block grows by `growth` per batch of a round, up to 16 x block */
    int64_t maxb = growth > 1 ? 16 * (int64_t)block : block;
    if (maxb > n) maxb = n;
    int nthr = 1;
#ifdef _OPENMP
    nthr = omp_get_max_threads();
#endif
    int32_t **lvl = (int32_t **)malloc(sizeof(void *) * (size_t)nthr);
    int32_t **mark = (int32_t **)malloc(sizeof(void *) * (size_t)nthr);
    int32_t **qs = (int32_t **)malloc(sizeof(void *) * (size_t)nthr);
    int32_t *stamps = (int32_t *)calloc((size_t)nthr, sizeof(int32_t));
    for (int t = 0; t < nthr; ++t) {
        lvl[t] = (int32_t *)malloc(sizeof(int32_t) * (size_t)n);
        mark[t] = (int32_t *)calloc((size_t)n, sizeof(int32_t));
        qs[t] = (int32_t *)malloc(sizeof(int32_t) * (size_t)n);
    }
    int32_t *order = (int32_t *)malloc(sizeof(int32_t) * (size_t)n);
    int32_t *dS = (int32_t *)malloc(sizeof(int32_t) * (size_t)n);
    int32_t *dnew = (int32_t *)malloc(sizeof(int32_t) * (size_t)n);
    int64_t *ub = (int64_t *)malloc(sizeof(int64_t) * (size_t)n);
    int32_t *batch = (int32_t *)malloc(sizeof(int32_t) * (size_t)maxb);
    int64_t *bg = (int64_t *)malloc(sizeof(int64_t) * (size_t)maxb);
    int64_t *be = (int64_t *)malloc(sizeof(int64_t) * (size_t)maxb);
    int *bc = (int *)malloc(sizeof(int) * (size_t)maxb);
    int rc = OR_OK;

    /* first node: decreasing degree, BFScut (sequential) */
    for (int64_t v = 0; v < n; ++v) order[v] = (int32_t)v;
    {
        /* counting sort by degree, descending, stable in id */
        int32_t maxd = 0;
        for (int64_t v = 0; v < n; ++v) if (rp[v + 1] - rp[v] > maxd) maxd = rp[v + 1] - rp[v];
        int64_t *cnt = (int64_t *)calloc((size_t)maxd + 2, sizeof(int64_t));
        for (int64_t v = 0; v < n; ++v) cnt[maxd - (rp[v + 1] - rp[v]) + 1]++;
        for (int32_t d = 0; d <= maxd; ++d) cnt[d + 1] += cnt[d];
        for (int64_t v = 0; v < n; ++v) order[cnt[maxd - (rp[v + 1] - rp[v])]++] = (int32_t)v;
        free(cnt);
    }
    int64_t bestF = -1;
    int32_t bestId = -1;
    for (int64_t i = 0; i < n; ++i) {
        int32_t v = order[i];
        int32_t st = ++stamps[0];
        int64_t F = bfscut(n, rp, ci, v, bestF, bestId, lvl[0], mark[0], st, qs[0]);
        if (F == -2) { rc = OR_EDISCONNECTED; goto done; }
        if (F < 0) continue;
        if (bestId < 0 || F < bestF || (F == bestF && v < bestId)) { bestF = F; bestId = v; }
    }
    group[0] = bestId;
    Fout[0] = bestF;
    or_bfs(n, rp, ci, bestId, dS, qs[0]);
    for (int64_t v = 0; v < n; ++v) ub[v] = INT64_MAX;
    if (evals) evals[0] = 0;
    if (edges) edges[0] = 0;
    if (cuts) cuts[0] = 0;
    int64_t F = bestF;
    for (int32_t r = 1; r < k; ++r) {
        int64_t bgain = -1;
        int32_t bid = -1;
        int64_t pos = 0, nev = 0, ned = 0, ncut = 0;
        int64_t cur = block < maxb ? block : maxb; /* batch size; the first round takes every node anyway */
        /* early exit inside the candidates' BFS: in the first round (mode 1)
           or every round (mode 2) */
        const int use_cut = cut_mode == 2 || (cut_mode == 1 && r == 1);
        int64_t *T = NULL;
        int32_t maxd = 0;
        if (use_cut) maxd = tail_sums(n, dS, &T);
        if (use_cut && r == 1) {
            /* the cut_seed candidates of largest degree (ties: smaller id)
               exactly, then every other candidate against their best, which
               stays fixed for the rest of the round; the order of those
               evaluations cannot change any result */
            int32_t *all = (int32_t *)malloc(sizeof(int32_t) * (size_t)n);
            int64_t *ag = (int64_t *)malloc(sizeof(int64_t) * (size_t)n);
            int64_t *ae = (int64_t *)malloc(sizeof(int64_t) * (size_t)n);
            int *ac = (int *)calloc((size_t)n, sizeof(int));
            uint8_t *seeded = (uint8_t *)calloc((size_t)n, 1);
            int64_t ns = 0, na = 0;
            for (int64_t i = 0; i < n && ns < cut_seed; ++i)
                if (dS[order[i]] > 0) { all[ns++] = order[i]; seeded[order[i]] = 1; }
            for (int pass = 0; pass < 2; ++pass) {
                int64_t b0 = pass == 0 ? 0 : ns;
                if (pass == 1) {
                    na = ns;
                    for (int64_t u = 0; u < n; ++u)
                        if (dS[u] > 0 && !seeded[u]) all[na++] = (int32_t)u;
                }
                int64_t b1 = pass == 0 ? ns : na;
                const int64_t thr = bgain;
                const int32_t thr_id = pass == 0 ? -1 : bid;
#pragma omp parallel for schedule(dynamic, 16)
                for (int64_t j = b0; j < b1; ++j) {
                    int t = 0;
#ifdef _OPENMP
                    t = omp_get_thread_num();
#endif
                    int64_t vis;
                    int32_t st = ++stamps[t];
                    ag[j] = pruned_gain_cut(rp, ci, dS, all[j], lvl[t], mark[t], st, qs[t], T, maxd, thr,
                                            thr_id, &ae[j], &vis, &ac[j]);
                }
                for (int64_t j = b0; j < b1; ++j) {
                    int32_t u = all[j];
                    ub[u] = ag[j];
                    ned += ae[j];
                    ncut += ac[j];
                    if (ac[j]) continue; /* a bound below the threshold, never the best */
                    if (bid < 0 || ag[j] > bgain || (ag[j] == bgain && u < bid)) { bgain = ag[j]; bid = u; }
                }
                nev += b1 - b0;
            }
            free(all); free(ag); free(ae); free(ac); free(seeded);
            pos = n; /* every candidate done */
        }
        for (; pos < n;) {
            int32_t nb = 0;
            while (pos < n && nb < cur) {
                int32_t u = (int32_t)pos++;
                if (dS[u] == 0) continue; /* u in S */
                if (bid >= 0 && (ub[u] < bgain || (ub[u] == bgain && u > bid))) continue;
                batch[nb++] = u;
            }
            if (nb == 0) break;
            const int64_t thr = bgain;
            const int32_t thr_id = use_cut ? bid : -1;
#pragma omp parallel for schedule(dynamic, 1) if (nb > 1)
            for (int32_t j = 0; j < nb; ++j) {
                int t = 0;
#ifdef _OPENMP
                t = omp_get_thread_num();
#endif
                int64_t vis;
                int32_t st = ++stamps[t];
                if (use_cut)
                    bg[j] = pruned_gain_cut(rp, ci, dS, batch[j], lvl[t], mark[t], st, qs[t], T, maxd, thr,
                                            thr_id, &be[j], &vis, &bc[j]);
                else {
                    bc[j] = 0;
                    bg[j] = pruned_gain(rp, ci, dS, batch[j], lvl[t], mark[t], st, qs[t], &be[j], &vis);
                }
            }
            for (int32_t j = 0; j < nb; ++j) {
                int32_t u = batch[j];
                ub[u] = bg[j];
                ned += be[j];
                ncut += bc[j];
                if (bc[j]) continue;
                if (bid < 0 || bg[j] > bgain || (bg[j] == bgain && u < bid)) { bgain = bg[j]; bid = u; }
            }
            nev += nb;
            /* the skip test sees the threshold only between batches: the
             * batch sizes decide how many candidates are evaluated, never
             * which one is picked */
            if (r >= 2 && cur * growth <= maxb) cur *= growth;
            else if (r >= 2) cur = maxb;
        }
        free(T);
        if (evals) evals[r] = nev;
        if (edges) edges[r] = ned;
        if (cuts) cuts[r] = ncut;
        /* pick and update d_S by a pruned BFS from the pick (Section 4.1: only
         * nodes with d(s,w) < d_S[w] change) */
        group[r] = bid;
        {
            int32_t st = ++stamps[0];
            int32_t *q = qs[0], *mk = mark[0], *lv = lvl[0];
            int64_t head = 0, tail = 0;
            mk[bid] = st; lv[bid] = 0; q[tail++] = bid;
            while (head < tail) {
                int32_t x = q[head++];
                dnew[x] = lv[x];
                for (int32_t e = rp[x]; e < rp[x + 1]; ++e) {
                    int32_t y = ci[e];
                    if (mk[y] == st) continue;
                    mk[y] = st;
                    if (lv[x] + 1 < dS[y]) { lv[y] = lv[x] + 1; q[tail++] = y; }
                }
            }
            for (int64_t i = 0; i < tail; ++i) dS[q[i]] = dnew[q[i]];
        }
        F -= bgain;
        Fout[r] = F;
    }
done:
    for (int t = 0; t < nthr; ++t) { free(lvl[t]); free(mark[t]); free(qs[t]); }
    free(lvl); free(mark); free(qs); free(stamps);
    free(order); free(dS); free(dnew); free(ub); free(batch); free(bg); free(be); free(bc);
    return rc;
}

/*
 * The early-exit search (pruned_gain_cut) for a candidate list against one
 * threshold: out[i] is the exact gain, or the bound at which the search
 * stopped when cut[i] = 1.
 */
int or_gains_cut(int64_t n, const int32_t *rp, const int32_t *ci, const int32_t *dS, const int32_t *cand,
                 int64_t count, int64_t thr, int32_t thr_id, int64_t *out, int32_t *cut) {
    int64_t *T = NULL;
    const int32_t maxd = tail_sums(n, dS, &T);
#pragma omp parallel
    {
        int32_t *lv = (int32_t *)malloc(sizeof(int32_t) * (size_t)n);
        int32_t *mk = (int32_t *)calloc((size_t)n, sizeof(int32_t));
        int32_t *q = (int32_t *)malloc(sizeof(int32_t) * (size_t)n);
        int32_t st = 0;
#pragma omp for schedule(dynamic, 16)
        for (int64_t i = 0; i < count; ++i) {
            int64_t e, v;
            int c;
            out[i] = pruned_gain_cut(rp, ci, dS, cand[i], lv, mk, ++st, q, T, maxd, thr, thr_id, &e, &v, &c);
            cut[i] = c;
        }
        free(lv); free(mk); free(q);
    }
    free(T);
    return OR_OK;
}

/*
 * Pruned-BFS statistics for a candidate list under a given d_S: per candidate
 * the gain, the number of counted nodes |V(v)| and the adjacency entries
 * scanned sum_{w in V(v)} deg(w).  Used to count algorithmic work.
 */
int or_pruned_stats(int64_t n, const int32_t *rp, const int32_t *ci, const int32_t *dS,
                    const int32_t *cand, int64_t count, int64_t *gain, int64_t *visited,
                    int64_t *edges) {
#pragma omp parallel
    {
        int32_t *lv = (int32_t *)malloc(sizeof(int32_t) * (size_t)n);
        int32_t *mk = (int32_t *)calloc((size_t)n, sizeof(int32_t));
        int32_t *q = (int32_t *)malloc(sizeof(int32_t) * (size_t)n);
        int32_t st = 0;
#pragma omp for schedule(dynamic, 16)
        for (int64_t i = 0; i < count; ++i) {
            int64_t e, v;
            gain[i] = pruned_gain(rp, ci, dS, cand[i], lv, mk, ++st, q, &e, &v);
            if (visited) visited[i] = v;
            if (edges) edges[i] = e;
        }
        free(lv); free(mk); free(q);
    }
    return OR_OK;
}

int or_num_threads(void) {
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

/* ------------------------------------------------------- weighted graphs --- */
/*
 * Section 2 names SSSP on weighted graphs as the distance computation in
 * general (BFS is its unweighted special case); Section 4.1's pruning is
 * stated for SSSP.  Here every arc e of the CSR carries an integer weight
 * w[e] >= 1 (uint8; an undirected edge has the same weight in both rows), and
 * d(u, v) is the least total weight of a path.  Everything below is the
 * textbook form: Dijkstra's algorithm with a binary heap of (distance, node)
 * pairs and lazy deletion.
 */

typedef struct { int64_t d; int32_t v; } or_hent;

static void heap_push(or_hent *h, int64_t *len, int64_t d, int32_t v) {
    int64_t i = (*len)++;
    h[i].d = d; h[i].v = v;
    while (i > 0) {
        int64_t p = (i - 1) / 2;
        if (h[p].d < h[i].d || (h[p].d == h[i].d && h[p].v <= h[i].v)) break;
        or_hent t = h[p]; h[p] = h[i]; h[i] = t; i = p;
    }
}

static or_hent heap_pop(or_hent *h, int64_t *len) {
    or_hent top = h[0];
    h[0] = h[--(*len)];
    int64_t i = 0;
    for (;;) {
        int64_t l = 2 * i + 1, r = l + 1, m = i;
        if (l < *len && (h[l].d < h[m].d || (h[l].d == h[m].d && h[l].v < h[m].v))) m = l;
        if (r < *len && (h[r].d < h[m].d || (h[r].d == h[m].d && h[r].v < h[m].v))) m = r;
        if (m == i) break;
        or_hent t = h[m]; h[m] = h[i]; h[i] = t; i = m;
    }
    return top;
}

/* Dijkstra from src: dist[w] = d(src, w) or -1 if unreachable; returns #reached.
 * heap: capacity nnz + 1 entries. */
static int64_t sssp_w(int64_t n, const int32_t *rp, const int32_t *ci, const uint8_t *w, int32_t src,
                      int32_t *dist, or_hent *heap) {
    for (int64_t i = 0; i < n; ++i) dist[i] = -1;
    int64_t len = 0, reached = 0;
    /* dist[w]: -1 unseen, -(t + 2) while w waits in the heap with tentative
     * distance t, d(src, w) once settled */
    dist[src] = -2;
    heap_push(heap, &len, 0, src);
    while (len > 0) {
        or_hent t = heap_pop(heap, &len);
        if (dist[t.v] >= 0) continue;             /* already settled */
        if (-(int64_t)dist[t.v] - 2 != t.d) continue; /* a stale entry */
        dist[t.v] = (int32_t)t.d;
        ++reached;
        for (int32_t e = rp[t.v]; e < rp[t.v + 1]; ++e) {
            int32_t y = ci[e];
            if (dist[y] >= 0) continue;
            int64_t nd = t.d + w[e];
            if (dist[y] == -1 || nd < -(int64_t)dist[y] - 2) {
                dist[y] = (int32_t)(-(nd + 2));
                heap_push(heap, &len, nd, y);
            }
        }
    }
    return reached;
}

int64_t or_sssp_w(int64_t n, const int32_t *rp, const int32_t *ci, const uint8_t *w, int32_t src,
                  int32_t *dist) {
    or_hent *heap = (or_hent *)malloc(sizeof(or_hent) * (size_t)(rp[n] + 2));
    int64_t r = sssp_w(n, rp, ci, w, src, dist, heap);
    free(heap);
    return r;
}

/* structure (as or_validate_graph), every weight >= 1, and for undirected
 * graphs the same weight in both rows of an edge */
int or_validate_w(int64_t n, const int32_t *rp, const int32_t *ci, const uint8_t *w, int32_t directed) {
    int rc = or_validate_graph(n, rp, ci, directed);
    if (rc != OR_OK) return rc;
    for (int64_t u = 0; u < n; ++u)
        for (int32_t e = rp[u]; e < rp[u + 1]; ++e) {
            if (w[e] < 1) return OR_EINVAL;
            if (directed) continue;
            int32_t v = ci[e], lo = rp[v], hi = rp[v + 1];
            while (lo < hi) {
                int32_t mid = lo + (hi - lo) / 2;
                if (ci[mid] < u) lo = mid + 1; else hi = mid;
            }
            if (w[lo] != w[e]) return OR_ENOTSYM;
        }
    return OR_OK;
}

int or_group_dist_w(int64_t n, const int32_t *rp, const int32_t *ci, const uint8_t *w, const int32_t *S,
                    int32_t ns, int32_t *dS) {
    if (ns < 1) return OR_EINVAL;
    int32_t *d = (int32_t *)malloc(sizeof(int32_t) * (size_t)n);
    or_hent *heap = (or_hent *)malloc(sizeof(or_hent) * (size_t)(rp[n] + 2));
    int rc = OR_OK;
    for (int32_t i = 0; i < ns && rc == OR_OK; ++i) {
        if (S[i] < 0 || S[i] >= n) { rc = OR_EINVAL; break; }
        if (sssp_w(n, rp, ci, w, S[i], d, heap) != n) { rc = OR_EDISCONNECTED; break; }
        for (int64_t v = 0; v < n; ++v)
            if (i == 0 || d[v] < dS[v]) dS[v] = d[v];
    }
    free(d); free(heap);
    return rc;
}

int or_farness_all_w(int64_t n, const int32_t *rp, const int32_t *ci, const uint8_t *w, int64_t *F) {
    int rc = OR_OK;
#pragma omp parallel
    {
        int32_t *d = (int32_t *)malloc(sizeof(int32_t) * (size_t)n);
        or_hent *heap = (or_hent *)malloc(sizeof(or_hent) * (size_t)(rp[n] + 2));
#pragma omp for schedule(dynamic, 16)
        for (int64_t v = 0; v < n; ++v) {
            int64_t r = sssp_w(n, rp, ci, w, (int32_t)v, d, heap);
            int64_t s = 0;
            for (int64_t u = 0; u < n; ++u) s += d[u];
            F[v] = s;
            if (r != n) {
#pragma omp atomic write
                rc = OR_EDISCONNECTED;
            }
        }
        free(d); free(heap);
    }
    return rc;
}

/* g(v,S) = sum_u (dS[u] - min(dS[u], d(v,u))) with a full Dijkstra from v */
int or_gains_w(int64_t n, const int32_t *rp, const int32_t *ci, const uint8_t *w, const int32_t *dS,
               const int32_t *cand, int64_t count, int64_t *gain) {
#pragma omp parallel
    {
        int32_t *d = (int32_t *)malloc(sizeof(int32_t) * (size_t)n);
        or_hent *heap = (or_hent *)malloc(sizeof(or_hent) * (size_t)(rp[n] + 2));
#pragma omp for schedule(dynamic, 4)
        for (int64_t i = 0; i < count; ++i) {
            sssp_w(n, rp, ci, w, cand[i], d, heap);
            int64_t g = 0;
            for (int64_t u = 0; u < n; ++u) g += dS[u] - (d[u] < dS[u] ? d[u] : dS[u]);
            gain[i] = g;
        }
        free(d); free(heap);
    }
    return OR_OK;
}

/*
 * Pruned Dijkstra from u (Section 4.1 for SSSP): a node reached with a
 * distance that is not below its d_S is not entered, and nothing behind it
 * is.  Returns g(u,S) = sum over settled w of (dS[w] - d(u,w)); *edges and
 * *visited as in pruned_gain.  With `write`, dS[w] is lowered to d(u,w) for
 * every settled w (the d(S,.) update after a pick).  tent: n entries, all
 * -1 on entry and on return.
 */
static int64_t pruned_gain_w(int64_t n, const int32_t *rp, const int32_t *ci, const uint8_t *w,
                             int32_t *dS, int32_t u, int32_t *tent, int32_t *done, or_hent *heap,
                             int32_t *touched, int write, int64_t *edges, int64_t *visited) {
    (void)n;
    int64_t g = 0, e_cnt = 0, v_cnt = 0, len = 0, nt = 0;
    *edges = 0; *visited = 0;
    if (!(0 < dS[u])) return 0;
    tent[u] = 0; touched[nt++] = u;
    heap_push(heap, &len, 0, u);
    while (len > 0) {
        or_hent t = heap_pop(heap, &len);
        if (done[t.v] || tent[t.v] != t.d) continue;
        done[t.v] = 1;
        g += dS[t.v] - t.d;
        v_cnt += 1;
        e_cnt += rp[t.v + 1] - rp[t.v];
        for (int32_t e = rp[t.v]; e < rp[t.v + 1]; ++e) {
            int32_t y = ci[e];
            int64_t nd = t.d + w[e];
            if (done[y] || nd >= dS[y]) continue;  /* pruned: S is at least as close */
            if (tent[y] < 0 || nd < tent[y]) {
                if (tent[y] < 0) touched[nt++] = y;
                tent[y] = (int32_t)nd;
                heap_push(heap, &len, nd, y);
            }
        }
    }
    for (int64_t i = 0; i < nt; ++i) {
        int32_t y = touched[i];
        if (write && done[y]) dS[y] = tent[y];
        tent[y] = -1; done[y] = 0;
    }
    *edges = e_cnt; *visited = v_cnt;
    return g;
}

int or_pruned_stats_w(int64_t n, const int32_t *rp, const int32_t *ci, const uint8_t *w, const int32_t *dS,
                      const int32_t *cand, int64_t count, int64_t *gain, int64_t *visited, int64_t *edges) {
#pragma omp parallel
    {
        int32_t *tent = (int32_t *)malloc(sizeof(int32_t) * (size_t)n);
        int32_t *done = (int32_t *)calloc((size_t)n, sizeof(int32_t));
        int32_t *touched = (int32_t *)malloc(sizeof(int32_t) * (size_t)n);
        or_hent *heap = (or_hent *)malloc(sizeof(or_hent) * (size_t)(rp[n] + 2));
        for (int64_t i = 0; i < n; ++i) tent[i] = -1;
#pragma omp for schedule(dynamic, 16)
        for (int64_t i = 0; i < count; ++i) {
            int64_t e, v;
            gain[i] = pruned_gain_w(n, rp, ci, w, (int32_t *)dS, cand[i], tent, done, heap, touched, 0, &e, &v);
            if (visited) visited[i] = v;
            if (edges) edges[i] = e;
        }
        free(tent); free(done); free(touched); free(heap);
    }
    return OR_OK;
}

/*
 * Tier A on a weighted graph: the plain greedy of Section 3.2 with Dijkstra
 * for every SSSP, ties to the smallest id, the same invariants as or_greedy.
 */
int or_greedy_w(int64_t n, const int32_t *rp, const int32_t *ci, const uint8_t *w, int32_t k,
                int32_t *group, int64_t *Fout, int32_t directed) {
    if (k < 1 || k > n) return OR_EINVAL;
    int vrc = or_validate_w(n, rp, ci, w, directed);
    if (vrc != OR_OK) return vrc;
    int64_t *Fv = (int64_t *)malloc(sizeof(int64_t) * (size_t)n);
    int64_t *prev = (int64_t *)malloc(sizeof(int64_t) * (size_t)n);
    int32_t *dS = (int32_t *)malloc(sizeof(int32_t) * (size_t)n);
    int32_t *dsnew = (int32_t *)malloc(sizeof(int32_t) * (size_t)n);
    uint8_t *inS = (uint8_t *)calloc((size_t)n, 1);
    or_hent *heap = (or_hent *)malloc(sizeof(or_hent) * (size_t)(rp[n] + 2));
    int rc = or_farness_all_w(n, rp, ci, w, Fv);
    if (rc == OR_OK) {
        int32_t s = 0;
        for (int64_t v = 1; v < n; ++v)
            if (Fv[v] < Fv[s]) s = (int32_t)v;
        group[0] = s;
        inS[s] = 1;
        sssp_w(n, rp, ci, w, s, dS, heap);
        int64_t F = Fv[s];
        Fout[0] = F;
        for (int64_t v = 0; v < n; ++v) prev[v] = INT64_MAX;
        for (int32_t i = 1; i < k && rc == OR_OK; ++i) {
            int bad = 0;
#pragma omp parallel
            {
                int32_t *d = (int32_t *)malloc(sizeof(int32_t) * (size_t)n);
                or_hent *hp = (or_hent *)malloc(sizeof(or_hent) * (size_t)(rp[n] + 2));
#pragma omp for schedule(dynamic, 4)
                for (int64_t v = 0; v < n; ++v) {
                    if (inS[v]) { Fv[v] = INT64_MAX; continue; }
                    sssp_w(n, rp, ci, w, (int32_t)v, d, hp);
                    int64_t t = 0;
                    for (int64_t u = 0; u < n; ++u) t += (d[u] < dS[u] ? d[u] : dS[u]);
                    Fv[v] = t;
                }
                free(d); free(hp);
            }
            int32_t best = -1;
            for (int64_t v = 0; v < n; ++v) {
                if (inS[v]) continue;
                int64_t g = F - Fv[v];
                if (g > prev[v]) bad = 1;             /* supermodularity */
                if (g < dS[v] || dS[v] < 1) bad = 1;  /* v itself drops to 0 */
                prev[v] = g;
                if (best < 0 || Fv[v] < Fv[best]) best = (int32_t)v;
            }
            sssp_w(n, rp, ci, w, best, dsnew, heap);
            int64_t sum = 0;
            for (int64_t u = 0; u < n; ++u) {
                int32_t m = dsnew[u] < dS[u] ? dsnew[u] : dS[u];
                if (m > dS[u]) bad = 1;
                dS[u] = m;
                sum += m;
            }
            if (sum != Fv[best] || !(Fv[best] < F)) bad = 1;
            F = Fv[best];
            group[i] = best;
            inS[best] = 1;
            Fout[i] = F;
            if (bad) rc = OR_EINVARIANT;
        }
    }
    free(Fv); free(prev); free(dS); free(dsnew); free(inS); free(heap);
    return rc;
}

/*
 * Tier B on a weighted graph: the first node by the closeness search in
 * decreasing degree order, each Dijkstra stopped, when the next node to
 * settle is at distance D, once sum + D * (unsettled) cannot beat the best
 * (every unsettled node is at D or more); then
 * the lazy loop of or_greedypp with pruned Dijkstra gains and the pruned
 * update.  Same batch schedule (block, growth) and evaluation counts.
 */
int or_greedypp_w(int64_t n, const int32_t *rp, const int32_t *ci, const uint8_t *w, int32_t k,
                  int32_t block, int32_t growth, int32_t *group, int64_t *Fout, int64_t *evals,
                  int64_t *edges, int32_t directed) {
    if (k < 1 || k > n || block < 1 || growth < 1 || growth > 8) return OR_EINVAL;
    int vrc = or_validate_w(n, rp, ci, w, directed);
    if (vrc != OR_OK) return vrc;
    int64_t maxb = growth > 1 ? 16 * (int64_t)block : block;
    if (maxb > n) maxb = n;
    int nthr = 1;
#ifdef _OPENMP
    nthr = omp_get_max_threads();
#endif
    int32_t **tent = (int32_t **)malloc(sizeof(void *) * (size_t)nthr);
    int32_t **done = (int32_t **)malloc(sizeof(void *) * (size_t)nthr);
    int32_t **tch = (int32_t **)malloc(sizeof(void *) * (size_t)nthr);
    or_hent **heaps = (or_hent **)malloc(sizeof(void *) * (size_t)nthr);
    for (int t = 0; t < nthr; ++t) {
        tent[t] = (int32_t *)malloc(sizeof(int32_t) * (size_t)n);
        for (int64_t i = 0; i < n; ++i) tent[t][i] = -1;
        done[t] = (int32_t *)calloc((size_t)n, sizeof(int32_t));
        tch[t] = (int32_t *)malloc(sizeof(int32_t) * (size_t)n);
        heaps[t] = (or_hent *)malloc(sizeof(or_hent) * (size_t)(rp[n] + 2));
    }
    int32_t *order = (int32_t *)malloc(sizeof(int32_t) * (size_t)n);
    int32_t *dS = (int32_t *)malloc(sizeof(int32_t) * (size_t)n);
    int64_t *ub = (int64_t *)malloc(sizeof(int64_t) * (size_t)n);
    int32_t *batch = (int32_t *)malloc(sizeof(int32_t) * (size_t)maxb);
    int64_t *bg = (int64_t *)malloc(sizeof(int64_t) * (size_t)maxb);
    int64_t *be = (int64_t *)malloc(sizeof(int64_t) * (size_t)maxb);
    int rc = OR_OK;
    {
        /* decreasing degree, ties ascending id (stable counting sort) */
        int32_t maxdeg = 0;
        for (int64_t v = 0; v < n; ++v) if (rp[v + 1] - rp[v] > maxdeg) maxdeg = rp[v + 1] - rp[v];
        int64_t *cnt = (int64_t *)calloc((size_t)maxdeg + 2, sizeof(int64_t));
        for (int64_t v = 0; v < n; ++v) cnt[maxdeg - (rp[v + 1] - rp[v]) + 1]++;
        for (int32_t x = 0; x <= maxdeg; ++x) cnt[x + 1] += cnt[x];
        for (int64_t v = 0; v < n; ++v) order[cnt[maxdeg - (rp[v + 1] - rp[v])]++] = (int32_t)v;
        free(cnt);
    }
    /* first node: Dijkstra with the distance-group cut, in degree order */
    int64_t bestF = -1;
    int32_t bestId = -1;
    for (int64_t i = 0; i < n; ++i) {
        int32_t v = order[i];
        int32_t *tv = tent[0], *dn = done[0], *tc = tch[0];
        or_hent *hp = heaps[0];
        int64_t len = 0, nt = 0, settled = 0, sum = 0, cur = -1;
        int cut = 0;
        tv[v] = 0; tc[nt++] = v;
        heap_push(hp, &len, 0, v);
        while (len > 0) {
            or_hent t = heap_pop(hp, &len);
            if (dn[t.v] || tv[t.v] != t.d) continue;
            if (t.d > cur) {
                /* every node closer than t.d is settled; Dijkstra pops in
                 * nondecreasing order, so every other node is at t.d or more */
                if (cur >= 0 && bestId >= 0) {
                    int64_t lb = sum + t.d * (n - settled);
                    if (lb > bestF || (lb == bestF && v > bestId)) { cut = 1; break; }
                }
                cur = t.d;
            }
            dn[t.v] = 1; settled += 1; sum += t.d;
            for (int32_t e = rp[t.v]; e < rp[t.v + 1]; ++e) {
                int32_t y = ci[e];
                int64_t nd = t.d + w[e];
                if (dn[y]) continue;
                if (tv[y] < 0 || nd < tv[y]) {
                    if (tv[y] < 0) tc[nt++] = y;
                    tv[y] = (int32_t)nd;
                    heap_push(hp, &len, nd, y);
                }
            }
        }
        for (int64_t j = 0; j < nt; ++j) { tv[tc[j]] = -1; dn[tc[j]] = 0; }
        if (cut) continue;
        if (settled != n) { rc = OR_EDISCONNECTED; goto done; }
        if (bestId < 0 || sum < bestF || (sum == bestF && v < bestId)) { bestF = sum; bestId = v; }
    }
    group[0] = bestId;
    Fout[0] = bestF;
    sssp_w(n, rp, ci, w, bestId, dS, heaps[0]);
    for (int64_t v = 0; v < n; ++v) ub[v] = INT64_MAX;
    if (evals) evals[0] = 0;
    if (edges) edges[0] = 0;
    {
        int64_t F = bestF;
        for (int32_t r = 1; r < k; ++r) {
            int64_t bgain = -1;
            int32_t bid = -1;
            int64_t pos = 0, nev = 0, ned = 0;
            int64_t cur = block < maxb ? block : maxb;
            for (;;) {
                int32_t nb = 0;
                while (pos < n && nb < cur) {
                    int32_t u = (int32_t)pos++;
                    if (dS[u] == 0) continue;
                    if (bid >= 0 && (ub[u] < bgain || (ub[u] == bgain && u > bid))) continue;
                    batch[nb++] = u;
                }
                if (nb == 0) break;
#pragma omp parallel for schedule(dynamic, 1) if (nb > 1)
                for (int32_t j = 0; j < nb; ++j) {
                    int t = 0;
#ifdef _OPENMP
                    t = omp_get_thread_num();
#endif
                    int64_t vis;
                    bg[j] = pruned_gain_w(n, rp, ci, w, dS, batch[j], tent[t], done[t], heaps[t], tch[t], 0,
                                          &be[j], &vis);
                }
                for (int32_t j = 0; j < nb; ++j) {
                    int32_t u = batch[j];
                    ub[u] = bg[j];
                    ned += be[j];
                    if (bid < 0 || bg[j] > bgain || (bg[j] == bgain && u < bid)) { bgain = bg[j]; bid = u; }
                }
                nev += nb;
                if (r >= 2 && cur * growth <= maxb) cur *= growth;
                else if (r >= 2) cur = maxb;
            }
            if (evals) evals[r] = nev;
            if (edges) edges[r] = ned;
            group[r] = bid;
            {
                int64_t e, v;
                pruned_gain_w(n, rp, ci, w, dS, bid, tent[0], done[0], heaps[0], tch[0], 1, &e, &v);
            }
            F -= bgain;
            Fout[r] = F;
        }
    }
done:
    for (int t = 0; t < nthr; ++t) { free(tent[t]); free(done[t]); free(tch[t]); free(heaps[t]); }
    free(tent); free(done); free(tch); free(heaps);
    free(order); free(dS); free(ub); free(batch); free(bg); free(be);
    return rc;
}
