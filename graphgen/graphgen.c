/*
 * Seeded synthetic graph generators and a CSR builder.
 *
 * This file produces inputs only.  It holds none of the group-closeness
 * arithmetic (no distances, no farness, no gains): both the CPU oracle and
 * the GPU library are fed from what it writes.
 *
 * Random numbers come from SplitMix64 (Steele, Lea and Flood, "Fast
 * splittable pseudorandom number generators", OOPSLA 2014), used in its
 * counter form: draw i of a stream keyed by `key` is mix(key + (i+1)*G) with
 * G = 0x9E3779B97F4A7C15.  The output is therefore identical on every
 * platform and numpy version.
 *
 * Build: gcc -O2 -fopenmp -shared -fPIC graphgen.c -o libgraphgen.so
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define GOLDEN 0x9E3779B97F4A7C15ULL

static inline uint64_t sm_mix(uint64_t z) {
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ULL;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBULL;
    return z ^ (z >> 31);
}

/* draw i (0-based) of the stream keyed by `key` */
static inline uint64_t sm_at(uint64_t key, uint64_t i) { return sm_mix(key + (i + 1) * GOLDEN); }

/* uniform integer in [0, m) by the multiply-high map (Lemire) */
static inline uint64_t sm_below(uint64_t x, uint64_t m) {
    return (uint64_t)(((unsigned __int128)x * m) >> 64);
}

/* uniform double in [0, 1) from the top 53 bits */
static inline double sm_unit(uint64_t x) { return (double)(x >> 11) * (1.0 / 9007199254740992.0); }

uint64_t gg_splitmix_at(uint64_t key, uint64_t i) { return sm_at(key, i); }

/*
 * Barabasi-Albert preferential attachment.
 * Nodes 0..m form the clique K_{m+1}.  Each later node t = m+1 .. n-1 picks m
 * distinct earlier nodes with probability proportional to their degree, by
 * drawing uniform positions in the endpoint list (every edge contributes both
 * endpoints) as it stood before t arrived, rejecting repeats.
 * Writes the undirected edge list (src[e], dst[e]) and returns the number of
 * edges, C(m+1,2) + m*(n-m-1); returns -1 on bad arguments.
 */
int64_t gg_ba(int64_t n, int32_t m, uint64_t seed, int32_t *src, int32_t *dst) {
    if (m < 1 || n < m + 1) return -1;
    int64_t ne = 0;
    for (int32_t i = 0; i <= m; ++i)
        for (int32_t j = i + 1; j <= m; ++j) { src[ne] = i; dst[ne] = j; ++ne; }
    /* endpoint list position p: edge p/2, endpoint p%2 */
    int32_t *chosen = (int32_t *)malloc(sizeof(int32_t) * (size_t)m);
    uint64_t draw = 0;
    for (int64_t t = m + 1; t < n; ++t) {
        int64_t len = 2 * ne;
        int32_t got = 0;
        while (got < m) {
            uint64_t p = sm_below(sm_at(seed, draw++), (uint64_t)len);
            int32_t v = (p & 1) ? dst[p >> 1] : src[p >> 1];
            int dup = 0;
            for (int32_t q = 0; q < got; ++q) dup |= (chosen[q] == v);
            if (!dup) chosen[got++] = v;
        }
        for (int32_t q = 0; q < m; ++q) { src[ne] = (int32_t)t; dst[ne] = chosen[q]; ++ne; }
    }
    free(chosen);
    return ne;
}

/*
 * R-MAT (Chakrabarti, Zhan, Faloutsos 2004) with quadrant probabilities
 * (a, b, c, 1-a-b-c) and no per-level noise, followed by a seeded random
 * relabelling of the 2^scale vertex ids (Fisher-Yates), as in Graph500.
 * Edge e at level l uses draw e*scale + l of the stream keyed by
 * sm_at(seed, 0); the permutation uses the stream keyed by sm_at(seed, 1).
 * Writes `m` directed edge draws (self-loops and repeats included; the CSR
 * builder removes them).
 */
int gg_rmat(int32_t scale, int64_t m, double a, double b, double c, uint64_t seed,
            int32_t *src, int32_t *dst) {
    if (scale < 1 || scale > 30 || m < 0) return -1;
    const uint64_t k_edge = sm_at(seed, 0), k_perm = sm_at(seed, 1);
    const int64_t nv = (int64_t)1 << scale;
    const double ab = a + b, abc = a + b + c;
#pragma omp parallel for schedule(static)
    for (int64_t e = 0; e < m; ++e) {
        uint32_t u = 0, v = 0;
        for (int32_t l = 0; l < scale; ++l) {
            double r = sm_unit(sm_at(k_edge, (uint64_t)e * (uint64_t)scale + (uint64_t)l));
            uint32_t bu, bv;
            if (r < a) { bu = 0; bv = 0; }
            else if (r < ab) { bu = 0; bv = 1; }
            else if (r < abc) { bu = 1; bv = 0; }
            else { bu = 1; bv = 1; }
            u = (u << 1) | bu;
            v = (v << 1) | bv;
        }
        src[e] = (int32_t)u;
        dst[e] = (int32_t)v;
    }
    int32_t *perm = (int32_t *)malloc(sizeof(int32_t) * (size_t)nv);
    for (int64_t i = 0; i < nv; ++i) perm[i] = (int32_t)i;
    for (int64_t i = nv - 1; i > 0; --i) {
        int64_t j = (int64_t)sm_below(sm_at(k_perm, (uint64_t)(nv - 1 - i)), (uint64_t)(i + 1));
        int32_t t = perm[i]; perm[i] = perm[j]; perm[j] = t;
    }
#pragma omp parallel for schedule(static)
    for (int64_t e = 0; e < m; ++e) { src[e] = perm[src[e]]; dst[e] = perm[dst[e]]; }
    free(perm);
    return 0;
}

/*
 * Perturbed 2D grid: rows x cols lattice in row-major ids; `drop` lattice
 * edges removed uniformly without replacement (partial Fisher-Yates over the
 * edge indices, stream sm_at(seed,0)), then `shortcuts` extra edges between
 * uniform node pairs that are neither equal nor already adjacent (stream
 * sm_at(seed,1), rejection).  Writes the kept lattice edges followed by the
 * shortcuts and returns the total count, or -1.
 * Capacity needed: 2*rows*cols edges.
 */
static int cmp_u64(const void *x, const void *y) {
    uint64_t a = *(const uint64_t *)x, b = *(const uint64_t *)y;
    return (a > b) - (a < b);
}

int64_t gg_grid(int32_t rows, int32_t cols, int64_t drop, int64_t shortcuts, uint64_t seed,
                int32_t *src, int32_t *dst) {
    const int64_t nv = (int64_t)rows * cols;
    const int64_t nh = (int64_t)rows * (cols - 1), nl = nh + (int64_t)(rows - 1) * cols;
    if (rows < 1 || cols < 1 || drop < 0 || drop > nl || shortcuts < 0) return -1;
    int64_t *idx = (int64_t *)malloc(sizeof(int64_t) * (size_t)(nl > 0 ? nl : 1));
    for (int64_t i = 0; i < nl; ++i) idx[i] = i;
    const uint64_t k_drop = sm_at(seed, 0), k_short = sm_at(seed, 1);
    /* the first `drop` slots after the partial shuffle are the dropped edges */
    for (int64_t i = 0; i < drop; ++i) {
        int64_t j = i + (int64_t)sm_below(sm_at(k_drop, (uint64_t)i), (uint64_t)(nl - i));
        int64_t t = idx[i]; idx[i] = idx[j]; idx[j] = t;
    }
    uint8_t *dead = (uint8_t *)calloc((size_t)(nl > 0 ? nl : 1), 1);
    for (int64_t i = 0; i < drop; ++i) dead[idx[i]] = 1;
    int64_t ne = 0;
    uint64_t *keys = (uint64_t *)malloc(sizeof(uint64_t) * (size_t)(nl + shortcuts + 1));
    for (int64_t e = 0; e < nl; ++e) {
        if (dead[e]) continue;
        int64_t u, v;
        if (e < nh) { int64_t r = e / (cols - 1), c = e % (cols - 1); u = r * cols + c; v = u + 1; }
        else { int64_t f = e - nh; u = f; v = f + cols; }
        src[ne] = (int32_t)u; dst[ne] = (int32_t)v;
        keys[ne] = ((uint64_t)u << 32) | (uint64_t)v;
        ++ne;
    }
    qsort(keys, (size_t)ne, sizeof(uint64_t), cmp_u64);
    int64_t nk = ne;
    uint64_t draw = 0;
    int64_t added = 0;
    while (added < shortcuts && nv > 1) {
        int64_t u = (int64_t)sm_below(sm_at(k_short, draw++), (uint64_t)nv);
        int64_t v = (int64_t)sm_below(sm_at(k_short, draw++), (uint64_t)nv);
        if (u == v) continue;
        int64_t lo = u < v ? u : v, hi = u < v ? v : u;
        uint64_t key = ((uint64_t)lo << 32) | (uint64_t)hi;
        /* adjacency test: binary search over the sorted lattice keys, linear over new ones */
        int64_t L = 0, R = nk;
        while (L < R) { int64_t M = (L + R) >> 1; if (keys[M] < key) L = M + 1; else R = M; }
        int present = (L < nk && keys[L] == key);
        for (int64_t q = nk; q < nk + added && !present; ++q) present = (keys[q] == key);
        if (present) continue;
        keys[nk + added] = key;
        src[ne] = (int32_t)lo; dst[ne] = (int32_t)hi; ++ne;
        ++added;
    }
    free(keys); free(dead); free(idx);
    return ne;
}

/*
 * CSR builder: symmetrise the edge list, drop self-loops and duplicates,
 * optionally keep only the largest connected component (ties go to the
 * component that holds the smallest vertex id), relabel the kept vertices in
 * ascending order of their old ids, and write rows sorted ascending.
 *   nv, ne, src, dst : input vertex count and edge list
 *   row_ptr          : capacity nv+1
 *   col_idx          : capacity 2*ne
 *   old_id           : capacity nv; old_id[new] = old vertex id
 *   out_n, out_nnz   : sizes of the result
 * Returns 0, or -1 on bad input (id out of range).
 */
int gg_build_csr(int64_t nv, int64_t ne, const int32_t *src, const int32_t *dst, int32_t keep_lcc,
                 int64_t *row_ptr, int32_t *col_idx, int32_t *old_id, int64_t *out_n,
                 int64_t *out_nnz) {
    for (int64_t e = 0; e < ne; ++e)
        if (src[e] < 0 || dst[e] < 0 || src[e] >= nv || dst[e] >= nv) return -1;
    int64_t *deg = (int64_t *)calloc((size_t)nv + 1, sizeof(int64_t));
    for (int64_t e = 0; e < ne; ++e)
        if (src[e] != dst[e]) { deg[src[e] + 1]++; deg[dst[e] + 1]++; }
    for (int64_t v = 0; v < nv; ++v) deg[v + 1] += deg[v];
    int64_t *fill = (int64_t *)malloc(sizeof(int64_t) * (size_t)(nv + 1));
    memcpy(fill, deg, sizeof(int64_t) * (size_t)(nv + 1));
    int32_t *adj = (int32_t *)malloc(sizeof(int32_t) * (size_t)(deg[nv] > 0 ? deg[nv] : 1));
    for (int64_t e = 0; e < ne; ++e) {
        int32_t u = src[e], v = dst[e];
        if (u == v) continue;
        adj[fill[u]++] = v;
        adj[fill[v]++] = u;
    }
    /* sort and dedupe each row in place; cnt[v] = distinct neighbours */
    int64_t *cnt = (int64_t *)malloc(sizeof(int64_t) * (size_t)(nv > 0 ? nv : 1));
#pragma omp parallel for schedule(dynamic, 4096)
    for (int64_t v = 0; v < nv; ++v) {
        int32_t *row = adj + deg[v];
        int64_t len = deg[v + 1] - deg[v];
        /* insertion sort for short rows, radix-free qsort for long ones */
        if (len < 32) {
            for (int64_t i = 1; i < len; ++i) {
                int32_t x = row[i]; int64_t j = i - 1;
                while (j >= 0 && row[j] > x) { row[j + 1] = row[j]; --j; }
                row[j + 1] = x;
            }
        } else {
            /* heap sort: no recursion, no extra memory */
            for (int64_t s = len / 2 - 1; s >= 0; --s) {
                int64_t r = s;
                for (;;) {
                    int64_t ch = 2 * r + 1; if (ch >= len) break;
                    if (ch + 1 < len && row[ch + 1] > row[ch]) ++ch;
                    if (row[r] >= row[ch]) break;
                    int32_t t = row[r]; row[r] = row[ch]; row[ch] = t; r = ch;
                }
            }
            for (int64_t end = len - 1; end > 0; --end) {
                int32_t t = row[0]; row[0] = row[end]; row[end] = t;
                int64_t r = 0;
                for (;;) {
                    int64_t ch = 2 * r + 1; if (ch >= end) break;
                    if (ch + 1 < end && row[ch + 1] > row[ch]) ++ch;
                    if (row[r] >= row[ch]) break;
                    int32_t u = row[r]; row[r] = row[ch]; row[ch] = u; r = ch;
                }
            }
        }
        int64_t w = 0;
        for (int64_t i = 0; i < len; ++i)
            if (w == 0 || row[i] != row[w - 1]) row[w++] = row[i];
        cnt[v] = w;
    }
    /* components by iterative BFS over the deduplicated rows */
    int32_t *comp = (int32_t *)malloc(sizeof(int32_t) * (size_t)(nv > 0 ? nv : 1));
    int32_t *queue = (int32_t *)malloc(sizeof(int32_t) * (size_t)(nv > 0 ? nv : 1));
    for (int64_t v = 0; v < nv; ++v) comp[v] = -1;
    int32_t best_c = -1; int64_t best_size = -1, ncomp = 0;
    for (int64_t s = 0; s < nv; ++s) {
        if (comp[s] >= 0) continue;
        int64_t h = 0, t = 0;
        queue[t++] = (int32_t)s; comp[s] = (int32_t)ncomp;
        while (h < t) {
            int32_t x = queue[h++];
            for (int64_t i = 0; i < cnt[x]; ++i) {
                int32_t y = adj[deg[x] + i];
                if (comp[y] < 0) { comp[y] = (int32_t)ncomp; queue[t++] = y; }
            }
        }
        /* components are discovered in order of their smallest id: strict > keeps the first */
        if (t > best_size) { best_size = t; best_c = (int32_t)ncomp; }
        ++ncomp;
    }
    int32_t *newid = queue; /* reuse */
    int64_t nn = 0;
    for (int64_t v = 0; v < nv; ++v) {
        if (!keep_lcc || comp[v] == best_c) { newid[v] = (int32_t)nn; old_id[nn] = (int32_t)v; ++nn; }
        else newid[v] = -1;
    }
    int64_t nnz = 0;
    row_ptr[0] = 0;
    for (int64_t i = 0; i < nn; ++i) {
        int32_t v = old_id[i];
        for (int64_t q = 0; q < cnt[v]; ++q) col_idx[nnz++] = newid[adj[deg[v] + q]];
        row_ptr[i + 1] = nnz;
    }
    *out_n = nn;
    *out_nnz = nnz;
    free(comp); free(queue); free(cnt); free(adj); free(fill); free(deg);
    return 0;
}

/*
 * Directed CSR: the edge list read as arcs src[e] -> dst[e] (not
 * symmetrised), self-loops and repeated arcs dropped, rows (out-neighbours)
 * sorted ascending.  With keep_scc the largest strongly connected component
 * is kept (ties: the component holding the smallest id) and relabelled in
 * ascending order of the old ids.  Strong components by Kosaraju's two
 * passes (finish order of a depth-first search on the arcs, then searches on
 * the reversed arcs in reverse finish order), both iterative.
 * Capacities: row_ptr nv+1, col_idx ne, old_id nv.  Returns 0 or -1.
 */
int gg_build_csr_directed(int64_t nv, int64_t ne, const int32_t *src, const int32_t *dst,
                          int32_t keep_scc, int64_t *row_ptr, int32_t *col_idx, int32_t *old_id,
                          int64_t *out_n, int64_t *out_nnz) {
    for (int64_t e = 0; e < ne; ++e)
        if (src[e] < 0 || dst[e] < 0 || src[e] >= nv || dst[e] >= nv) return -1;
    int64_t *deg = (int64_t *)calloc((size_t)nv + 1, sizeof(int64_t));
    for (int64_t e = 0; e < ne; ++e)
        if (src[e] != dst[e]) deg[src[e] + 1]++;
    for (int64_t v = 0; v < nv; ++v) deg[v + 1] += deg[v];
    int64_t *fill = (int64_t *)malloc(sizeof(int64_t) * (size_t)(nv + 1));
    memcpy(fill, deg, sizeof(int64_t) * (size_t)(nv + 1));
    int32_t *adj = (int32_t *)malloc(sizeof(int32_t) * (size_t)(deg[nv] > 0 ? deg[nv] : 1));
    for (int64_t e = 0; e < ne; ++e)
        if (src[e] != dst[e]) adj[fill[src[e]]++] = dst[e];
    int64_t *cnt = (int64_t *)malloc(sizeof(int64_t) * (size_t)(nv > 0 ? nv : 1));
    for (int64_t v = 0; v < nv; ++v) {
        int32_t *row = adj + deg[v];
        int64_t len = deg[v + 1] - deg[v];
        for (int64_t i = 1; i < len; ++i) { /* insertion sort (rows of generated digraphs are short) */
            int32_t x = row[i]; int64_t j = i - 1;
            while (j >= 0 && row[j] > x) { row[j + 1] = row[j]; --j; }
            row[j + 1] = x;
        }
        int64_t w = 0;
        for (int64_t i = 0; i < len; ++i)
            if (w == 0 || row[i] != row[w - 1]) row[w++] = row[i];
        cnt[v] = w;
    }
    /* reversed arcs */
    int64_t *rdeg = (int64_t *)calloc((size_t)nv + 1, sizeof(int64_t));
    for (int64_t v = 0; v < nv; ++v)
        for (int64_t i = 0; i < cnt[v]; ++i) rdeg[adj[deg[v] + i] + 1]++;
    for (int64_t v = 0; v < nv; ++v) rdeg[v + 1] += rdeg[v];
    int64_t *rfill = (int64_t *)malloc(sizeof(int64_t) * (size_t)(nv + 1));
    memcpy(rfill, rdeg, sizeof(int64_t) * (size_t)(nv + 1));
    int32_t *radj = (int32_t *)malloc(sizeof(int32_t) * (size_t)(rdeg[nv] > 0 ? rdeg[nv] : 1));
    for (int64_t v = 0; v < nv; ++v)
        for (int64_t i = 0; i < cnt[v]; ++i) radj[rfill[adj[deg[v] + i]]++] = (int32_t)v;
    /* pass 1: finish order */
    int32_t *order = (int32_t *)malloc(sizeof(int32_t) * (size_t)(nv > 0 ? nv : 1));
    int32_t *stk = (int32_t *)malloc(sizeof(int32_t) * (size_t)(nv > 0 ? nv : 1));
    int64_t *pos = (int64_t *)malloc(sizeof(int64_t) * (size_t)(nv > 0 ? nv : 1));
    uint8_t *seen = (uint8_t *)calloc((size_t)(nv > 0 ? nv : 1), 1);
    int64_t nord = 0;
    for (int64_t s = 0; s < nv; ++s) {
        if (seen[s]) continue;
        int64_t top = 0;
        stk[top++] = (int32_t)s; pos[s] = 0; seen[s] = 1;
        while (top > 0) {
            int32_t x = stk[top - 1];
            if (pos[x] < cnt[x]) {
                int32_t y = adj[deg[x] + pos[x]++];
                if (!seen[y]) { seen[y] = 1; pos[y] = 0; stk[top++] = y; }
            } else {
                order[nord++] = x;
                --top;
            }
        }
    }
    /* pass 2: components on the reversed arcs, in reverse finish order */
    int32_t *comp = (int32_t *)malloc(sizeof(int32_t) * (size_t)(nv > 0 ? nv : 1));
    for (int64_t v = 0; v < nv; ++v) comp[v] = -1;
    int64_t ncomp = 0, best_size = -1;
    int32_t best_c = -1, best_min = INT32_MAX;
    for (int64_t i = nord - 1; i >= 0; --i) {
        int32_t s = order[i];
        if (comp[s] >= 0) continue;
        int64_t h = 0, t = 0;
        int32_t mn = s;
        stk[t++] = s; comp[s] = (int32_t)ncomp;
        while (h < t) {
            int32_t x = stk[h++];
            if (x < mn) mn = x;
            for (int64_t q = rdeg[x]; q < rdeg[x + 1]; ++q) {
                int32_t y = radj[q];
                if (comp[y] < 0) { comp[y] = (int32_t)ncomp; stk[t++] = y; }
            }
        }
        if (t > best_size || (t == best_size && mn < best_min)) { best_size = t; best_c = (int32_t)ncomp; best_min = mn; }
        ++ncomp;
    }
    int32_t *newid = stk; /* reuse */
    int64_t nn = 0;
    for (int64_t v = 0; v < nv; ++v) {
        if (!keep_scc || comp[v] == best_c) { newid[v] = (int32_t)nn; old_id[nn] = (int32_t)v; ++nn; }
        else newid[v] = -1;
    }
    int64_t nnz = 0;
    row_ptr[0] = 0;
    for (int64_t i = 0; i < nn; ++i) {
        int32_t v = old_id[i];
        for (int64_t q = 0; q < cnt[v]; ++q) {
            int32_t y = newid[adj[deg[v] + q]];
            if (y >= 0) col_idx[nnz++] = y; /* ids ascend with old ids: rows stay sorted */
        }
        row_ptr[i + 1] = nnz;
    }
    *out_n = nn;
    *out_nnz = nnz;
    free(comp); free(seen); free(pos); free(stk); free(order); free(radj); free(rfill); free(rdeg);
    free(cnt); free(adj); free(fill); free(deg);
    return 0;
}

/* Integer arc weights in [1, wmax] from SplitMix64 keyed by the (unordered,
 * unless directed) endpoint pair, so both rows of an undirected edge carry
 * the same weight. */
int gg_edge_weights(int64_t n, const int32_t *rp, const int32_t *ci, int32_t wmax, uint64_t seed,
                    int32_t directed, uint8_t *w) {
    if (wmax < 1 || wmax > 255) return -1;
#pragma omp parallel for schedule(static)
    for (int64_t u = 0; u < n; ++u)
        for (int32_t e = rp[u]; e < rp[u + 1]; ++e) {
            int64_t a = u, b = ci[e];
            if (!directed && b < a) { int64_t t = a; a = b; b = t; }
            w[e] = (uint8_t)(1 + sm_at(seed, (uint64_t)a * (uint64_t)n + (uint64_t)b) % (uint64_t)wmax);
        }
    return 0;
}
