/*
 * CPU oracle for exact k-clique counting and low out-degree orientation.
 *
 * TEST INFRASTRUCTURE ONLY.  Only the test suite, the smoke check and the CPU
 * baseline leg of the benchmark may load this library.  It shares no code, header,
 * table or helper with the HIP library; the two agree only because both follow the
 * paper (Shi, Dhulipala, Shun, "Parallel Clique Counting and Peeling Algorithms").
 *
 * Contents
 *   orc_validate            simple undirected graph check (Sec. 2, graph notation)
 *   orc_orient              Barenboim-Elkin style peel with the average-degree threshold
 *                           (Sec. 3.1 and Alg. 4 of the appendix), ranks, directed CSR
 *                           (Sec. 3.1, last paragraph)
 *   orc_orient_method       the same with the degree, Goodrich-Pszona (Alg. 3) or k-core
 *                           ordering
 *   orc_count               Chiba-Nishizeki recursion with level labels (Sec. 3.4; the
 *                           count is the plain definition: every k-vertex subset whose
 *                           pairs are all adjacent, counted once from its first vertex)
 *   orc_brute               brute force over all k-subsets, n <= 64
 *   orc_degeneracy          exact degeneracy (k-core decomposition by bin sort, Batagelj-Zaversnik 2003)
 *   orc_local_cliques       c_j(v) = number of j-cliques inside G[N+(v)] of a directed
 *                           graph (the per-root subproblem of Alg. 1)
 *   orc_local_cliques_roots the same for a list of roots (sampled checks of large graphs)
 *   orc_sparsify            colorful sparsification: the edges whose endpoints share a
 *                           colour (Sec. 3.3, appendix sampling theorem)
 *   orc_vertex_cliques      the number of k-cliques containing each listed vertex of an
 *                           undirected graph, from its own neighbourhood (arb-count-v's
 *                           per-vertex count, Sec. 3.2, by definition)
 *
 * Arithmetic: counts are uint64 modulo 2^64 (the paper fixes no width; its largest
 * printed count is below 2^63).  A 128-bit shadow of the total reports overflow.
 * Floating point is used once, for the peel threshold, in IEEE double with no
 * contraction (build with -ffp-contract=off).
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#include <math.h>
#ifdef _OPENMP
#include <omp.h>
#endif

typedef unsigned __int128 u128;

/* ------------------------------------------------------------------ validate */

/* 0 ok, 1 bad offsets, 2 index out of range, 3 self-loop, 4 row not strictly
 * ascending (unsorted or duplicate), 5 asymmetric. */
int orc_validate(int64_t n, const int64_t *off, const int32_t *idx)
{
    if (n < 0 || off[0] != 0) return 1;
    for (int64_t v = 0; v < n; v++)
        if (off[v + 1] < off[v]) return 1;
    for (int64_t v = 0; v < n; v++) {
        for (int64_t e = off[v]; e < off[v + 1]; e++) {
            int64_t u = idx[e];
            if (u < 0 || u >= n) return 2;
            if (u == v) return 3;
            if (e > off[v] && idx[e - 1] >= idx[e]) return 4;
        }
    }
    for (int64_t v = 0; v < n; v++) {
        for (int64_t e = off[v]; e < off[v + 1]; e++) {
            int64_t u = idx[e];
            /* binary search v in N(u) */
            int64_t lo = off[u], hi = off[u + 1];
            while (lo < hi) {
                int64_t mid = lo + (hi - lo) / 2;
                if (idx[mid] < v) lo = mid + 1; else hi = mid;
            }
            if (lo >= off[u + 1] || idx[lo] != v) return 5;
        }
    }
    return 0;
}

/* ------------------------------------------------------------------ orientation */

static const int32_t *g_round_key, *g_dap_key;

static int cmp_rank_key(const void *a, const void *b)
{
    int32_t x = *(const int32_t *)a, y = *(const int32_t *)b;
    if (g_round_key[x] != g_round_key[y]) return g_round_key[x] < g_round_key[y] ? -1 : 1;
    if (g_dap_key[x] != g_dap_key[y]) return g_dap_key[x] < g_dap_key[y] ? -1 : 1;
    return x < y ? -1 : (x > y);
}

static int cmp_i32(const void *a, const void *b)
{
    int32_t x = *(const int32_t *)a, y = *(const int32_t *)b;
    return x < y ? -1 : (x > y);
}

/*
 * Peel in rounds until no vertex is left.  In round r, over the vertices still
 * present: S = sum of their current degrees, c = their number,
 *     T = floor(((2 + eps) * S) / c)          (IEEE double, in this order)
 * and every present vertex with degree <= T is removed; its round is r and its
 * degree at removal is its degree at the start of the round.  After the removal,
 * each removed vertex lowers the degree of each neighbour that is still present.
 * Vertices removed earlier come earlier in the ordering; inside a round the order is
 * by degree at removal, then by id.  rank[v] is v's position.  The directed graph
 * keeps u -> w iff rank(u) < rank(w) and is written in rank space with every row
 * sorted ascending: ooff[rank(u)] .. holds rank(w).
 *
 * thr_out (nullable, max_rounds entries) receives T per round.  Returns the number of
 * rounds, or -1 if max_rounds is exceeded.
 */
/* present vertices sorted by (degree, id) (Goodrich-Pszona rounds) */
static const int32_t *g_deg_key;
static int cmp_deg_id(const void *a, const void *b)
{
    int32_t x = *(const int32_t *)a, y = *(const int32_t *)b;
    if (g_deg_key[x] != g_deg_key[y]) return g_deg_key[x] < g_deg_key[y] ? -1 : 1;
    return x < y ? -1 : (x > y);
}

/*
 * The same with another rule for the vertices removed in round r (method):
 *   0  degree <= floor(((2 + eps) * S) / c), as above;
 *   1  degree ordering: every vertex in round 0 (the rank is by degree, then id);
 *   2  Goodrich-Pszona (Alg. 3): the ceil((eps * c) / (2 + eps)) present vertices of
 *      lowest (degree, id), at least one;
 *   3  k-core ordering: degree <= T_r, T_r = max(T_{r-1}, least present degree), T_{-1} = 0.
 * thr_out receives T per round for methods 0 and 3.
 */
int orc_orient_method(int64_t n, const int64_t *off, const int32_t *idx, int method, double eps,
                      int32_t *round_out, int32_t *dap_out, int32_t *rank_out,
                      int64_t *ooff_out, int32_t *oidx_out, int64_t *thr_out, int max_rounds)
{
    int32_t *deg = (int32_t *)malloc(sizeof(int32_t) * (n + 1));
    uint8_t *present = (uint8_t *)malloc(n + 1);
    int32_t *peeled = (int32_t *)malloc(sizeof(int32_t) * (n + 1));
    int32_t *inv = (int32_t *)malloc(sizeof(int32_t) * (n + 1));
    int64_t left = n;
    int r = 0;
    int64_t Tk = 0;                     /* k-core: running threshold */
    for (int64_t v = 0; v < n; v++) {
        deg[v] = (int32_t)(off[v + 1] - off[v]);
        present[v] = 1;
    }
    while (left > 0) {
        if (r >= max_rounds) { r = -1; goto done; }
        int64_t S = 0, c = 0, mn = INT64_MAX;
        for (int64_t v = 0; v < n; v++)
            if (present[v]) { S += deg[v]; c++; if (deg[v] < mn) mn = deg[v]; }
        int64_t np = 0;
        if (method == 2) {
            /* the s present vertices of lowest (degree, id) */
            int64_t sr = (int64_t)ceil((eps * (double)c) / (2.0 + eps));
            if (sr < 1) sr = 1;
            if (sr > c) sr = c;
            int64_t q = 0;
            for (int64_t v = 0; v < n; v++) if (present[v]) inv[q++] = (int32_t)v;
            g_deg_key = deg;
            qsort(inv, (size_t)c, sizeof(int32_t), cmp_deg_id);
            for (int64_t i = 0; i < sr; i++) {
                int32_t v = inv[i];
                peeled[np++] = v;
                round_out[v] = r;
                dap_out[v] = deg[v];
            }
        } else {
            int64_t T;
            if (method == 0) {
                double t = ((2.0 + eps) * (double)S) / (double)c;
                T = (int64_t)floor(t);
            } else if (method == 1) {
                T = INT64_MAX;
            } else {
                if (mn > Tk) Tk = mn;
                T = Tk;
            }
            if (thr_out && method != 1) thr_out[r] = T;
            for (int64_t v = 0; v < n; v++) {
                if (present[v] && (int64_t)deg[v] <= T) {
                    peeled[np++] = (int32_t)v;
                    round_out[v] = r;
                    dap_out[v] = deg[v];
                }
            }
        }
        for (int64_t i = 0; i < np; i++) present[peeled[i]] = 0;
        for (int64_t i = 0; i < np; i++) {
            int32_t v = peeled[i];
            for (int64_t e = off[v]; e < off[v + 1]; e++)
                if (present[idx[e]]) deg[idx[e]]--;
        }
        left -= np;
        r++;
    }
    for (int64_t v = 0; v < n; v++) inv[v] = (int32_t)v;
    g_round_key = round_out;
    g_dap_key = dap_out;
    qsort(inv, (size_t)n, sizeof(int32_t), cmp_rank_key);
    for (int64_t p = 0; p < n; p++) rank_out[inv[p]] = (int32_t)p;
    /* directed CSR in rank space */
    ooff_out[0] = 0;
    for (int64_t p = 0; p < n; p++) {
        int32_t v = inv[p];
        int64_t d = 0;
        for (int64_t e = off[v]; e < off[v + 1]; e++)
            if (rank_out[idx[e]] > p) d++;
        ooff_out[p + 1] = ooff_out[p] + d;
    }
    for (int64_t p = 0; p < n; p++) {
        int32_t v = inv[p];
        int64_t w = ooff_out[p];
        for (int64_t e = off[v]; e < off[v + 1]; e++)
            if (rank_out[idx[e]] > p) oidx_out[w++] = rank_out[idx[e]];
        qsort(oidx_out + ooff_out[p], (size_t)(ooff_out[p + 1] - ooff_out[p]), sizeof(int32_t), cmp_i32);
    }
done:
    free(deg); free(present); free(peeled); free(inv);
    return r;
}

int orc_orient(int64_t n, const int64_t *off, const int32_t *idx, double eps,
               int32_t *round_out, int32_t *dap_out, int32_t *rank_out,
               int64_t *ooff_out, int32_t *oidx_out, int64_t *thr_out, int max_rounds)
{
    return orc_orient_method(n, off, idx, 0, eps, round_out, dap_out, rank_out, ooff_out, oidx_out, thr_out,
                             max_rounds);
}

/* ------------------------------------------------------------------ CN counting */

typedef struct {
    const int64_t *doff;   /* directed adjacency, original ids */
    const int32_t *didx;
    int8_t *lab;           /* level labels, one per vertex, 0 when unused */
    int32_t **lvl;         /* candidate buffer per level */
    int32_t *stack;        /* vertices chosen so far */
    uint64_t *pv;          /* per-vertex counts (nullable) */
} cn_ctx;

/* Number of l-cliques inside the candidate set I (all of whose members carry label l),
 * each extending the clique already on the stack (depth entries). */
static uint64_t cn_rec(cn_ctx *c, int l, const int32_t *I, int64_t sz, int depth)
{
    if (l == 1) {
        if (c->pv) {
            for (int s = 0; s < depth; s++) c->pv[c->stack[s]] += (uint64_t)sz;
            for (int64_t i = 0; i < sz; i++) c->pv[I[i]] += 1;
        }
        return (uint64_t)sz;
    }
    if (sz < l) return 0;
    uint64_t t = 0;
    int32_t *J = c->lvl[l - 1];
    for (int64_t i = 0; i < sz; i++) {
        int32_t u = I[i];
        int64_t jz = 0;
        for (int64_t e = c->doff[u]; e < c->doff[u + 1]; e++) {
            int32_t w = c->didx[e];
            if (c->lab[w] == l) J[jz++] = w;
        }
        for (int64_t j = 0; j < jz; j++) c->lab[J[j]] = (int8_t)(l - 1);
        c->stack[depth] = u;
        t += cn_rec(c, l - 1, J, jz, depth + 1);
        for (int64_t j = 0; j < jz; j++) c->lab[J[j]] = (int8_t)l;
    }
    return t;
}

static const int64_t *g_deg_off;

static int cmp_cn_order(const void *a, const void *b)
{
    int32_t x = *(const int32_t *)a, y = *(const int32_t *)b;
    int64_t dx = g_deg_off[x + 1] - g_deg_off[x], dy = g_deg_off[y + 1] - g_deg_off[y];
    if (dx != dy) return dx > dy ? -1 : 1;          /* non-increasing degree */
    return x < y ? -1 : (x > y);                    /* then smaller id first */
}

/*
 * Total number of k-cliques of the undirected graph, and (if pv != NULL) for every
 * vertex the number of k-cliques containing it.  Chiba-Nishizeki: vertices are taken
 * in non-increasing degree order (ties: smaller id first); each vertex v counts the
 * (k-1)-cliques among its neighbours that come after it, then is deleted.  Candidate
 * sets are kept as level labels as in Sec. 3.4.
 *
 * Only roots whose position p in that order has p % stride == phase are counted
 * (stride 1, phase 0 counts everything).  nthreads > 1 splits the roots across
 * OpenMP threads.  *overflow is set if the 128-bit shadow total reaches 2^64.
 * Requires 1 <= k <= 64.  pv must hold n entries and is added to, not cleared.
 */
uint64_t orc_count(int64_t n, const int64_t *off, const int32_t *idx, int k,
                   uint64_t *pv, int nthreads, int64_t stride, int64_t phase, int *overflow)
{
    *overflow = 0;
    if (k < 1 || k > 64 || stride < 1) return 0;
    if (k == 1) {
        uint64_t t = 0;
        for (int64_t p = 0; p < n; p++)
            if (p % stride == phase) t++;
        if (pv) {
            int32_t *ord = (int32_t *)malloc(sizeof(int32_t) * (n + 1));
            for (int64_t v = 0; v < n; v++) ord[v] = (int32_t)v;
            g_deg_off = off;
            qsort(ord, (size_t)n, sizeof(int32_t), cmp_cn_order);
            for (int64_t p = 0; p < n; p++) if (p % stride == phase) pv[ord[p]] += 1;
            free(ord);
        }
        return t;
    }
    int32_t *ord = (int32_t *)malloc(sizeof(int32_t) * (n + 1));
    int64_t *pos = (int64_t *)malloc(sizeof(int64_t) * (n + 1));
    for (int64_t v = 0; v < n; v++) ord[v] = (int32_t)v;
    g_deg_off = off;
    qsort(ord, (size_t)n, sizeof(int32_t), cmp_cn_order);
    for (int64_t p = 0; p < n; p++) pos[ord[p]] = p;
    /* later neighbours of each vertex */
    int64_t *doff = (int64_t *)malloc(sizeof(int64_t) * (n + 1));
    doff[0] = 0;
    int64_t dmax = 0;
    for (int64_t v = 0; v < n; v++) {
        int64_t d = 0;
        for (int64_t e = off[v]; e < off[v + 1]; e++)
            if (pos[idx[e]] > pos[v]) d++;
        doff[v + 1] = doff[v] + d;
        if (d > dmax) dmax = d;
    }
    int32_t *didx = (int32_t *)malloc(sizeof(int32_t) * (doff[n] + 1));
    for (int64_t v = 0; v < n; v++) {
        int64_t w = doff[v];
        for (int64_t e = off[v]; e < off[v + 1]; e++)
            if (pos[idx[e]] > pos[v]) didx[w++] = idx[e];
    }
    if (nthreads < 1) nthreads = 1;
    u128 grand = 0;
#pragma omp parallel num_threads(nthreads)
    {
        cn_ctx c;
        c.doff = doff;
        c.didx = didx;
        c.lab = (int8_t *)calloc((size_t)n + 1, 1);
        c.lvl = (int32_t **)malloc(sizeof(int32_t *) * (size_t)k);
        for (int l = 0; l < k; l++) c.lvl[l] = (int32_t *)malloc(sizeof(int32_t) * (dmax + 1));
        c.stack = (int32_t *)malloc(sizeof(int32_t) * (size_t)(k + 1));
        uint64_t *mine = NULL;
        if (pv) mine = (uint64_t *)calloc((size_t)n + 1, sizeof(uint64_t));
        c.pv = mine;
        u128 acc = 0;
#pragma omp for schedule(dynamic, 16)
        for (int64_t p = 0; p < n; p++) {
            if (p % stride != phase) continue;
            int32_t v = ord[p];
            const int32_t *I = didx + doff[v];
            int64_t sz = doff[v + 1] - doff[v];
            for (int64_t i = 0; i < sz; i++) c.lab[I[i]] = (int8_t)(k - 1);
            c.stack[0] = v;
            acc += cn_rec(&c, k - 1, I, sz, 1);
            for (int64_t i = 0; i < sz; i++) c.lab[I[i]] = 0;
        }
#pragma omp critical
        {
            grand += acc;
            if (pv)
                for (int64_t v = 0; v < n; v++) pv[v] += mine[v];
        }
        free(c.lab);
        for (int l = 0; l < k; l++) free(c.lvl[l]);
        free(c.lvl);
        free(c.stack);
        free(mine);
    }
    if (grand >> 64) *overflow = 1;
    free(ord); free(pos); free(doff); free(didx);
    return (uint64_t)grand;
}

/* ------------------------------------------------------------------ brute force */

/* Every k-subset of the n <= 64 vertices is tested pair by pair.  pv (nullable) gets
 * +1 for each member of each clique found.  Returns the number of k-cliques. */
uint64_t orc_brute(int64_t n, const int64_t *off, const int32_t *idx, int k, uint64_t *pv)
{
    if (n > 64 || k < 1 || k > n) return 0;
    uint64_t adj[64];
    memset(adj, 0, sizeof(adj));
    for (int64_t v = 0; v < n; v++)
        for (int64_t e = off[v]; e < off[v + 1]; e++) adj[v] |= 1ull << idx[e];
    int c[64];
    for (int i = 0; i < k; i++) c[i] = i;
    uint64_t t = 0;
    for (;;) {
        int ok = 1;
        for (int i = 0; i < k && ok; i++)
            for (int j = i + 1; j < k; j++)
                if (!((adj[c[i]] >> c[j]) & 1)) { ok = 0; break; }
        if (ok) {
            t++;
            if (pv) for (int i = 0; i < k; i++) pv[c[i]]++;
        }
        /* next combination in lexicographic order */
        int i = k - 1;
        while (i >= 0 && c[i] == (int)n - k + i) i--;
        if (i < 0) break;
        c[i]++;
        for (int j = i + 1; j < k; j++) c[j] = c[j - 1] + 1;
    }
    return t;
}

/* ------------------------------------------------------------------ degeneracy */

/* Exact degeneracy: the largest minimum degree seen while repeatedly deleting a
 * vertex of minimum current degree, kept in degree bins (the bin-sort core decomposition
 * of Batagelj and Zaversnik, 2003). */
int64_t orc_degeneracy(int64_t n, const int64_t *off, const int32_t *idx)
{
    if (n == 0) return 0;
    int64_t md = 0;
    int64_t *deg = (int64_t *)malloc(sizeof(int64_t) * n);
    for (int64_t v = 0; v < n; v++) { deg[v] = off[v + 1] - off[v]; if (deg[v] > md) md = deg[v]; }
    int64_t *bin = (int64_t *)calloc((size_t)md + 2, sizeof(int64_t));
    int64_t *vert = (int64_t *)malloc(sizeof(int64_t) * n);
    int64_t *where = (int64_t *)malloc(sizeof(int64_t) * n);
    for (int64_t v = 0; v < n; v++) bin[deg[v]]++;
    int64_t start = 0;
    for (int64_t d = 0; d <= md; d++) { int64_t c = bin[d]; bin[d] = start; start += c; }
    for (int64_t v = 0; v < n; v++) { where[v] = bin[deg[v]]; vert[where[v]] = v; bin[deg[v]]++; }
    for (int64_t d = md; d >= 1; d--) bin[d] = bin[d - 1];
    bin[0] = 0;
    int64_t best = 0;
    for (int64_t i = 0; i < n; i++) {
        int64_t v = vert[i];
        if (deg[v] > best) best = deg[v];
        for (int64_t e = off[v]; e < off[v + 1]; e++) {
            int64_t u = idx[e];
            if (deg[u] > deg[v]) {
                int64_t du = deg[u], pu = where[u], pw = bin[du], w = vert[pw];
                if (u != w) { where[u] = pw; vert[pu] = w; where[w] = pu; vert[pw] = u; }
                bin[du]++;
                deg[u]--;
            }
        }
    }
    free(deg); free(bin); free(vert); free(where);
    return best;
}

/* ------------------------------------------------------------------ local cliques */

static uint64_t dag_rec(const int64_t *ooff, const int32_t *oidx, const int32_t *I, int64_t sz,
                        int depth, int jmax, uint64_t *cj, int32_t **buf)
{
    /* every member of I completes a clique of size depth inside G[N+(root)] */
    cj[depth - 1] += (uint64_t)sz;
    if (depth == jmax) return 0;
    int32_t *J = buf[depth];
    for (int64_t i = 0; i < sz; i++) {
        int32_t u = I[i];
        /* merge-intersect I[i+1..] with N+(u): both ascending */
        int64_t a = i + 1, b = ooff[u], jz = 0;
        while (a < sz && b < ooff[u + 1]) {
            if (I[a] < oidx[b]) a++;
            else if (I[a] > oidx[b]) b++;
            else { J[jz++] = I[a]; a++; b++; }
        }
        dag_rec(ooff, oidx, J, jz, depth + 1, jmax, cj, buf);
    }
    return 0;
}

/*
 * Directed graph with ascending arcs and ascending rows (ooff/oidx).  For every root
 * v and j = 1..jmax: out[v*jmax + j-1] = number of j-cliques inside the subgraph
 * induced by N+(v).  (c_1 = d+(v), c_2 = edges of G[N+(v)], ...)
 */
void orc_local_cliques(int64_t n, const int64_t *ooff, const int32_t *oidx, int jmax, uint64_t *out)
{
    int64_t dmax = 0;
    for (int64_t v = 0; v < n; v++) if (ooff[v + 1] - ooff[v] > dmax) dmax = ooff[v + 1] - ooff[v];
    int32_t **buf = (int32_t **)malloc(sizeof(int32_t *) * (size_t)(jmax + 1));
    for (int j = 0; j <= jmax; j++) buf[j] = (int32_t *)malloc(sizeof(int32_t) * (dmax + 1));
    for (int64_t v = 0; v < n; v++) {
        uint64_t *cj = out + v * jmax;
        for (int j = 0; j < jmax; j++) cj[j] = 0;
        if (jmax >= 1)
            dag_rec(ooff, oidx, oidx + ooff[v], ooff[v + 1] - ooff[v], 1, jmax, cj, buf);
    }
    for (int j = 0; j <= jmax; j++) free(buf[j]);
    free(buf);
}

/*
 * orc_local_cliques for the listed roots only: out[r*jmax + j-1] = number of j-cliques in
 * G[N+(roots[r])].  Roots are independent and run in parallel when built with OpenMP.
 */
void orc_local_cliques_roots(int64_t n, const int64_t *ooff, const int32_t *oidx, int jmax,
                             const int64_t *roots, int64_t nroots, int nthreads, uint64_t *out)
{
    int64_t dmax = 0;
    for (int64_t r = 0; r < nroots; r++) {
        int64_t v = roots[r];
        if (ooff[v + 1] - ooff[v] > dmax) dmax = ooff[v + 1] - ooff[v];
    }
    (void)n;
#ifdef _OPENMP
    if (nthreads > 0) omp_set_num_threads(nthreads);
#pragma omp parallel
#endif
    {
        int32_t **buf = (int32_t **)malloc(sizeof(int32_t *) * (size_t)(jmax + 1));
        for (int j = 0; j <= jmax; j++) buf[j] = (int32_t *)malloc(sizeof(int32_t) * (dmax + 1));
#ifdef _OPENMP
#pragma omp for schedule(dynamic, 1)
#endif
        for (int64_t r = 0; r < nroots; r++) {
            int64_t v = roots[r];
            uint64_t *cj = out + r * jmax;
            for (int j = 0; j < jmax; j++) cj[j] = 0;
            if (jmax >= 1)
                dag_rec(ooff, oidx, oidx + ooff[v], ooff[v + 1] - ooff[v], 1, jmax, cj, buf);
        }
        for (int j = 0; j <= jmax; j++) free(buf[j]);
        free(buf);
    }
}

/* number of `need`-cliques inside the vertex set I (ascending ids) of the undirected
 * graph: each clique is enumerated once, in ascending id order */
static uint64_t nbr_rec(const int64_t *off, const int32_t *idx, const int32_t *I, int64_t sz, int need,
                        int32_t **buf)
{
    if (need == 0) return 1;
    if (need == 1) return (uint64_t)sz;
    uint64_t total = 0;
    int32_t *J = buf[need];
    for (int64_t i = 0; i + need <= sz; i++) {
        int32_t u = I[i];
        /* members of I after u that are adjacent to u (N(u) ascending) */
        int64_t a = i + 1, b = off[u], jz = 0;
        while (a < sz && b < off[u + 1]) {
            if (I[a] < idx[b]) a++;
            else if (I[a] > idx[b]) b++;
            else { J[jz++] = I[a]; a++; b++; }
        }
        total += nbr_rec(off, idx, J, jz, need - 1, buf);
    }
    return total;
}

/*
 * For each listed vertex v of the undirected CSR (sorted rows): out[r] = number of
 * k-cliques that contain v = number of (k-1)-cliques inside G[N(v)] (k >= 1).
 */
void orc_vertex_cliques(int64_t n, const int64_t *off, const int32_t *idx, int k, const int64_t *verts,
                        int64_t nverts, int nthreads, uint64_t *out)
{
    int64_t dmax = 0;
    for (int64_t r = 0; r < nverts; r++) {
        int64_t v = verts[r];
        if (off[v + 1] - off[v] > dmax) dmax = off[v + 1] - off[v];
    }
    (void)n;
#ifdef _OPENMP
    if (nthreads > 0) omp_set_num_threads(nthreads);
#pragma omp parallel
#endif
    {
        int32_t **buf = (int32_t **)malloc(sizeof(int32_t *) * (size_t)(k + 1));
        for (int j = 0; j <= k; j++) buf[j] = (int32_t *)malloc(sizeof(int32_t) * (dmax + 1));
#ifdef _OPENMP
#pragma omp for schedule(dynamic, 1)
#endif
        for (int64_t r = 0; r < nverts; r++) {
            int64_t v = verts[r];
            out[r] = k < 1 ? 0 : nbr_rec(off, idx, idx + off[v], off[v + 1] - off[v], k - 1, buf);
        }
        for (int j = 0; j <= k; j++) free(buf[j]);
        free(buf);
    }
}

/*
 * Colorful sparsification: keep the edge {u, v} iff colors[u] == colors[v].  Rows keep
 * their order.  out_off has n+1 entries, out_idx room for every entry of idx; returns
 * the number of kept entries.
 */
int64_t orc_sparsify(int64_t n, const int64_t *off, const int32_t *idx, const int32_t *colors, int64_t *out_off,
                     int32_t *out_idx)
{
    int64_t at = 0;
    for (int64_t v = 0; v < n; v++) {
        out_off[v] = at;
        for (int64_t e = off[v]; e < off[v + 1]; e++)
            if (colors[idx[e]] == colors[v]) out_idx[at++] = idx[e];
    }
    out_off[n] = at;
    return at;
}
