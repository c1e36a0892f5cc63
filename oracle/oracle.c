/*
 * CPU ORACLE for k-clique and induced k-motif counting — TEST INFRASTRUCTURE.
 *
 * Only the test-suite, the smoke check and the benchmark's CPU-baseline leg use
 * this file.  It shares no code, header, table or helper with the GPU library:
 * it has its own CSR handling, its own canonical coder and its own enumerators.
 * It is deliberately plain and slow.
 *
 * What it computes (DuMato, Ferraz et al., arXiv 2212.04551):
 *   - Induced subgraphs and neighbourhoods: Section II (Background), Defs. 1-3.
 *   - The enumeration function E(G, tr, k) with property P and output A:
 *     Section II, Eq. (1).  Clique counting is P = "fully connected", A = count;
 *     motif counting is A = count per canonical representative (pattern).
 *   - Clique counting problem statement: Section IV-E (Programming with DuMato).
 *   - Motif counting problem statement: Section IV-E; only connected
 *     traversals are patterns (Section IV-C, Aggregate).
 *   - Canonical representative = isomorphism class.  Class ids are contiguous
 *     (Section IV-C, Aggregate); their order is not given by the paper and is
 *     read as (edge count ascending, canonical code ascending), where the
 *     canonical code is the minimum, over all k! relabellings, of the
 *     upper-triangle edge bitmap in column order: bit i(i-1)/2 + t is the edge
 *     between vertices t < i, so the edges of vertex i to its predecessors are
 *     contiguous (the bitmap layout of Section IV-C, Aggregate).
 *
 * Levels:
 *   L1  brute force over every k-subset, straight from the definitions.
 *   L2  plain enumerators: clique backtracking in (degree, id) rank order, and
 *       ESU (Wernicke 2006) for connected k-sets rooted at their lowest
 *       (degree, id) vertex.
 *       Multi-threaded over roots with pthreads.
 *
 * Per-root outputs (used for sampled parity at sizes where a full run is
 * infeasible): every clique and every connected k-set is credited to its
 * lowest vertex in (degree asc, id asc) rank.  For a root r,
 *   leaves(r) = number of k-vertex results credited to r,
 *   nodes(r)  = number of j-vertex traversals (1 <= j <= k-1) credited to r
 *               (j-cliques, or connected j-sets, whose root is r),
 *   reads(r)  = sum over those traversals of the degree (out-degree in rank
 *               order for cliques) of the vertex added last.  For cliques the
 *               last vertex is the highest-ranked one.  For motifs it is the
 *               last vertex of the set's canonical order (the reading of the
 *               canonicality filter of Section IV-E used throughout: start at
 *               the lowest-ranked vertex, then repeatedly add the lowest-ranked
 *               vertex adjacent to those already taken), so the figure depends
 *               on the set only, not on the order an enumerator visits it in.
 *
 * Per-root time budget (for choosing heavy roots the oracle can finish):
 * with root_budget > 0 each root may run for that many seconds; done[i] = 1
 * marks the roots that finished, and only those enter the totals.
 */
#define _POSIX_C_SOURCE 200809L
#include <pthread.h>
#include <stdatomic.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#include <time.h>

#define OR_MAXK 8          /* vertex arrays sized for up to 8 traversal vertices */
#define OR_MAX_MOTIF_K 8     /* class tables are built for k <= 8 */
#define OR_MAX_CLASSES 11117 /* classes of connected graphs on 8 vertices */

/* ====================================================================== */
/* canonical codes                                                         */
/* ====================================================================== */

static inline int pair_bit(int t, int i) { /* t < i */
    return i * (i - 1) / 2 + t;
}

/* graph on k labelled vertices -> edge bitmap */
static uint32_t code_from_adj(int k, const unsigned char adj[OR_MAXK][OR_MAXK]) {
    uint32_t c = 0;
    for (int i = 1; i < k; ++i)
        for (int t = 0; t < i; ++t)
            if (adj[t][i]) c |= 1u << pair_bit(t, i);
    return c;
}

static void adj_from_code(int k, uint32_t c, unsigned char adj[OR_MAXK][OR_MAXK]) {
    memset(adj, 0, sizeof(unsigned char) * OR_MAXK * OR_MAXK);
    for (int i = 1; i < k; ++i)
        for (int t = 0; t < i; ++t)
            if (c >> pair_bit(t, i) & 1u) adj[t][i] = adj[i][t] = 1;
}

static int connected_code(int k, uint32_t c) {
    unsigned char adj[OR_MAXK][OR_MAXK];
    adj_from_code(k, c, adj);
    int seen[OR_MAXK] = {0}, stack[OR_MAXK], sp = 0, cnt = 1;
    seen[0] = 1;
    stack[sp++] = 0;
    while (sp) {
        int x = stack[--sp];
        for (int y = 0; y < k; ++y)
            if (adj[x][y] && !seen[y]) { seen[y] = 1; cnt++; stack[sp++] = y; }
    }
    return cnt == k;
}

/* next permutation in lexicographic order; returns 0 after the last one */
static int next_perm(int* p, int k) {
    int i = k - 2;
    while (i >= 0 && p[i] > p[i + 1]) --i;
    if (i < 0) return 0;
    int j = k - 1;
    while (p[j] < p[i]) --j;
    int t = p[i]; p[i] = p[j]; p[j] = t;
    for (int a = i + 1, b = k - 1; a < b; ++a, --b) { t = p[a]; p[a] = p[b]; p[b] = t; }
    return 1;
}

/* minimum code over all k! relabellings */
uint32_t or_canon(int k, uint32_t c) {
    unsigned char adj[OR_MAXK][OR_MAXK];
    adj_from_code(k, c, adj);
    int p[OR_MAXK];
    for (int i = 0; i < k; ++i) p[i] = i;
    uint32_t best = 0xffffffffu;
    do {
        /* relabelled graph: new vertex p[x] takes old vertex x */
        uint32_t d = 0;
        for (int i = 1; i < k; ++i)
            for (int t = 0; t < i; ++t)
                if (adj[t][i]) {
                    int a = p[t], b = p[i];
                    d |= 1u << (a < b ? pair_bit(a, b) : pair_bit(b, a));
                }
        if (d < best) best = d;
    } while (next_perm(p, k));
    return best;
}

typedef struct {
    int ready;
    int ncls;
    uint32_t* canon;         /* ncls canonical codes, class order */
    int16_t* class_of_code;  /* 2^(k(k-1)/2) entries, -1 when disconnected */
    int64_t n_connected;     /* labelled connected graphs on k vertices */
} class_info;

static class_info g_cls[OR_MAX_MOTIF_K + 1];
static pthread_mutex_t g_cls_lock = PTHREAD_MUTEX_INITIALIZER;

static int cmp_canon(const void* a, const void* b) {
    uint32_t x = *(const uint32_t*)a, y = *(const uint32_t*)b;
    int px = __builtin_popcount(x), py = __builtin_popcount(y);
    if (px != py) return px < py ? -1 : 1;
    return x < y ? -1 : (x > y ? 1 : 0);
}

/* canonical code of every connected code, by one of two methods:
   - per code: the minimum over all k! relabellings (or_canon);
   - by orbits: codes are visited in increasing order; the first connected
     code not yet labelled is the smallest member of its orbit (every smaller
     code is labelled already, and relabelling maps an orbit onto itself), so
     all k! relabellings of it are labelled with it.
   The second visits each class once instead of each code, which is what
   makes k = 7 (2^21 codes, 853 classes) and k = 8 (2^28 codes, 11117
   classes) affordable.  canon_of[c] =
   0xffffffff for disconnected codes; returns the number of connected codes. */
static int64_t canon_table(int k, uint32_t* canon_of, int by_orbits) {
    const uint32_t ncodes = 1u << (k * (k - 1) / 2);
    int64_t n_conn = 0;
    if (!by_orbits) {
        for (uint32_t c = 0; c < ncodes; ++c) {
            if (!connected_code(k, c)) { canon_of[c] = 0xffffffffu; continue; }
            n_conn++;
            canon_of[c] = or_canon(k, c);
        }
        return n_conn;
    }
    const uint32_t unset = 0xfffffffeu;
    for (uint32_t c = 0; c < ncodes; ++c) canon_of[c] = unset;
    for (uint32_t c = 0; c < ncodes; ++c) {
        if (canon_of[c] != unset) continue;
        if (!connected_code(k, c)) { canon_of[c] = 0xffffffffu; continue; }
        /* the code's edges as (t, i) pairs, relabelled by every permutation */
        int et[32], ei[32], ne = 0;
        for (int i = 1; i < k; ++i)
            for (int t = 0; t < i; ++t)
                if (c >> pair_bit(t, i) & 1u) { et[ne] = t; ei[ne] = i; ++ne; }
        int p[OR_MAXK];
        for (int i = 0; i < k; ++i) p[i] = i;
        do {
            uint32_t d = 0;
            for (int e = 0; e < ne; ++e) {
                int a = p[et[e]], b = p[ei[e]];
                d |= 1u << (a < b ? pair_bit(a, b) : pair_bit(b, a));
            }
            canon_of[d] = c;
        } while (next_perm(p, k));
    }
    for (uint32_t c = 0; c < ncodes; ++c)
        if (canon_of[c] != 0xffffffffu) n_conn++;
    return n_conn;
}

static int cmp_u32(const void* a, const void* b) {
    uint32_t x = *(const uint32_t*)a, y = *(const uint32_t*)b;
    return x < y ? -1 : (x > y ? 1 : 0);
}

static const class_info* classes(int k) {
    if (k < 1 || k > OR_MAX_MOTIF_K) return NULL;
    pthread_mutex_lock(&g_cls_lock);
    class_info* ci = &g_cls[k];
    if (!ci->ready) {
        uint32_t ncodes = 1u << (k * (k - 1) / 2);
        uint32_t* canon_of = (uint32_t*)malloc(sizeof(uint32_t) * ncodes);
        ci->n_connected = canon_table(k, canon_of, k >= 7);
        /* classes: the distinct canonical codes (each is its own canon) */
        int nu = 0;
        for (uint32_t c = 0; c < ncodes; ++c)
            if (canon_of[c] == c) nu++;
        uint32_t* uniq = (uint32_t*)malloc(sizeof(uint32_t) * (size_t)(nu > 0 ? nu : 1));
        nu = 0;
        for (uint32_t c = 0; c < ncodes; ++c)
            if (canon_of[c] == c) uniq[nu++] = c;
        qsort(uniq, (size_t)nu, sizeof(uint32_t), cmp_canon);
        ci->ncls = nu;
        ci->canon = (uint32_t*)malloc(sizeof(uint32_t) * (size_t)(nu > 0 ? nu : 1));
        memcpy(ci->canon, uniq, sizeof(uint32_t) * (size_t)nu);
        /* canonical code -> class id, through a code-sorted copy */
        typedef struct { uint32_t code; int16_t cls; } pair_t;
        pair_t* byc = (pair_t*)malloc(sizeof(pair_t) * (size_t)(nu > 0 ? nu : 1));
        for (int q = 0; q < nu; ++q) { byc[q].code = ci->canon[q]; byc[q].cls = (int16_t)q; }
        qsort(byc, (size_t)nu, sizeof(pair_t), cmp_u32);  /* code is the first member */
        ci->class_of_code = (int16_t*)malloc(sizeof(int16_t) * ncodes);
        for (uint32_t c = 0; c < ncodes; ++c) {
            ci->class_of_code[c] = -1;
            if (canon_of[c] == 0xffffffffu) continue;
            int lo = 0, hi = nu - 1;
            while (lo < hi) {
                int mid = (lo + hi) / 2;
                if (byc[mid].code < canon_of[c]) lo = mid + 1; else hi = mid;
            }
            ci->class_of_code[c] = byc[lo].cls;
        }
        free(byc);
        free(canon_of);
        free(uniq);
        ci->ready = 1;
    }
    pthread_mutex_unlock(&g_cls_lock);
    return ci;
}

/* 1 when the orbit method and the per-code minimum give the same canonical
   code for every code on k vertices (k <= 6), 0 otherwise, -1 if unsupported */
int or_canon_methods_agree(int k) {
    if (k < 1 || k > 6) return -1;
    uint32_t ncodes = 1u << (k * (k - 1) / 2);
    uint32_t* a = (uint32_t*)malloc(sizeof(uint32_t) * ncodes);
    uint32_t* b = (uint32_t*)malloc(sizeof(uint32_t) * ncodes);
    int64_t na = canon_table(k, a, 0), nb = canon_table(k, b, 1);
    int same = na == nb && memcmp(a, b, sizeof(uint32_t) * ncodes) == 0;
    free(a);
    free(b);
    return same;
}

/* number of classes of connected graphs on k vertices, -1 if unsupported */
int or_num_classes(int k) {
    const class_info* ci = classes(k);
    return ci ? ci->ncls : -1;
}

/* canonical codes in class order; returns ncls */
int or_class_canon(int k, uint32_t* out, int cap) {
    const class_info* ci = classes(k);
    if (!ci) return -1;
    for (int q = 0; q < ci->ncls && q < cap; ++q) out[q] = ci->canon[q];
    return ci->ncls;
}

int64_t or_num_connected_labelled(int k) {
    const class_info* ci = classes(k);
    return ci ? ci->n_connected : -1;
}

/* class of a full edge bitmap, -1 when disconnected or k unsupported */
int or_class_of_code(int k, uint32_t code) {
    const class_info* ci = classes(k);
    if (!ci || code >= (1u << (k * (k - 1) / 2))) return -1;
    return ci->class_of_code[code];
}

/* the same for an array of codes (out[i] = class of codes[i], or -1) */
void or_class_of_codes(int k, const int64_t* codes, int64_t n, int64_t* out) {
    for (int64_t i = 0; i < n; ++i) out[i] = or_class_of_code(k, (uint32_t)codes[i]);
}

/* ====================================================================== */
/* graph helpers                                                           */
/* ====================================================================== */

typedef struct {
    int32_t n;
    const int64_t* rp;
    const int32_t* col;
} graph_t;

static int has_edge(const graph_t* g, int32_t a, int32_t b) {
    int64_t lo = g->rp[a], hi = g->rp[a + 1];
    while (lo < hi) {
        int64_t mid = (lo + hi) / 2;
        int32_t x = g->col[mid];
        if (x == b) return 1;
        if (x < b) lo = mid + 1; else hi = mid;
    }
    return 0;
}

static inline int64_t deg_of(const graph_t* g, int32_t v) { return g->rp[v + 1] - g->rp[v]; }

/* ====================================================================== */
/* L1: brute force over k-subsets                                          */
/* ====================================================================== */

/* out_total: number of k-cliques; per_root_leaves (nullable, n): credited to min rank */
int or_clique_brute(int32_t n, const int64_t* rp, const int32_t* col, int k,
                    uint64_t* out_total, uint64_t* per_root_leaves) {
    graph_t g = { n, rp, col };
    if (k < 1 || k > 32) return -1;
    *out_total = 0;
    if (per_root_leaves) memset(per_root_leaves, 0, sizeof(uint64_t) * (size_t)n);
    if (k > n) return 0;
    int idx[32];
    for (int i = 0; i < k; ++i) idx[i] = i;
    for (;;) {
        int ok = 1;
        for (int a = 0; a < k && ok; ++a)
            for (int b = a + 1; b < k && ok; ++b)
                if (!has_edge(&g, idx[a], idx[b])) ok = 0;
        if (ok) {
            (*out_total)++;
            if (per_root_leaves) {
                int r = idx[0];
                for (int a = 1; a < k; ++a) {
                    int x = idx[a];
                    int64_t dx = deg_of(&g, x), dr = deg_of(&g, r);
                    if (dx < dr || (dx == dr && x < r)) r = x;
                }
                per_root_leaves[r]++;
            }
        }
        int i = k - 1;
        while (i >= 0 && idx[i] == n - k + i) --i;
        if (i < 0) break;
        idx[i]++;
        for (int j = i + 1; j < k; ++j) idx[j] = idx[j - 1] + 1;
    }
    return 0;
}

/* out_counts: ncls entries; per_root_leaves (nullable, n): connected k-sets by min id */
int or_motif_brute(int32_t n, const int64_t* rp, const int32_t* col, int k,
                   uint64_t* out_counts, uint64_t* per_root_leaves) {
    graph_t g = { n, rp, col };
    const class_info* ci = classes(k);
    if (!ci || k < 2) return -1;
    memset(out_counts, 0, sizeof(uint64_t) * (size_t)ci->ncls);
    if (per_root_leaves) memset(per_root_leaves, 0, sizeof(uint64_t) * (size_t)n);
    if (k > n) return 0;
    int idx[OR_MAXK];
    for (int i = 0; i < k; ++i) idx[i] = i;
    unsigned char adj[OR_MAXK][OR_MAXK];
    for (;;) {
        memset(adj, 0, sizeof adj);
        for (int a = 0; a < k; ++a)
            for (int b = a + 1; b < k; ++b)
                if (has_edge(&g, idx[a], idx[b])) adj[a][b] = adj[b][a] = 1;
        uint32_t c = code_from_adj(k, adj);
        int q = ci->class_of_code[c];
        if (q >= 0) {
            out_counts[q]++;
            if (per_root_leaves) {
                int r = idx[0];
                for (int a = 1; a < k; ++a) {
                    int x = idx[a];
                    int64_t dx = deg_of(&g, x), dr = deg_of(&g, r);
                    if (dx < dr || (dx == dr && x < r)) r = x;
                }
                per_root_leaves[r]++;
            }
        }
        int i = k - 1;
        while (i >= 0 && idx[i] == n - k + i) --i;
        if (i < 0) break;
        idx[i]++;
        for (int j = i + 1; j < k; ++j) idx[j] = idx[j - 1] + 1;
    }
    return 0;
}

/* ====================================================================== */
/* L2 shared plumbing: a root list processed by a thread pool               */
/* ====================================================================== */

typedef struct {
    graph_t g;
    int k;
    const int32_t* roots;
    int64_t nroots;
    atomic_llong next;
    uint64_t* leaves;   /* nroots, nullable */
    uint64_t* nodes;    /* nroots, nullable */
    uint64_t* reads;    /* nroots, nullable */
    /* clique */
    const int64_t* rank;
    const int64_t* outdeg;   /* neighbours of higher rank */
    /* motif */
    const class_info* ci;
    /* optional per-root budget (seconds; 0 = none), completion flags, and
       per-root class counts (motifs; nroots x ncls) */
    double root_budget;
    uint8_t* done;
    uint64_t* root_counts;
    /* optional wall-clock deadline (CLOCK_MONOTONIC seconds; 0 = none) */
    double deadline;
    atomic_int expired;
    atomic_llong started;
    /* reduction */
    pthread_mutex_t lock;
    uint64_t total;
    uint64_t counts[OR_MAX_CLASSES];
    int overflow;
} job_t;

static void add_u64(uint64_t* acc, uint64_t x, int* ovf) {
    if (__builtin_add_overflow(*acc, x, acc)) *ovf = 1;
}

static double now_s(void) {
    struct timespec ts;
    clock_gettime(CLOCK_MONOTONIC, &ts);
    return (double)ts.tv_sec + 1e-9 * (double)ts.tv_nsec;
}

/* Per-thread stop state for the current root: its own budget's deadline
   (0 = none) and whether it ran out. */
typedef struct {
    double deadline;
    int out;
} root_clock;

/* true once the job's deadline or the current root's budget has passed
   (the clock is read every 4096 calls per thread) */
static int past_deadline(job_t* J, unsigned* tick, root_clock* rc) {
    if (rc->out) return 1;
    if (J->deadline <= 0.0 && rc->deadline <= 0.0) return 0;
    if (J->deadline > 0.0 && atomic_load(&J->expired)) return 1;
    if ((++*tick & 4095u) == 0) {
        double t = now_s();
        if (J->deadline > 0.0 && t > J->deadline) atomic_store(&J->expired, 1);
        if (rc->deadline > 0.0 && t > rc->deadline) rc->out = 1;
    }
    return rc->out || (J->deadline > 0.0 && atomic_load(&J->expired));
}

static void root_clock_start(const job_t* J, root_clock* rc) {
    rc->out = 0;
    rc->deadline = J->root_budget > 0.0 ? now_s() + J->root_budget : 0.0;
}

/* ---------------------------------------------------------------- cliques */

typedef struct {
    uint64_t leaves, nodes, reads;
    int ovf;
    int32_t* buf[33];   /* candidate list per depth */
    int64_t cap;
    unsigned tick;
    root_clock rc;
} clq_ctx;


/*
 * cand: vertices (sorted by id) adjacent to every traversal vertex and ranked
 * above the last one; s = traversal size.  The traversal is a clique of size s
 * whose last vertex is `last`.
 */
static void clq_expand(job_t* J, clq_ctx* C, int s, int32_t last, const int32_t* cand, int64_t nc) {
    if (past_deadline(J, &C->tick, &C->rc)) return;
    add_u64(&C->nodes, 1, &C->ovf);
    add_u64(&C->reads, (uint64_t)J->outdeg[last], &C->ovf);
    if (s == J->k - 1) { add_u64(&C->leaves, (uint64_t)nc, &C->ovf); return; }
    int32_t* nxt = C->buf[s + 1];
    for (int64_t i = 0; i < nc; ++i) {
        int32_t u = cand[i];
        /* cand ∩ N(u), keeping ranks above u (merge of two id-sorted lists) */
        int64_t a = 0, b = J->g.rp[u], be = J->g.rp[u + 1], m = 0;
        while (a < nc && b < be) {
            int32_t x = cand[a], y = J->g.col[b];
            if (x < y) a++;
            else if (y < x) b++;
            else { if (J->rank[x] > J->rank[u]) nxt[m++] = x; a++; b++; }
        }
        clq_expand(J, C, s + 1, u, nxt, m);
    }
}

static void* clq_worker(void* arg) {
    job_t* J = (job_t*)arg;
    clq_ctx C;
    memset(&C, 0, sizeof C);
    int64_t maxd = 0;
    for (int32_t v = 0; v < J->g.n; ++v) if (deg_of(&J->g, v) > maxd) maxd = deg_of(&J->g, v);
    for (int s = 0; s <= J->k && s <= 32; ++s) C.buf[s] = (int32_t*)malloc(sizeof(int32_t) * (size_t)(maxd + 1));
    uint64_t total = 0;
    int ovf = 0;
    for (;;) {
        if (J->deadline > 0.0 && (atomic_load(&J->expired) || now_s() > J->deadline)) break;
        int64_t i = atomic_fetch_add(&J->next, 1);
        if (i >= J->nroots) break;
        atomic_fetch_add(&J->started, 1);
        int32_t r = J->roots[i];
        C.leaves = C.nodes = C.reads = 0;
        root_clock_start(J, &C.rc);
        if (J->k == 1) {
            C.leaves = 1;
        } else {
            int64_t m = 0;
            for (int64_t e = J->g.rp[r]; e < J->g.rp[r + 1]; ++e)
                if (J->rank[J->g.col[e]] > J->rank[r]) C.buf[1][m++] = J->g.col[e];
            clq_expand(J, &C, 1, r, C.buf[1], m);
        }
        if (J->leaves) J->leaves[i] = C.leaves;
        if (J->nodes) J->nodes[i] = C.nodes;
        if (J->reads) J->reads[i] = C.reads;
        if (J->done) J->done[i] = C.rc.out ? 0 : 1;
        /* a root stopped by its own budget does not enter the total */
        if (!C.rc.out || J->deadline > 0.0) add_u64(&total, C.leaves, &ovf);
    }
    for (int s = 0; s <= J->k && s <= 32; ++s) free(C.buf[s]);
    pthread_mutex_lock(&J->lock);
    add_u64(&J->total, total, &J->overflow);
    if (ovf || C.ovf) J->overflow = 1;
    pthread_mutex_unlock(&J->lock);
    return NULL;
}

static int cmp_rank_key(const void* a, const void* b) {
    const int64_t* x = (const int64_t*)a;
    const int64_t* y = (const int64_t*)b;
    if (x[0] != y[0]) return x[0] < y[0] ? -1 : 1;
    return x[1] < y[1] ? -1 : (x[1] > y[1] ? 1 : 0);
}

/* rank[v] = position of v in (degree asc, id asc) order */
static int64_t* make_rank(const graph_t* g) {
    int64_t* key = (int64_t*)malloc(sizeof(int64_t) * 2 * (size_t)(g->n > 0 ? g->n : 1));
    for (int32_t v = 0; v < g->n; ++v) { key[2 * v] = deg_of(g, v); key[2 * v + 1] = v; }
    qsort(key, (size_t)g->n, 2 * sizeof(int64_t), cmp_rank_key);
    int64_t* rank = (int64_t*)malloc(sizeof(int64_t) * (size_t)(g->n > 0 ? g->n : 1));
    for (int32_t i = 0; i < g->n; ++i) rank[key[2 * i + 1]] = i;
    free(key);
    return rank;
}

static void run_pool(job_t* J, int nthreads, void* (*fn)(void*)) {
    if (nthreads < 1) nthreads = 1;
    if (nthreads > 256) nthreads = 256;
    pthread_t th[256];
    for (int t = 0; t < nthreads; ++t) pthread_create(&th[t], NULL, fn, J);
    for (int t = 0; t < nthreads; ++t) pthread_join(th[t], NULL);
}

/*
 * k-cliques credited to the listed roots (all vertices when roots == NULL).
 * leaves / nodes / reads (nullable, nroots entries) get the per-root records.
 * With root_budget > 0 each root runs for at most that many seconds; done
 * (nullable) marks the roots that finished, and only those are in *out_total.
 * Returns 0, or 1 when a uint64 sum overflowed, or -1 on bad arguments.
 */
int or_clique_roots(int32_t n, const int64_t* rp, const int32_t* col, int k,
                    const int32_t* roots, int64_t nroots, int nthreads, uint64_t* out_total,
                    uint64_t* leaves, uint64_t* nodes, uint64_t* reads, double root_budget,
                    uint8_t* done) {
    if (k < 1 || k > 32 || n < 0) return -1;
    job_t* J = (job_t*)calloc(1, sizeof(job_t));
    J->g = (graph_t){ n, rp, col };
    J->k = k;
    int32_t* all = NULL;
    if (!roots) {
        all = (int32_t*)malloc(sizeof(int32_t) * (size_t)(n > 0 ? n : 1));
        for (int32_t v = 0; v < n; ++v) all[v] = v;
        roots = all;
        nroots = n;
    }
    J->roots = roots;
    J->nroots = nroots;
    atomic_init(&J->next, 0);
    J->leaves = leaves; J->nodes = nodes; J->reads = reads;
    J->root_budget = root_budget;
    J->done = done;
    J->rank = make_rank(&J->g);
    int64_t* od = (int64_t*)calloc((size_t)(n > 0 ? n : 1), sizeof(int64_t));
    for (int32_t v = 0; v < n; ++v)
        for (int64_t e = rp[v]; e < rp[v + 1]; ++e)
            if (J->rank[col[e]] > J->rank[v]) od[v]++;
    J->outdeg = od;
    pthread_mutex_init(&J->lock, NULL);
    run_pool(J, nthreads, clq_worker);
    free(od);
    *out_total = J->total;
    int ret = J->overflow ? 1 : 0;
    free((void*)J->rank);
    free(all);
    pthread_mutex_destroy(&J->lock);
    free(J);
    return ret;
}

/* ---------------------------------------------------------------- motifs (ESU)
 * ESU over the total order (degree, id): a connected k-set is enumerated once,
 * from its lowest-ranked vertex (Wernicke 2006 works for any total order). */

typedef struct {
    job_t* J;
    unsigned tick;
    int32_t root;
    int32_t sub[OR_MAXK];
    int32_t* ext[OR_MAXK + 1];  /* extension list per depth */
    int32_t* blocked;           /* # of sub vertices adjacent to x, or in sub (n entries) */
    uint64_t leaves, nodes, reads;
    uint64_t counts[OR_MAX_CLASSES]; /* per class, the current root only */
    int ovf;
    root_clock rc;
} esu_ctx;

/* edge bitmap (column order) of sub[0..s-1] */
static uint32_t sub_code(const esu_ctx* E, int s) {
    const graph_t* g = &E->J->g;
    uint32_t c = 0;
    for (int i = 1; i < s; ++i)
        for (int t = 0; t < i; ++t)
            if (has_edge(g, E->sub[t], E->sub[i])) c |= 1u << pair_bit(t, i);
    return c;
}

/* the k-set sub[0..k-2] + w: its class from the edge bitmap; `prefix` is the
   bitmap of sub[0..k-2] */
static void esu_leaf(esu_ctx* E, uint32_t prefix, int32_t w) {
    const job_t* J = E->J;
    int k = J->k;
    uint32_t c = prefix;
    for (int t = 0; t < k - 1; ++t)
        if (has_edge(&J->g, E->sub[t], w)) c |= 1u << pair_bit(t, k - 1);
    int q = J->ci->class_of_code[c];
    if (q >= 0) add_u64(&E->counts[q], 1, &E->ovf);
    add_u64(&E->leaves, 1, &E->ovf);
}

/* Last vertex of the canonical order of the connected set sub[0..s-1]: start
   at the lowest-ranked vertex, then repeatedly take the lowest-ranked vertex
   adjacent to one already taken. */
static int32_t canonical_last(const esu_ctx* E, int s) {
    const job_t* J = E->J;
    int taken[OR_MAXK] = {0};
    int first = 0;
    for (int i = 1; i < s; ++i)
        if (J->rank[E->sub[i]] < J->rank[E->sub[first]]) first = i;
    taken[first] = 1;
    int last = first;
    for (int step = 1; step < s; ++step) {
        int best = -1;
        for (int i = 0; i < s; ++i) {
            if (taken[i]) continue;
            int adj = 0;
            for (int t = 0; t < s && !adj; ++t)
                if (taken[t] && has_edge(&J->g, E->sub[t], E->sub[i])) adj = 1;
            if (adj && (best < 0 || J->rank[E->sub[i]] < J->rank[E->sub[best]])) best = i;
        }
        taken[best] = 1;
        last = best;
    }
    return E->sub[last];
}

/* mark / unmark the closed neighbourhood of a vertex that joins / leaves sub */
static void esu_block(esu_ctx* E, int32_t w, int d) {
    const graph_t* g = &E->J->g;
    E->blocked[w] += d;
    for (int64_t e = g->rp[w]; e < g->rp[w + 1]; ++e) E->blocked[g->col[e]] += d;
}

/*
 * ESU step: sub has s vertices (blocked[] marks sub and N(sub)); ext holds
 * candidate vertices (ranked above the root, in the exclusive neighbourhood).
 */
static void esu_extend(esu_ctx* E, int s, const int32_t* ext, int64_t ne) {
    job_t* J = E->J;
    const graph_t* g = &J->g;
    if (past_deadline(J, &E->tick, &E->rc)) return;
    add_u64(&E->nodes, 1, &E->ovf);
    add_u64(&E->reads, (uint64_t)deg_of(g, canonical_last(E, s)), &E->ovf);
    if (s == J->k - 1) {
        /* every candidate completes a k-set: classify it; the extension list
           and neighbourhood marks of a deeper level are not needed */
        uint32_t prefix = sub_code(E, s);
        for (int64_t i = ne - 1; i >= 0; --i) esu_leaf(E, prefix, ext[i]);
        return;
    }
    int32_t* nxt = E->ext[s + 1];
    /* remove candidates one at a time from the back of the list */
    for (int64_t i = ne - 1; i >= 0; --i) {
        int32_t w = ext[i];
        /* remaining extension: ext[0..i-1] plus exclusive neighbours of w above the root */
        int64_t m = 0;
        for (int64_t j = 0; j < i; ++j) nxt[m++] = ext[j];
        for (int64_t e = g->rp[w]; e < g->rp[w + 1]; ++e) {
            int32_t u = g->col[e];
            if (J->rank[u] > J->rank[E->root] && E->blocked[u] == 0) nxt[m++] = u;
        }
        E->sub[s] = w;
        esu_block(E, w, +1);
        esu_extend(E, s + 1, nxt, m);
        esu_block(E, w, -1);
    }
}

static void* esu_worker(void* arg) {
    job_t* J = (job_t*)arg;
    esu_ctx E;
    memset(&E, 0, sizeof E);
    E.J = J;
    int64_t maxd = 0;
    for (int32_t v = 0; v < J->g.n; ++v) if (deg_of(&J->g, v) > maxd) maxd = deg_of(&J->g, v);
    for (int s = 0; s <= J->k; ++s)
        E.ext[s] = (int32_t*)malloc(sizeof(int32_t) * (size_t)((maxd + 1) * (s + 1) + 1));
    E.blocked = (int32_t*)calloc((size_t)(J->g.n > 0 ? J->g.n : 1), sizeof(int32_t));
    for (;;) {
        if (J->deadline > 0.0 && (atomic_load(&J->expired) || now_s() > J->deadline)) break;
        int64_t i = atomic_fetch_add(&J->next, 1);
        if (i >= J->nroots) break;
        atomic_fetch_add(&J->started, 1);
        int32_t r = J->roots[i];
        E.root = r;
        E.leaves = E.nodes = E.reads = 0;
        memset(E.counts, 0, sizeof E.counts);
        root_clock_start(J, &E.rc);
        E.sub[0] = r;
        if (J->k == 1) {
            add_u64(&E.counts[0], 1, &E.ovf);
            E.leaves = 1;
        } else {
            int64_t m = 0;
            for (int64_t e = J->g.rp[r]; e < J->g.rp[r + 1]; ++e)
                if (J->rank[J->g.col[e]] > J->rank[r]) E.ext[1][m++] = J->g.col[e];
            esu_block(&E, r, +1);
            esu_extend(&E, 1, E.ext[1], m);
            esu_block(&E, r, -1);
        }
        if (J->leaves) J->leaves[i] = E.leaves;
        if (J->nodes) J->nodes[i] = E.nodes;
        if (J->reads) J->reads[i] = E.reads;
        if (J->done) J->done[i] = E.rc.out ? 0 : 1;
        if (J->root_counts)
            for (int q = 0; q < J->ci->ncls; ++q) J->root_counts[i * J->ci->ncls + q] = E.counts[q];
        /* a root stopped by its own budget does not enter the totals */
        if (!E.rc.out || J->deadline > 0.0) {
            pthread_mutex_lock(&J->lock);
            for (int q = 0; q < J->ci->ncls; ++q) add_u64(&J->counts[q], E.counts[q], &J->overflow);
            pthread_mutex_unlock(&J->lock);
        }
    }
    pthread_mutex_lock(&J->lock);
    if (E.ovf) J->overflow = 1;
    pthread_mutex_unlock(&J->lock);
    for (int s = 0; s <= J->k; ++s) free(E.ext[s]);
    free(E.blocked);
    return NULL;
}

/*
 * Connected induced k-sets credited to the listed roots (all when roots == NULL),
 * counted per class into out_counts (ncls entries).  Per-root records as for
 * cliques, plus root_counts (nullable, nroots x ncls) with each root's own
 * class counts; root_budget / done as for cliques (out_counts then holds the
 * finished roots only).  Returns 0, 1 on overflow, -1 on bad arguments.
 */
int or_motif_roots(int32_t n, const int64_t* rp, const int32_t* col, int k,
                   const int32_t* roots, int64_t nroots, int nthreads, uint64_t* out_counts,
                   uint64_t* leaves, uint64_t* nodes, uint64_t* reads, double root_budget,
                   uint8_t* done, uint64_t* root_counts) {
    const class_info* ci = classes(k);
    if (!ci || n < 0 || k > OR_MAX_MOTIF_K) return -1;
    job_t* J = (job_t*)calloc(1, sizeof(job_t));
    J->g = (graph_t){ n, rp, col };
    J->k = k;
    J->ci = ci;
    int32_t* all = NULL;
    if (!roots) {
        all = (int32_t*)malloc(sizeof(int32_t) * (size_t)(n > 0 ? n : 1));
        for (int32_t v = 0; v < n; ++v) all[v] = v;
        roots = all;
        nroots = n;
    }
    J->roots = roots;
    J->nroots = nroots;
    atomic_init(&J->next, 0);
    J->leaves = leaves; J->nodes = nodes; J->reads = reads;
    J->root_budget = root_budget;
    J->done = done;
    J->root_counts = root_counts;
    J->rank = make_rank(&J->g);
    pthread_mutex_init(&J->lock, NULL);
    run_pool(J, nthreads, esu_worker);
    for (int q = 0; q < ci->ncls; ++q) out_counts[q] = J->counts[q];
    int ret = J->overflow ? 1 : 0;
    free((void*)J->rank);
    free(all);
    pthread_mutex_destroy(&J->lock);
    free(J);
    return ret;
}

/* ====================================================================== */
/* per-vertex features (degree, 2-hop degree sum, core number, triangles)   */
/* ====================================================================== */

/* twohop[v] = sum of deg(u) over neighbours u of v */
void or_twohop(int32_t n, const int64_t* rp, const int32_t* col, int64_t* out) {
    for (int32_t v = 0; v < n; ++v) {
        int64_t s = 0;
        for (int64_t e = rp[v]; e < rp[v + 1]; ++e) s += rp[col[e] + 1] - rp[col[e]];
        out[v] = s;
    }
}

/* triangles containing each vertex: one pass over edges u < v, merging N(u), N(v) */
void or_triangles(int32_t n, const int64_t* rp, const int32_t* col, int64_t* out) {
    memset(out, 0, sizeof(int64_t) * (size_t)n);
    for (int32_t u = 0; u < n; ++u)
        for (int64_t e = rp[u]; e < rp[u + 1]; ++e) {
            int32_t v = col[e];
            if (v <= u) continue;
            int64_t a = rp[u], b = rp[v];
            while (a < rp[u + 1] && b < rp[v + 1]) {
                int32_t x = col[a], y = col[b];
                if (x < y) a++;
                else if (y < x) b++;
                else { if (x > v) { out[u]++; out[v]++; out[x]++; } a++; b++; }
            }
        }
}

/*
 * Core numbers by repeated removal of a minimum-degree vertex (the peeling
 * definition of the k-core decomposition), with the bucket queue of
 * Batagelj & Zaversnik (2003).
 */
void or_core(int32_t n, const int64_t* rp, const int32_t* col, int32_t* core) {
    if (n <= 0) return;
    int32_t* deg = (int32_t*)malloc(sizeof(int32_t) * (size_t)n);
    int32_t md = 0;
    for (int32_t v = 0; v < n; ++v) { deg[v] = (int32_t)(rp[v + 1] - rp[v]); if (deg[v] > md) md = deg[v]; }
    int32_t* bin = (int32_t*)calloc((size_t)md + 2, sizeof(int32_t));
    int32_t* pos = (int32_t*)malloc(sizeof(int32_t) * (size_t)n);
    int32_t* vert = (int32_t*)malloc(sizeof(int32_t) * (size_t)n);
    for (int32_t v = 0; v < n; ++v) bin[deg[v]]++;
    int32_t start = 0;
    for (int32_t d = 0; d <= md; ++d) { int32_t num = bin[d]; bin[d] = start; start += num; }
    for (int32_t v = 0; v < n; ++v) { pos[v] = bin[deg[v]]; vert[pos[v]] = v; bin[deg[v]]++; }
    for (int32_t d = md; d >= 1; --d) bin[d] = bin[d - 1];
    bin[0] = 0;
    for (int32_t i = 0; i < n; ++i) {
        int32_t v = vert[i];
        for (int64_t e = rp[v]; e < rp[v + 1]; ++e) {
            int32_t u = col[e];
            if (deg[u] > deg[v]) {
                int32_t du = deg[u], pu = pos[u], pw = bin[du], w = vert[pw];
                if (u != w) { pos[u] = pw; vert[pu] = w; pos[w] = pu; vert[pw] = u; }
                bin[du]++;
                deg[u]--;
            }
        }
    }
    for (int32_t v = 0; v < n; ++v) core[v] = deg[v];
    free(deg); free(bin); free(pos); free(vert);
}

/* ====================================================================== */
/* time-bounded runs (CPU throughput baseline)                             */
/* ====================================================================== */

/*
 * Same enumeration as or_clique_roots / or_motif_roots over the listed roots,
 * stopped once `seconds` of wall-clock time have passed: threads take no new
 * root and abandon the current one.  Every subgraph found before the stop is
 * counted.  Returns the subgraphs found; *started = roots begun, *elapsed =
 * seconds used.
 */
uint64_t or_clique_timed(int32_t n, const int64_t* rp, const int32_t* col, int k, const int32_t* roots,
                         int64_t nroots, int nthreads, double seconds, int64_t* started, double* elapsed) {
    job_t* J = (job_t*)calloc(1, sizeof(job_t));
    J->g = (graph_t){ n, rp, col };
    J->k = k;
    J->roots = roots;
    J->nroots = nroots;
    atomic_init(&J->next, 0);
    atomic_init(&J->expired, 0);
    atomic_init(&J->started, 0);
    J->rank = make_rank(&J->g);
    int64_t* od = (int64_t*)calloc((size_t)(n > 0 ? n : 1), sizeof(int64_t));
    for (int32_t v = 0; v < n; ++v)
        for (int64_t e = rp[v]; e < rp[v + 1]; ++e)
            if (J->rank[col[e]] > J->rank[v]) od[v]++;
    J->outdeg = od;
    pthread_mutex_init(&J->lock, NULL);
    double t0 = now_s();
    J->deadline = t0 + seconds;
    run_pool(J, nthreads, clq_worker);
    *elapsed = now_s() - t0;
    *started = atomic_load(&J->started);
    uint64_t tot = J->total;
    free(od);
    free((void*)J->rank);
    pthread_mutex_destroy(&J->lock);
    free(J);
    return tot;
}

uint64_t or_motif_timed(int32_t n, const int64_t* rp, const int32_t* col, int k, const int32_t* roots,
                        int64_t nroots, int nthreads, double seconds, int64_t* started, double* elapsed) {
    const class_info* ci = classes(k);
    if (!ci) return 0;
    job_t* J = (job_t*)calloc(1, sizeof(job_t));
    J->g = (graph_t){ n, rp, col };
    J->k = k;
    J->ci = ci;
    J->roots = roots;
    J->nroots = nroots;
    atomic_init(&J->next, 0);
    atomic_init(&J->expired, 0);
    atomic_init(&J->started, 0);
    J->rank = make_rank(&J->g);
    pthread_mutex_init(&J->lock, NULL);
    double t0 = now_s();
    J->deadline = t0 + seconds;
    run_pool(J, nthreads, esu_worker);
    free((void*)J->rank);
    *elapsed = now_s() - t0;
    *started = atomic_load(&J->started);
    uint64_t tot = 0;
    for (int q = 0; q < ci->ncls; ++q) tot += J->counts[q];
    pthread_mutex_destroy(&J->lock);
    free(J);
    return tot;
}

/* ====================================================================== */
/* Directed graphs (Section II: the method is stated for undirected graphs */
/* and said to extend to directed ones).  A k-vertex digraph in a vertex    */
/* order is coded with two bits per pair t < i: bit 2 p(t,i) = arc t -> i,  */
/* bit 2 p(t,i) + 1 = arc i -> t, p(t,i) = i(i-1)/2 + t.  Its class is the  */
/* minimum code over all k! vertex orders; classes are the weakly connected */
/* ones, numbered by increasing minimum code.  k <= 5 (20-bit codes).       */
/* ====================================================================== */

#define OR_MAX_DMOTIF_K 5

static uint32_t dcode_from_arcs(int k, const unsigned char arc[OR_MAXK][OR_MAXK]) {
    uint32_t c = 0;
    for (int i = 1; i < k; ++i)
        for (int t = 0; t < i; ++t) {
            if (arc[t][i]) c |= 1u << (2 * pair_bit(t, i));
            if (arc[i][t]) c |= 1u << (2 * pair_bit(t, i) + 1);
        }
    return c;
}

static void arcs_from_dcode(int k, uint32_t c, unsigned char arc[OR_MAXK][OR_MAXK]) {
    memset(arc, 0, sizeof(unsigned char) * OR_MAXK * OR_MAXK);
    for (int i = 1; i < k; ++i)
        for (int t = 0; t < i; ++t) {
            if (c >> (2 * pair_bit(t, i)) & 1u) arc[t][i] = 1;
            if (c >> (2 * pair_bit(t, i) + 1) & 1u) arc[i][t] = 1;
        }
}

/* weakly connected: connected after forgetting directions */
static int weakly_connected_dcode(int k, uint32_t c) {
    unsigned char arc[OR_MAXK][OR_MAXK];
    arcs_from_dcode(k, c, arc);
    int seen[OR_MAXK] = {0}, stack[OR_MAXK], sp = 0, cnt = 1;
    seen[0] = 1;
    stack[sp++] = 0;
    while (sp) {
        int x = stack[--sp];
        for (int y = 0; y < k; ++y)
            if ((arc[x][y] || arc[y][x]) && !seen[y]) { seen[y] = 1; cnt++; stack[sp++] = y; }
    }
    return cnt == k;
}

/* minimum code over all k! vertex orders (new position p[x] for old vertex x) */
uint32_t or_dcanon(int k, uint32_t c) {
    unsigned char arc[OR_MAXK][OR_MAXK];
    arcs_from_dcode(k, c, arc);
    int ax[OR_MAXK * OR_MAXK], ay[OR_MAXK * OR_MAXK], na = 0;
    for (int x = 0; x < k; ++x)
        for (int y = 0; y < k; ++y)
            if (arc[x][y]) { ax[na] = x; ay[na] = y; ++na; }
    int p[OR_MAXK];
    for (int i = 0; i < k; ++i) p[i] = i;
    uint32_t best = 0xffffffffu;
    do {
        /* the arc x -> y becomes p[x] -> p[y] */
        uint32_t d = 0;
        for (int e = 0; e < na; ++e) {
            const int a = p[ax[e]], b = p[ay[e]];
            d |= a < b ? 1u << (2 * pair_bit(a, b)) : 1u << (2 * pair_bit(b, a) + 1);
        }
        if (d < best) best = d;
    } while (next_perm(p, k));
    return best;
}

typedef struct {
    int ready;
    int ncls;
    uint32_t* canon;       /* [ncls] minimum codes, ascending */
    int32_t* class_of;     /* [4^C(k,2)] class id of every code, -1 if not weakly connected */
} dclass_info;

static dclass_info g_dcls[OR_MAX_DMOTIF_K + 1];

/* Every code's minimum by brute force over the k! orders (memoised per
 * code), then the connected minima sorted. */
static const dclass_info* dclasses(int k) {
    if (k < 1 || k > OR_MAX_DMOTIF_K) return NULL;
    pthread_mutex_lock(&g_cls_lock);
    dclass_info* D = &g_dcls[k];
    if (!D->ready) {
        const int bits = k * (k - 1);
        const int64_t ncodes = (int64_t)1 << bits;
        uint32_t* mins = (uint32_t*)malloc(sizeof(uint32_t) * (size_t)ncodes);
        D->class_of = (int32_t*)malloc(sizeof(int32_t) * (size_t)ncodes);
        uint32_t* reps = (uint32_t*)malloc(sizeof(uint32_t) * (size_t)ncodes);
        int64_t nrep = 0;
        for (int64_t c = 0; c < ncodes; ++c) {
            mins[c] = or_dcanon(k, (uint32_t)c);
            if (mins[c] == (uint32_t)c && weakly_connected_dcode(k, (uint32_t)c)) reps[nrep++] = (uint32_t)c;
        }
        /* reps are already ascending (c runs upwards) */
        D->ncls = (int)nrep;
        D->canon = (uint32_t*)malloc(sizeof(uint32_t) * (size_t)(nrep > 0 ? nrep : 1));
        memcpy(D->canon, reps, sizeof(uint32_t) * (size_t)nrep);
        for (int64_t c = 0; c < ncodes; ++c) {
            D->class_of[c] = -1;
            if (!weakly_connected_dcode(k, (uint32_t)c)) continue;
            int64_t lo = 0, hi = nrep;
            while (lo < hi) {
                int64_t mid = (lo + hi) / 2;
                if (reps[mid] < mins[c]) lo = mid + 1; else hi = mid;
            }
            D->class_of[c] = (int32_t)lo;
        }
        free(mins);
        free(reps);
        D->ready = 1;
    }
    pthread_mutex_unlock(&g_cls_lock);
    return D;
}

int or_dnum_classes(int k) {
    const dclass_info* D = dclasses(k);
    return D ? D->ncls : -1;
}

int or_dclass_canon(int k, uint32_t* out, int cap) {
    const dclass_info* D = dclasses(k);
    if (!D || cap < D->ncls) return -1;
    memcpy(out, D->canon, sizeof(uint32_t) * (size_t)D->ncls);
    return D->ncls;
}

int or_dclass_of_code(int k, uint32_t code) {
    const dclass_info* D = dclasses(k);
    if (!D || (uint64_t)code >> (k * (k - 1))) return -2;
    return D->class_of[code];
}

/* number of labelled weakly connected digraphs on k vertices */
int64_t or_dnum_connected_labelled(int k) {
    const dclass_info* D = dclasses(k);
    if (!D) return -1;
    int64_t cnt = 0;
    for (int64_t c = 0; c < ((int64_t)1 << (k * (k - 1))); ++c) cnt += D->class_of[c] >= 0;
    return cnt;
}

/* L1: every k-subset of a digraph given by sorted out-lists; out_counts[ncls] */
int or_dmotif_brute(int32_t n, const int64_t* rp, const int32_t* col, int k, uint64_t* out_counts) {
    graph_t g = { n, rp, col };
    const dclass_info* D = dclasses(k);
    if (!D || k < 2) return -1;
    memset(out_counts, 0, sizeof(uint64_t) * (size_t)D->ncls);
    if (k > n) return 0;
    int idx[OR_MAXK];
    for (int i = 0; i < k; ++i) idx[i] = i;
    unsigned char arc[OR_MAXK][OR_MAXK];
    for (;;) {
        memset(arc, 0, sizeof arc);
        for (int a = 0; a < k; ++a)
            for (int b = 0; b < k; ++b)
                if (a != b && has_edge(&g, idx[a], idx[b])) arc[a][b] = 1;
        int q = D->class_of[dcode_from_arcs(k, arc)];
        if (q >= 0) out_counts[q]++;
        int i = k - 1;
        while (i >= 0 && idx[i] == n - k + i) --i;
        if (i < 0) break;
        idx[i]++;
        for (int j = i + 1; j < k; ++j) idx[j] = idx[j - 1] + 1;
    }
    return 0;
}

/* L2: ESU (Wernicke's enumeration of connected k-subsets: a subset grows by
 * a vertex of its extension set; a new vertex w adds to the extension set its
 * neighbours above the root that are neither in the subset nor adjacent to
 * it), over the underlying undirected graph, each subset classified by its
 * arcs.  Threads take roots from a shared counter. */
typedef struct {
    graph_t out;           /* arcs */
    const int64_t* urp;    /* underlying undirected graph, sorted */
    const int32_t* ucol;
    int k;
    const dclass_info* D;
    int64_t next;
    int32_t n;
    pthread_mutex_t lock;
    uint64_t* total;       /* [ncls] */
} desu_job;

static int u_adjacent(const desu_job* J, int32_t a, int32_t b) {
    int64_t lo = J->urp[a], hi = J->urp[a + 1];
    while (lo < hi) {
        int64_t mid = (lo + hi) / 2;
        if (J->ucol[mid] == b) return 1;
        if (J->ucol[mid] < b) lo = mid + 1; else hi = mid;
    }
    return 0;
}

static void desu_extend(const desu_job* J, int32_t* sub, int s, int32_t* ext, int64_t ne, uint64_t* cnt) {
    if (s == J->k) {
        unsigned char arc[OR_MAXK][OR_MAXK];
        memset(arc, 0, sizeof arc);
        for (int a = 0; a < s; ++a)
            for (int b = 0; b < s; ++b)
                if (a != b && has_edge(&J->out, sub[a], sub[b])) arc[a][b] = 1;
        int q = J->D->class_of[dcode_from_arcs(s, arc)];
        if (q >= 0) cnt[q]++;
        return;
    }
    const int32_t v = sub[0];
    while (ne > 0) {
        const int32_t w = ext[--ne];
        /* new extension set: what is left of ext plus w's exclusive neighbours */
        int64_t cap = ne + (J->urp[w + 1] - J->urp[w]);
        int32_t* nx = (int32_t*)malloc(sizeof(int32_t) * (size_t)(cap > 0 ? cap : 1));
        int64_t nn = 0;
        for (int64_t i = 0; i < ne; ++i) nx[nn++] = ext[i];
        for (int64_t e = J->urp[w]; e < J->urp[w + 1]; ++e) {
            const int32_t u = J->ucol[e];
            if (u <= v) continue;
            int excl = 1;
            for (int a = 0; a < s && excl; ++a)
                if (sub[a] == u || u_adjacent(J, sub[a], u)) excl = 0;
            for (int64_t i = 0; i < nn && excl; ++i)
                if (nx[i] == u) excl = 0;
            if (excl) nx[nn++] = u;
        }
        sub[s] = w;
        desu_extend(J, sub, s + 1, nx, nn, cnt);
        free(nx);
    }
}

static void* desu_worker(void* arg) {
    desu_job* J = (desu_job*)arg;
    uint64_t* cnt = (uint64_t*)calloc((size_t)J->D->ncls, sizeof(uint64_t));
    int32_t sub[OR_MAXK];
    for (;;) {
        pthread_mutex_lock(&J->lock);
        int64_t v = J->next++;
        pthread_mutex_unlock(&J->lock);
        if (v >= J->n) break;
        int64_t d = J->urp[v + 1] - J->urp[v];
        int32_t* ext = (int32_t*)malloc(sizeof(int32_t) * (size_t)(d > 0 ? d : 1));
        int64_t ne = 0;
        for (int64_t e = J->urp[v]; e < J->urp[v + 1]; ++e)
            if (J->ucol[e] > v) ext[ne++] = J->ucol[e];
        sub[0] = (int32_t)v;
        if (J->k == 1) cnt[J->D->class_of[0]]++;
        else desu_extend(J, sub, 1, ext, ne, cnt);
        free(ext);
    }
    pthread_mutex_lock(&J->lock);
    for (int c = 0; c < J->D->ncls; ++c) J->total[c] += cnt[c];
    pthread_mutex_unlock(&J->lock);
    free(cnt);
    return NULL;
}

/* rp/col: the arcs (sorted out-lists); urp/ucol: the underlying undirected
 * graph (sorted, symmetric), built by the caller */
int or_dmotif_esu(int32_t n, const int64_t* rp, const int32_t* col, const int64_t* urp, const int32_t* ucol, int k,
                  int nthreads, uint64_t* out_counts) {
    const dclass_info* D = dclasses(k);
    if (!D || k < 2) return -1;
    memset(out_counts, 0, sizeof(uint64_t) * (size_t)D->ncls);
    desu_job J;
    J.out.n = n; J.out.rp = rp; J.out.col = col;
    J.urp = urp; J.ucol = ucol; J.k = k; J.D = D; J.next = 0; J.n = n; J.total = out_counts;
    pthread_mutex_init(&J.lock, NULL);
    if (nthreads < 1) nthreads = 1;
    pthread_t th[64];
    if (nthreads > 64) nthreads = 64;
    for (int t = 0; t < nthreads; ++t) pthread_create(&th[t], NULL, desu_worker, &J);
    for (int t = 0; t < nthreads; ++t) pthread_join(th[t], NULL);
    pthread_mutex_destroy(&J.lock);
    return 0;
}

/* the class of every directed code on k vertices (-1: not weakly connected) */
int or_dclass_table(int k, int32_t* out, int64_t len) {
    const dclass_info* D = dclasses(k);
    if (!D || len < ((int64_t)1 << (k * (k - 1)))) return -1;
    memcpy(out, D->class_of, sizeof(int32_t) * (size_t)((int64_t)1 << (k * (k - 1))));
    return 0;
}
