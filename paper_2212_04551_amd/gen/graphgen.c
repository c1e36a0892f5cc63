/*
 * Seeded synthetic graph generators.
 *
 * This module only produces input graphs; it holds none of the enumeration
 * arithmetic.  The GPU library, the CPU oracle, the tests and the benchmark all
 * read the CSR it writes, so a graph is a pure function of (generator, params,
 * seed).
 *
 * Random numbers: xoshiro256** seeded through SplitMix64, both written from
 * Blackman & Vigna, "Scrambled linear pseudorandom number generators" (2018).
 *
 * Output format: undirected simple graph as CSR with int64 row offsets and
 * int32 column ids; every adjacency list is sorted strictly ascending, with
 * no self-loops and both directions of every edge present.  After an edge set
 * is drawn, vertex ids are shuffled by a seeded Fisher-Yates permutation so
 * that id order carries no degree or block information.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

typedef struct {
    int32_t n;
    int64_t nnz;
    int64_t* row_ptr;  /* n+1 */
    int32_t* col;      /* nnz */
} gg_csr;

/* ---------------- PRNG ---------------- */

typedef struct { uint64_t s[4]; } rng_t;

static uint64_t splitmix64_next(uint64_t* x) {
    uint64_t z = (*x += 0x9e3779b97f4a7c15ULL);
    z = (z ^ (z >> 30)) * 0xbf58476d1ce4e5b9ULL;
    z = (z ^ (z >> 27)) * 0x94d049bb133111ebULL;
    return z ^ (z >> 31);
}

static inline uint64_t rotl64(uint64_t x, int k) { return (x << k) | (x >> (64 - k)); }

static uint64_t rng_next(rng_t* r) {
    uint64_t* s = r->s;
    const uint64_t result = rotl64(s[1] * 5, 7) * 9;
    const uint64_t t = s[1] << 17;
    s[2] ^= s[0];
    s[3] ^= s[1];
    s[1] ^= s[2];
    s[0] ^= s[3];
    s[2] ^= t;
    s[3] = rotl64(s[3], 45);
    return result;
}

/* A stream is identified by (generator tag, seed); distinct tags never share state. */
static void rng_seed(rng_t* r, uint64_t tag, uint64_t seed) {
    uint64_t x = seed ^ (tag * 0xd1b54a32d192ed03ULL);
    for (int i = 0; i < 4; ++i) r->s[i] = splitmix64_next(&x);
}

/* uniform integer in [0, bound) by the 128-bit multiply-high map */
static inline uint64_t rng_below(rng_t* r, uint64_t bound) {
    return (uint64_t)(((__uint128_t)rng_next(r) * bound) >> 64);
}

/* uniform double in [0, 1) from the top 53 bits */
static inline double rng_unit(rng_t* r) { return (double)(rng_next(r) >> 11) * 0x1.0p-53; }

/* ---------------- edge set (open addressing) ---------------- */

typedef struct {
    uint64_t* keys;  /* 0 = empty; stored key = pair code + 1 */
    uint64_t mask;
    int64_t count;
} edge_set;

static int es_init(edge_set* h, int64_t expected) {
    uint64_t cap = 16;
    while (cap < (uint64_t)(expected * 2 + 16)) cap <<= 1;
    h->keys = (uint64_t*)calloc(cap, sizeof(uint64_t));
    h->mask = cap - 1;
    h->count = 0;
    return h->keys ? 0 : -1;
}

static inline uint64_t mix64(uint64_t z) {
    z = (z ^ (z >> 30)) * 0xbf58476d1ce4e5b9ULL;
    z = (z ^ (z >> 27)) * 0x94d049bb133111ebULL;
    return z ^ (z >> 31);
}

/* returns 1 if inserted, 0 if already present */
static int es_insert(edge_set* h, uint64_t code) {
    uint64_t key = code + 1;
    uint64_t i = mix64(key) & h->mask;
    for (;;) {
        uint64_t k = h->keys[i];
        if (k == 0) { h->keys[i] = key; h->count++; return 1; }
        if (k == key) return 0;
        i = (i + 1) & h->mask;
    }
}

/* ---------------- edge list -> CSR ---------------- */

typedef struct {
    int32_t* u;
    int32_t* v;
    int64_t m;
    int64_t cap;
} edge_list;

static int el_init(edge_list* e, int64_t cap) {
    e->u = (int32_t*)malloc(sizeof(int32_t) * (size_t)(cap > 0 ? cap : 1));
    e->v = (int32_t*)malloc(sizeof(int32_t) * (size_t)(cap > 0 ? cap : 1));
    e->m = 0;
    e->cap = cap;
    return (e->u && e->v) ? 0 : -1;
}

static int el_push(edge_list* e, int32_t a, int32_t b) {
    if (e->m == e->cap) {
        int64_t nc = e->cap * 2 + 16;
        int32_t* nu = (int32_t*)realloc(e->u, sizeof(int32_t) * (size_t)nc);
        if (!nu) return -1;
        e->u = nu;
        int32_t* nv = (int32_t*)realloc(e->v, sizeof(int32_t) * (size_t)nc);
        if (!nv) return -1;
        e->v = nv;
        e->cap = nc;
    }
    e->u[e->m] = a;
    e->v[e->m] = b;
    e->m++;
    return 0;
}

static void el_free(edge_list* e) { free(e->u); free(e->v); }

/*
 * Shuffle ids with a seeded permutation, then build the sorted CSR with two
 * stable counting sorts (by destination, then by source).
 */
static gg_csr* build_csr(int32_t n, edge_list* e, rng_t* r) {
    gg_csr* g = (gg_csr*)calloc(1, sizeof(gg_csr));
    if (!g) return NULL;
    int32_t* perm = (int32_t*)malloc(sizeof(int32_t) * (size_t)(n > 0 ? n : 1));
    for (int32_t i = 0; i < n; ++i) perm[i] = i;
    for (int32_t i = n - 1; i > 0; --i) {
        int32_t j = (int32_t)rng_below(r, (uint64_t)i + 1);
        int32_t t = perm[i]; perm[i] = perm[j]; perm[j] = t;
    }
    int64_t arcs = 2 * e->m;
    int32_t* src = (int32_t*)malloc(sizeof(int32_t) * (size_t)(arcs > 0 ? arcs : 1));
    int32_t* dst = (int32_t*)malloc(sizeof(int32_t) * (size_t)(arcs > 0 ? arcs : 1));
    int32_t* tsrc = (int32_t*)malloc(sizeof(int32_t) * (size_t)(arcs > 0 ? arcs : 1));
    int32_t* tdst = (int32_t*)malloc(sizeof(int32_t) * (size_t)(arcs > 0 ? arcs : 1));
    int64_t* cnt = (int64_t*)calloc((size_t)n + 1, sizeof(int64_t));
    for (int64_t i = 0; i < e->m; ++i) {
        int32_t a = perm[e->u[i]], b = perm[e->v[i]];
        src[2 * i] = a; dst[2 * i] = b;
        src[2 * i + 1] = b; dst[2 * i + 1] = a;
    }
    free(perm);
    /* pass 1: stable counting sort by dst into t* */
    memset(cnt, 0, sizeof(int64_t) * ((size_t)n + 1));
    for (int64_t i = 0; i < arcs; ++i) cnt[dst[i] + 1]++;
    for (int32_t i = 0; i < n; ++i) cnt[i + 1] += cnt[i];
    for (int64_t i = 0; i < arcs; ++i) {
        int64_t p = cnt[dst[i]]++;
        tsrc[p] = src[i]; tdst[p] = dst[i];
    }
    /* pass 2: stable counting sort by src back into dst-array order */
    memset(cnt, 0, sizeof(int64_t) * ((size_t)n + 1));
    for (int64_t i = 0; i < arcs; ++i) cnt[tsrc[i] + 1]++;
    for (int32_t i = 0; i < n; ++i) cnt[i + 1] += cnt[i];
    g->row_ptr = (int64_t*)malloc(sizeof(int64_t) * ((size_t)n + 1));
    memcpy(g->row_ptr, cnt, sizeof(int64_t) * ((size_t)n + 1));
    g->col = (int32_t*)malloc(sizeof(int32_t) * (size_t)(arcs > 0 ? arcs : 1));
    for (int64_t i = 0; i < arcs; ++i) {
        int64_t p = cnt[tsrc[i]]++;
        g->col[p] = tdst[i];
    }
    free(src); free(dst); free(tsrc); free(tdst); free(cnt);
    g->n = n;
    g->nnz = arcs;
    return g;
}

void gg_free(gg_csr* g) {
    if (!g) return;
    free(g->row_ptr);
    free(g->col);
    free(g);
}

enum { TAG_ER = 1, TAG_CL = 2, TAG_BA = 3, TAG_SBM = 4 };

/* ---------------- G(n, m): uniform distinct pairs ---------------- */

gg_csr* gg_erdos_renyi(int32_t n, int64_t m, uint64_t seed) {
    if (n < 0 || m < 0) return NULL;
    int64_t maxm = (int64_t)n * (n - 1) / 2;
    if (m > maxm) m = maxm;
    rng_t r;
    rng_seed(&r, TAG_ER, seed);
    edge_set h;
    edge_list e;
    if (es_init(&h, m) || el_init(&e, m)) return NULL;
    while (e.m < m) {
        int32_t a = (int32_t)rng_below(&r, (uint64_t)n);
        int32_t b = (int32_t)rng_below(&r, (uint64_t)n);
        if (a == b) continue;
        int32_t lo = a < b ? a : b, hi = a < b ? b : a;
        if (es_insert(&h, (uint64_t)lo * (uint64_t)n + (uint64_t)hi)) el_push(&e, lo, hi);
    }
    free(h.keys);
    gg_csr* g = build_csr(n, &e, &r);
    el_free(&e);
    return g;
}

/* ---------------- Chung-Lu with a power-law weight sequence ---------------- */

/* w_i = wmax * ((i + i0) / i0)^(-1/(gamma-1)); mean over i is increasing in i0 */
static double cl_mean(int32_t n, double gamma, double wmax, double i0) {
    double a = -1.0 / (gamma - 1.0), s = 0.0;
    for (int32_t i = 0; i < n; ++i) s += wmax * pow(((double)i + i0) / i0, a);
    return s / (double)n;
}

gg_csr* gg_chung_lu(int32_t n, int64_t m, double gamma, double wmax, uint64_t seed,
                    double* i0_out) {
    if (n < 2 || m < 0 || gamma <= 1.0 || wmax <= 0.0) return NULL;
    double target = 2.0 * (double)m / (double)n;
    if (target >= wmax) return NULL;
    double lo = 1e-9, hi = 1e12;
    for (int it = 0; it < 200; ++it) {
        double mid = sqrt(lo * hi);
        if (cl_mean(n, gamma, wmax, mid) < target) lo = mid; else hi = mid;
    }
    double i0 = sqrt(lo * hi);
    if (i0_out) *i0_out = i0;
    /* Vose alias table over the weights */
    double* prob = (double*)malloc(sizeof(double) * (size_t)n);
    int32_t* alias = (int32_t*)malloc(sizeof(int32_t) * (size_t)n);
    int32_t* small = (int32_t*)malloc(sizeof(int32_t) * (size_t)n);
    int32_t* large = (int32_t*)malloc(sizeof(int32_t) * (size_t)n);
    double a = -1.0 / (gamma - 1.0), tot = 0.0;
    for (int32_t i = 0; i < n; ++i) { prob[i] = wmax * pow(((double)i + i0) / i0, a); tot += prob[i]; }
    int32_t ns = 0, nl = 0;
    for (int32_t i = 0; i < n; ++i) {
        prob[i] = prob[i] * (double)n / tot;
        if (prob[i] < 1.0) small[ns++] = i; else large[nl++] = i;
    }
    while (ns > 0 && nl > 0) {
        int32_t s = small[--ns], l = large[--nl];
        alias[s] = l;
        prob[l] = (prob[l] + prob[s]) - 1.0;
        if (prob[l] < 1.0) small[ns++] = l; else large[nl++] = l;
    }
    while (nl > 0) { int32_t l = large[--nl]; prob[l] = 1.0; alias[l] = l; }
    while (ns > 0) { int32_t s = small[--ns]; prob[s] = 1.0; alias[s] = s; }
    free(small); free(large);

    rng_t r;
    rng_seed(&r, TAG_CL, seed);
    edge_set h;
    edge_list e;
    if (es_init(&h, m) || el_init(&e, m)) return NULL;
    int64_t maxm = (int64_t)n * (n - 1) / 2;
    if (m > maxm) m = maxm;
    while (e.m < m) {
        int32_t x = (int32_t)rng_below(&r, (uint64_t)n);
        int32_t u = rng_unit(&r) < prob[x] ? x : alias[x];
        int32_t y = (int32_t)rng_below(&r, (uint64_t)n);
        int32_t v = rng_unit(&r) < prob[y] ? y : alias[y];
        if (u == v) continue;
        int32_t lo2 = u < v ? u : v, hi2 = u < v ? v : u;
        if (es_insert(&h, (uint64_t)lo2 * (uint64_t)n + (uint64_t)hi2)) el_push(&e, lo2, hi2);
    }
    free(h.keys); free(prob); free(alias);
    gg_csr* g = build_csr(n, &e, &r);
    el_free(&e);
    return g;
}

/* ---------------- Barabasi-Albert (preferential attachment) ---------------- */

gg_csr* gg_barabasi_albert(int32_t n, int32_t m0, uint64_t seed) {
    if (m0 < 1 || n < m0 + 1) return NULL;
    rng_t r;
    rng_seed(&r, TAG_BA, seed);
    int64_t m = (int64_t)m0 * (m0 + 1) / 2 + (int64_t)(n - m0 - 1) * m0;
    edge_list e;
    if (el_init(&e, m)) return NULL;
    int32_t* ends = (int32_t*)malloc(sizeof(int32_t) * (size_t)(2 * m));
    int64_t ne = 0;
    for (int32_t i = 0; i <= m0; ++i)
        for (int32_t j = i + 1; j <= m0; ++j) {
            el_push(&e, i, j);
            ends[ne++] = i; ends[ne++] = j;
        }
    int32_t* pick = (int32_t*)malloc(sizeof(int32_t) * (size_t)m0);
    for (int32_t t = m0 + 1; t < n; ++t) {
        int32_t got = 0;
        while (got < m0) {
            int32_t c = ends[rng_below(&r, (uint64_t)ne)];
            int dup = 0;
            for (int32_t q = 0; q < got; ++q) if (pick[q] == c) { dup = 1; break; }
            if (!dup) pick[got++] = c;
        }
        for (int32_t q = 0; q < m0; ++q) {
            el_push(&e, pick[q], t);
            ends[ne++] = pick[q]; ends[ne++] = t;
        }
    }
    free(pick); free(ends);
    gg_csr* g = build_csr(n, &e, &r);
    el_free(&e);
    return g;
}

/* ---------------- planted-partition stochastic block model ---------------- */

gg_csr* gg_sbm(int32_t blocks, int32_t block_size, double p_in, double p_out, uint64_t seed) {
    if (blocks < 1 || block_size < 1) return NULL;
    int64_t n64 = (int64_t)blocks * block_size;
    if (n64 > 2000000000LL) return NULL;
    int32_t n = (int32_t)n64;
    rng_t r;
    rng_seed(&r, TAG_SBM, seed);
    edge_list e;
    if (el_init(&e, 1024)) return NULL;
    /*
     * Every pair (u < v) is an independent Bernoulli trial.  Runs of failures are
     * skipped geometrically (Batagelj & Brandes 2005) inside each row segment of
     * constant probability.
     */
    for (int32_t u = 0; u < n; ++u) {
        int32_t bu = u / block_size;
        int32_t seg_lo[2] = { u + 1, (bu + 1) * block_size };
        int32_t seg_hi[2] = { (bu + 1) * block_size, n };
        double seg_p[2] = { p_in, p_out };
        for (int sgi = 0; sgi < 2; ++sgi) {
            int32_t lo = seg_lo[sgi], hi = seg_hi[sgi];
            double p = seg_p[sgi];
            if (lo >= hi || p <= 0.0) continue;
            if (p >= 1.0) { for (int32_t v = lo; v < hi; ++v) el_push(&e, u, v); continue; }
            double lq = log1p(-p);
            int64_t v = (int64_t)lo - 1;
            for (;;) {
                double x = rng_unit(&r);
                v += 1 + (int64_t)floor(log1p(-x) / lq);
                if (v >= hi) break;
                el_push(&e, u, (int32_t)v);
            }
        }
    }
    gg_csr* g = build_csr(n, &e, &r);
    el_free(&e);
    return g;
}

/* ---------------- accessors for foreign-function callers ---------------- */

int32_t gg_n(const gg_csr* g) { return g->n; }
int64_t gg_nnz(const gg_csr* g) { return g->nnz; }
void gg_copy(const gg_csr* g, int64_t* row_ptr, int32_t* col) {
    memcpy(row_ptr, g->row_ptr, sizeof(int64_t) * ((size_t)g->n + 1));
    if (g->nnz) memcpy(col, g->col, sizeof(int32_t) * (size_t)g->nnz);
}

/* FNV-1a 64 over n (int64 LE), row_ptr (int64 LE) and col (int32 LE) */
uint64_t gg_fnv1a64(int32_t n, const int64_t* row_ptr, const int32_t* col) {
    uint64_t h = 0xcbf29ce484222325ULL;
    const uint64_t P = 0x100000001b3ULL;
    int64_t nn = n;
    const unsigned char* p = (const unsigned char*)&nn;
    for (int i = 0; i < 8; ++i) { h ^= p[i]; h *= P; }
    p = (const unsigned char*)row_ptr;
    for (size_t i = 0; i < 8 * ((size_t)n + 1); ++i) { h ^= p[i]; h *= P; }
    p = (const unsigned char*)col;
    for (size_t i = 0; i < 4 * (size_t)row_ptr[n]; ++i) { h ^= p[i]; h *= P; }
    return h;
}

/*
 * Parameters of graph i of the uneven-batch workload: n uniform in [nlo, nhi];
 * an even i is G(n, round(n*d/2)) with d uniform in [dlo, dhi); an odd i is
 * preferential attachment with m0 uniform in [mlo, mhi].
 */
void gg_batch_params(uint64_t i, int32_t nlo, int32_t nhi, double dlo, double dhi,
                     int32_t mlo, int32_t mhi, int32_t* n, int64_t* m, int32_t* m0) {
    rng_t r;
    rng_seed(&r, 5, i);
    *n = nlo + (int32_t)rng_below(&r, (uint64_t)(nhi - nlo + 1));
    double d = dlo + (dhi - dlo) * rng_unit(&r);
    *m = (int64_t)llround((double)(*n) * d / 2.0);
    *m0 = mlo + (int32_t)rng_below(&r, (uint64_t)(mhi - mlo + 1));
}
