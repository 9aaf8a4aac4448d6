/*
 * Seeded synthetic bipartite edge lists (inputs only; no counting here).
 *
 * Random stream: SplitMix64 (Steele, Lea, Flood, "Fast splittable
 * pseudorandom number generators", OOPSLA 2014) from the 64-bit seed.
 * Draws:
 *   - uniform index below n: the high 64 bits of x * n for a 64-bit draw x
 *     (multiply-shift; the bias is below n / 2^64, irrelevant for inputs);
 *   - weighted index: Walker's alias method on the given weights, one draw
 *     picks the column (multiply-shift) and one the coin (top 53 bits).
 * Pairs (l, r) are drawn until m distinct ones exist; the first m distinct
 * pairs in draw order are kept (an open-addressing set of l * n_right + r).
 * Optionally both sides' ids are then relabelled by Fisher-Yates
 * permutations drawn from the same stream.
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

typedef struct { uint64_t s; } sm64_t;

static inline uint64_t sm64_next(sm64_t *g) {
    uint64_t z = (g->s += 0x9E3779B97F4A7C15ull);
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}

static inline uint64_t below(sm64_t *g, uint64_t n) {
    return (uint64_t)(((unsigned __int128)sm64_next(g) * n) >> 64);
}

static inline double unit(sm64_t *g) { return (double)(sm64_next(g) >> 11) * 0x1.0p-53; }

typedef struct { double *prob; uint32_t *alias; uint32_t n; } alias_t;

/* Vose's construction of Walker's alias table. */
static int alias_build(alias_t *a, const double *w, uint32_t n) {
    a->n = n;
    a->prob = (double *)malloc(sizeof(double) * (n ? n : 1));
    a->alias = (uint32_t *)malloc(sizeof(uint32_t) * (n ? n : 1));
    uint32_t *small = (uint32_t *)malloc(sizeof(uint32_t) * (n ? n : 1));
    uint32_t *large = (uint32_t *)malloc(sizeof(uint32_t) * (n ? n : 1));
    double *p = (double *)malloc(sizeof(double) * (n ? n : 1));
    if (!a->prob || !a->alias || !small || !large || !p) return -1;
    double tot = 0;
    for (uint32_t i = 0; i < n; i++) tot += w[i];
    uint32_t ns = 0, nl = 0;
    for (uint32_t i = 0; i < n; i++) {
        p[i] = w[i] * n / tot;
        if (p[i] < 1.0) small[ns++] = i; else large[nl++] = i;
    }
    while (ns && nl) {
        uint32_t s = small[--ns], l = large[--nl];
        a->prob[s] = p[s];
        a->alias[s] = l;
        p[l] = (p[l] + p[s]) - 1.0;
        if (p[l] < 1.0) small[ns++] = l; else large[nl++] = l;
    }
    while (nl) { uint32_t l = large[--nl]; a->prob[l] = 1.0; a->alias[l] = l; }
    while (ns) { uint32_t s = small[--ns]; a->prob[s] = 1.0; a->alias[s] = s; }
    free(small); free(large); free(p);
    return 0;
}

static inline uint32_t alias_draw(const alias_t *a, sm64_t *g) {
    uint32_t c = (uint32_t)below(g, a->n);
    return unit(g) < a->prob[c] ? c : a->alias[c];
}

static void alias_free(alias_t *a) { free(a->prob); free(a->alias); }

static inline uint64_t mix(uint64_t k) {
    k ^= k >> 33; k *= 0xff51afd7ed558ccdull; k ^= k >> 33; k *= 0xc4ceb9fe1a85ec53ull;
    return k ^ (k >> 33);
}

/* Shared driver: wl/wr NULL = uniform side.  Returns 0, -1 (memory) or -2
 * (cannot find m distinct pairs within 64 m draws). */
static int draw_edges(uint32_t nl, uint32_t nr, uint64_t m, const double *wl, const double *wr,
                      uint64_t seed, int permute, uint32_t *out_l, uint32_t *out_r) {
    sm64_t g = {seed};
    alias_t al = {0}, ar = {0};
    if (wl && alias_build(&al, wl, nl)) return -1;
    if (wr && alias_build(&ar, wr, nr)) return -1;
    uint64_t cap = 1;
    while (cap < 2 * m + 16) cap <<= 1;
    uint64_t *set = (uint64_t *)malloc(cap * sizeof(uint64_t));
    if (!set) return -1;
    memset(set, 0xFF, cap * sizeof(uint64_t));
    uint64_t have = 0, draws = 0;
    while (have < m) {
        if (draws++ > 64 * m + 1000000) { free(set); alias_free(&al); alias_free(&ar); return -2; }
        uint32_t l = wl ? alias_draw(&al, &g) : (uint32_t)below(&g, nl);
        uint32_t r = wr ? alias_draw(&ar, &g) : (uint32_t)below(&g, nr);
        uint64_t key = (uint64_t)l * nr + r;
        uint64_t h = mix(key) & (cap - 1);
        for (;;) {
            if (set[h] == UINT64_MAX) {
                set[h] = key;
                out_l[have] = l;
                out_r[have] = r;
                have++;
                break;
            }
            if (set[h] == key) break;
            h = (h + 1) & (cap - 1);
        }
    }
    free(set);
    alias_free(&al);
    alias_free(&ar);
    if (permute) {
        uint32_t *pl = (uint32_t *)malloc(sizeof(uint32_t) * (nl ? nl : 1));
        uint32_t *pr = (uint32_t *)malloc(sizeof(uint32_t) * (nr ? nr : 1));
        if (!pl || !pr) { free(pl); free(pr); return -1; }
        for (uint32_t i = 0; i < nl; i++) pl[i] = i;
        for (uint32_t i = 0; i < nr; i++) pr[i] = i;
        for (uint32_t i = nl; i > 1; i--) { uint32_t j = (uint32_t)below(&g, i); uint32_t t = pl[i - 1]; pl[i - 1] = pl[j]; pl[j] = t; }
        for (uint32_t i = nr; i > 1; i--) { uint32_t j = (uint32_t)below(&g, i); uint32_t t = pr[i - 1]; pr[i - 1] = pr[j]; pr[j] = t; }
        for (uint64_t i = 0; i < m; i++) { out_l[i] = pl[out_l[i]]; out_r[i] = pr[out_r[i]]; }
        free(pl); free(pr);
    }
    return 0;
}

int gen_er(uint32_t nl, uint32_t nr, uint64_t m, uint64_t seed, uint32_t *l, uint32_t *r) {
    if ((uint64_t)nl * nr < m) return -3;
    return draw_edges(nl, nr, m, NULL, NULL, seed, 0, l, r);
}

int gen_weighted(uint32_t nl, uint32_t nr, uint64_t m, const double *wl, const double *wr,
                 uint64_t seed, int permute, uint32_t *l, uint32_t *r) {
    return draw_edges(nl, nr, m, wl, wr, seed, permute, l, r);
}
