/*
 * graphgen.c -- seeded synthetic graph generators (input side only).
 *
 * This file produces the synthetic stand-in graphs the estimator is run on:
 * random geometric graphs with independent edge thinning (road-like), and
 * Chung-Lu graphs with given expected degrees (social / power-law).  It also
 * canonicalises an undirected edge list into a CSR adjacency with ascending
 * rows, no self-loops and no duplicate entries.
 *
 * Nothing here computes any part of the Kemeny-constant method.  Both the
 * CPU oracle and the GPU library consume the CSR this file writes.
 *
 * Randomness: xoshiro256** seeded through splitmix64 (Blackman & Vigna).
 * Chung-Lu edges follow the skipping algorithm of Miller & Hagberg,
 * "Efficient generation of networks with given expected degrees" (WAW 2011):
 * vertices are sorted by weight, and for each u the candidates v > u are
 * visited by geometric skips with the current upper bound on p_uv.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

typedef struct { uint64_t s[4]; } rng_t;

static uint64_t splitmix64(uint64_t *x) {
    uint64_t z = (*x += 0x9E3779B97F4A7C15ULL);
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ULL;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBULL;
    return z ^ (z >> 31);
}

static void rng_seed(rng_t *r, uint64_t seed) {
    uint64_t x = seed;
    for (int i = 0; i < 4; ++i) r->s[i] = splitmix64(&x);
}

static inline uint64_t rotl(uint64_t x, int k) { return (x << k) | (x >> (64 - k)); }

static inline uint64_t rng_next(rng_t *r) {
    uint64_t *s = r->s;
    uint64_t result = rotl(s[1] * 5, 7) * 9;
    uint64_t t = s[1] << 17;
    s[2] ^= s[0]; s[3] ^= s[1]; s[1] ^= s[2]; s[0] ^= s[3];
    s[2] ^= t; s[3] = rotl(s[3], 45);
    return result;
}

/* uniform double in (0, 1] (never 0, so log() is finite) */
static inline double rng_unit(rng_t *r) {
    return ((double)(rng_next(r) >> 11) + 1.0) * (1.0 / 9007199254740992.0);
}

/* stateless hash of an unordered pair, for order-independent edge thinning */
static inline double pair_unit(uint64_t seed, uint64_t a, uint64_t b) {
    uint64_t x = seed ^ (a * 0xD6E8FEB86659FD93ULL) ^ (b * 0x9E3779B97F4A7C15ULL);
    uint64_t z = splitmix64(&x);
    z = splitmix64(&z);
    return ((double)(z >> 11) + 0.5) * (1.0 / 9007199254740992.0);
}

static int cmp_i32(const void *a, const void *b) {
    int32_t x = *(const int32_t *)a, y = *(const int32_t *)b;
    return (x > y) - (x < y);
}

/*
 * Canonical CSR from an undirected edge list.  offsets has n+1 slots;
 * indices must hold 2*m entries.  Returns the number of directed entries
 * kept (2 * number of distinct undirected non-loop edges).
 */
int64_t gg_build_csr(int64_t n, int64_t m, const int32_t *eu, const int32_t *ev,
                     int64_t *offsets, int32_t *indices) {
    int64_t *cur = (int64_t *)calloc((size_t)n + 1, sizeof(int64_t));
    if (!cur) return -1;
    memset(offsets, 0, sizeof(int64_t) * (size_t)(n + 1));
    for (int64_t e = 0; e < m; ++e) {
        int32_t u = eu[e], v = ev[e];
        if (u == v) continue;
        offsets[u + 1]++;
        offsets[v + 1]++;
    }
    for (int64_t i = 0; i < n; ++i) offsets[i + 1] += offsets[i];
    for (int64_t i = 0; i <= n; ++i) cur[i] = offsets[i];
    for (int64_t e = 0; e < m; ++e) {
        int32_t u = eu[e], v = ev[e];
        if (u == v) continue;
        indices[cur[u]++] = v;
        indices[cur[v]++] = u;
    }
    /* sort each row and drop duplicates, compacting in place */
    int64_t w = 0;
    int64_t row_start = offsets[0];
    for (int64_t i = 0; i < n; ++i) {
        int64_t a = row_start, b = offsets[i + 1];
        row_start = b;
        qsort(indices + a, (size_t)(b - a), sizeof(int32_t), cmp_i32);
        int64_t new_start = w;
        for (int64_t k = a; k < b; ++k) {
            if (k > a && indices[k] == indices[k - 1]) continue;
            indices[w++] = indices[k];
        }
        offsets[i] = new_start;
    }
    offsets[n] = w;
    free(cur);
    return w;
}

/*
 * Random geometric graph on npts uniform points of the unit square, radius
 * `radius`; every geometric edge is then kept independently with
 * probability keep_q.  Points are relabelled in row-major cell order so that
 * vertex ids have spatial locality.  Writes up to cap edges; returns the
 * number of edges, or -(needed) if cap was too small.
 */
int64_t gg_rgg_edges(int64_t npts, double radius, double keep_q, uint64_t seed,
                     int32_t *eu, int32_t *ev, int64_t cap) {
    rng_t r;
    rng_seed(&r, seed);
    double *x = (double *)malloc(sizeof(double) * (size_t)npts);
    double *y = (double *)malloc(sizeof(double) * (size_t)npts);
    for (int64_t i = 0; i < npts; ++i) {
        x[i] = (double)(rng_next(&r) >> 11) * (1.0 / 9007199254740992.0);
        y[i] = (double)(rng_next(&r) >> 11) * (1.0 / 9007199254740992.0);
    }
    int64_t g = (int64_t)floor(1.0 / radius);
    if (g < 1) g = 1;
    int64_t ncell = g * g;
    int64_t *cstart = (int64_t *)calloc((size_t)ncell + 1, sizeof(int64_t));
    int64_t *cellof = (int64_t *)malloc(sizeof(int64_t) * (size_t)npts);
    for (int64_t i = 0; i < npts; ++i) {
        int64_t cx = (int64_t)(x[i] * g), cy = (int64_t)(y[i] * g);
        if (cx >= g) cx = g - 1;
        if (cy >= g) cy = g - 1;
        cellof[i] = cy * g + cx;
        cstart[cellof[i] + 1]++;
    }
    for (int64_t c = 0; c < ncell; ++c) cstart[c + 1] += cstart[c];
    int64_t *fill = (int64_t *)malloc(sizeof(int64_t) * (size_t)ncell);
    memcpy(fill, cstart, sizeof(int64_t) * (size_t)ncell);
    double *sx = (double *)malloc(sizeof(double) * (size_t)npts);
    double *sy = (double *)malloc(sizeof(double) * (size_t)npts);
    for (int64_t i = 0; i < npts; ++i) {
        int64_t p = fill[cellof[i]]++;
        sx[p] = x[i];
        sy[p] = y[i];
    }
    free(x); free(y); free(fill); free(cellof);
    double r2 = radius * radius;
    int64_t cnt = 0;
    static const int dxs[5] = {0, 1, -1, 0, 1};
    static const int dys[5] = {0, 0, 1, 1, 1};
    for (int64_t cy = 0; cy < g; ++cy) {
        for (int64_t cx = 0; cx < g; ++cx) {
            int64_t c = cy * g + cx;
            for (int k = 0; k < 5; ++k) {
                int64_t nx = cx + dxs[k], ny = cy + dys[k];
                if (nx < 0 || nx >= g || ny >= g) continue;
                int64_t d = ny * g + nx;
                for (int64_t i = cstart[c]; i < cstart[c + 1]; ++i) {
                    int64_t j0 = (k == 0) ? i + 1 : cstart[d];
                    for (int64_t j = j0; j < cstart[d + 1]; ++j) {
                        double ddx = sx[i] - sx[j], ddy = sy[i] - sy[j];
                        if (ddx * ddx + ddy * ddy > r2) continue;
                        int64_t a = i < j ? i : j, b = i < j ? j : i;
                        if (keep_q < 1.0 && pair_unit(seed ^ 0x5A5A5A5AULL, (uint64_t)a, (uint64_t)b) >= keep_q)
                            continue;
                        if (cnt < cap) {
                            eu[cnt] = (int32_t)a;
                            ev[cnt] = (int32_t)b;
                        }
                        cnt++;
                    }
                }
            }
        }
    }
    free(sx); free(sy); free(cstart);
    return cnt <= cap ? cnt : -cnt;
}

/*
 * Chung-Lu graph: edge {u,v} (u != v) present independently with
 * probability min(1, w_u w_v / S), S = sum of weights.  w must be sorted in
 * non-increasing order.  Returns the number of edges written, or -(needed).
 */
int64_t gg_chung_lu_edges(int64_t n, const double *w, uint64_t seed,
                          int32_t *eu, int32_t *ev, int64_t cap) {
    rng_t r;
    rng_seed(&r, seed);
    double S = 0.0;
    for (int64_t i = 0; i < n; ++i) S += w[i];
    int64_t cnt = 0;
    for (int64_t u = 0; u + 1 < n; ++u) {
        int64_t v = u + 1;
        double p = w[u] * w[v] / S;
        if (p > 1.0) p = 1.0;
        while (v < n && p > 0.0) {
            if (p != 1.0) {
                double rr = rng_unit(&r);
                double skip = floor(log(rr) / log1p(-p));
                if (skip > (double)(n - v)) break;
                v += (int64_t)skip;
            }
            if (v < n) {
                double q = w[u] * w[v] / S;
                if (q > 1.0) q = 1.0;
                double rr = rng_unit(&r);
                if (rr < q / p) {
                    if (cnt < cap) {
                        eu[cnt] = (int32_t)u;
                        ev[cnt] = (int32_t)v;
                    }
                    cnt++;
                }
                p = q;
                v += 1;
            }
        }
    }
    return cnt <= cap ? cnt : -cnt;
}

/*
 * Largest connected component of a CSR graph, relabelled in original vertex
 * order (the relabelling is monotone, so rows stay ascending).  Components
 * are found by breadth-first search from each unlabelled vertex in
 * ascending order; ties between equally large components go to the one
 * holding the smallest vertex.  Writes the component's CSR into off_out
 * (n_out+1 slots) and idx_out (at most offsets[n] entries) and returns its
 * vertex count n_out (n when the graph is connected), or -1 on allocation
 * failure.
 */
int64_t gg_lcc(int64_t n, const int64_t *off, const int32_t *idx, int64_t *off_out, int32_t *idx_out) {
    int32_t *comp = (int32_t *)malloc(sizeof(int32_t) * (size_t)n);
    int32_t *queue = (int32_t *)malloc(sizeof(int32_t) * (size_t)n);
    if (!comp || !queue) { free(comp); free(queue); return -1; }
    for (int64_t v = 0; v < n; ++v) comp[v] = -1;
    int32_t ncomp = 0, best = -1;
    int64_t best_size = 0;
    for (int64_t s = 0; s < n; ++s) {
        if (comp[s] >= 0) continue;
        int64_t qh = 0, qt = 0;
        comp[s] = ncomp;
        queue[qt++] = (int32_t)s;
        while (qh < qt) {
            int32_t x = queue[qh++];
            for (int64_t e = off[x]; e < off[x + 1]; ++e) {
                int32_t y = idx[e];
                if (comp[y] < 0) { comp[y] = ncomp; queue[qt++] = y; }
            }
        }
        if (qt > best_size) { best_size = qt; best = ncomp; }
        ncomp++;
    }
    /* new id of each kept vertex, in original order */
    int32_t *newid = queue;
    int64_t k = 0;
    for (int64_t v = 0; v < n; ++v) newid[v] = comp[v] == best ? (int32_t)k++ : -1;
    int64_t w = 0;
    off_out[0] = 0;
    for (int64_t v = 0; v < n; ++v) {
        if (newid[v] < 0) continue;
        for (int64_t e = off[v]; e < off[v + 1]; ++e) idx_out[w++] = newid[idx[e]];
        off_out[newid[v] + 1] = w;
    }
    free(comp); free(queue);
    return k;
}
