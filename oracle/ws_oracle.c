/*
 * ws_oracle.c -- TEST INFRASTRUCTURE ONLY.
 *
 * A plain, sequential, deliberately slow CPU implementation of what the
 * watershed / waterfall hot path computes, written from "Parallel Watershed
 * Partitioning: GPU-Based Hierarchical Image Segmentation" (arXiv 2410.08946).
 * Only the tests, the smoke check and the benchmark's CPU-baseline leg may load
 * it. The HIP library never includes, links or calls anything in this file, and
 * this file includes nothing from the HIP library.
 *
 * Conventions
 *   - Pixels are indexed linearly, p = x + nx*(y + ny*z) (row-major order, the
 *     fixed pixel order required by Step I, Section 3.1).
 *   - N(p): in-image pixels at unit distance. conn 4/6 = von Neumann, 8/26 =
 *     Moore (Section 3.1, definition of the neighbourhood). Out-of-image
 *     positions are not neighbours; a pixel with no neighbour is a strict
 *     local minimum (state 1).
 *   - Grey values are passed as uint16 (uint8 images are widened exactly).
 *   - Floating point is double throughout (gradient pre-processing).
 *
 * Readings where the paper is silent (each is listed in the design notes):
 *   - Step II picks, among the qualifying neighbours q of p (state 0, same
 *     grey value, at the start of the sweep), the one with the smallest
 *     linear index. The paper only requires that such a q exists.
 *   - The final label of a basin is the smallest linear index in the basin
 *     (canonical label); the paper leaves the set representative free.
 *   - The waterfall level is the graph waterfall: every region merges along
 *     its lowest boundary pass (Alg. 4, Step V height), ties broken by the
 *     smaller neighbouring label; merged regions take the smallest label.
 *   - Gradient: separable Gaussian blur with radius floor(4*sigma + 0.5) and
 *     half-sample-symmetric ("reflect") borders, unnormalised Sobel, Euclidean
 *     magnitude, quantisation rint(mag * Q / max(mag)) (ties to even).
 *
 * Parity pins: every function below is pinned by the CPU test-suite against
 * the paper's worked examples, brute-force definitions and invariants.
 */
#include <math.h>
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

/* Progress lines on stderr after each step of a long run (off by default). */
static int or_progress = 0;
void or_set_progress(int on) { or_progress = on; }
#define OR_SAY(...)                           \
    do {                                      \
        if (or_progress) {                    \
            fprintf(stderr, __VA_ARGS__);     \
            fflush(stderr);                   \
        }                                     \
    } while (0)

#define OR_OK 0
#define OR_EINVAL (-1)
#define OR_ENOMEM (-2)

/* ------------------------------------------------------------------------ */
/* Neighbourhood (Section 3.1): in-image pixels at unit distance.           */
/* The loops run over (dz, dy, dx) in lexicographic order; for in-image     */
/* pixels that order equals increasing linear index, so the returned list    */
/* is sorted by index.                                                        */
/* ------------------------------------------------------------------------ */
static int neighbours(int64_t p, int64_t nx, int64_t ny, int64_t nz, int conn, int64_t *out)
{
    int64_t x = p % nx, y = (p / nx) % ny, z = p / (nx * ny);
    int moore = (conn == 8 || conn == 26);
    int n = 0;
    for (int dz = -1; dz <= 1; ++dz)
        for (int dy = -1; dy <= 1; ++dy)
            for (int dx = -1; dx <= 1; ++dx) {
                int m = abs(dx) + abs(dy) + abs(dz);
                if (m == 0) continue;
                if (!moore && m != 1) continue;
                int64_t xx = x + dx, yy = y + dy, zz = z + dz;
                if (xx < 0 || xx >= nx || yy < 0 || yy >= ny || zz < 0 || zz >= nz) continue;
                out[n++] = xx + nx * (yy + ny * zz);
            }
    return n;
}

static int valid_dims(int64_t nx, int64_t ny, int64_t nz, int conn)
{
    if (nx < 1 || ny < 1 || nz < 1) return 0;
    if (conn != 4 && conn != 6 && conn != 8 && conn != 26) return 0;
    return 1;
}

/* ------------------------------------------------------------------------ */
/* Step I (Alg. 1 first loop, Eq. (1)).                                      */
/* q = the last neighbour, in pixel order, among those with the minimum     */
/* grey value. States: 0 lower neighbour, 1 local minimum, 2 plateau pixel  */
/* with an equal neighbour after it, 3 equal neighbours only before it.     */
/* ------------------------------------------------------------------------ */
int or_step1(const uint16_t *I, int64_t nx, int64_t ny, int64_t nz, int conn,
             int32_t *S, int32_t *L)
{
    if (!valid_dims(nx, ny, nz, conn) || !I || !S || !L) return OR_EINVAL;
    int64_t N = nx * ny * nz, nb[26];
    for (int64_t p = 0; p < N; ++p) {
        int n = neighbours(p, nx, ny, nz, conn, nb);
        if (n == 0) { L[p] = (int32_t)p; S[p] = 1; continue; }
        int64_t q = nb[0];
        for (int k = 1; k < n; ++k)
            if (I[nb[k]] <= I[q]) q = nb[k];   /* ties: later (larger) index wins */
        if (I[q] < I[p])      { L[p] = (int32_t)q; S[p] = 0; }
        else if (I[q] > I[p]) { L[p] = (int32_t)p; S[p] = 1; }
        else if (q > p)       { L[p] = (int32_t)q; S[p] = 2; }
        else                  { L[p] = (int32_t)p; S[p] = 3; }
    }
    return OR_OK;
}

/* ------------------------------------------------------------------------ */
/* Step II, synchronous form (Alg. 1 second loop, with the S' buffer of     */
/* Section 3.3). In every sweep, each pixel with S >= 2 that has a          */
/* neighbour q with S(q) = 0 and I(q) = I(p) -- S as it was at the start of */
/* the sweep -- takes L(p) = q and becomes state 0. Among several such q    */
/* the smallest index is taken. `dist` receives the sweep number in which a */
/* pixel was resolved (its geodesic distance to the plateau's lower border) */
/* and 0 otherwise. Returns the number of sweeps run, the last one being    */
/* the sweep that changed nothing (unless max_sweeps stopped it first).     */
/* ------------------------------------------------------------------------ */
static int64_t step2_sync(const uint16_t *I, int64_t nx, int64_t ny, int64_t nz, int conn,
                          int32_t *S, int32_t *L, int32_t *dist, int64_t max_sweeps)
{
    int64_t N = nx * ny * nz, nb[26];
    /* Only pixels with S >= 2 can change; keep them in a list (same result). */
    int64_t npend = 0;
    for (int64_t p = 0; p < N; ++p) { dist[p] = 0; if (S[p] >= 2) ++npend; }
    int64_t *pend = (int64_t *)malloc(sizeof(int64_t) * (size_t)(npend ? npend : 1));
    int64_t *res_p = (int64_t *)malloc(sizeof(int64_t) * (size_t)(npend ? npend : 1));
    int64_t *res_q = (int64_t *)malloc(sizeof(int64_t) * (size_t)(npend ? npend : 1));
    if (!pend || !res_p || !res_q) { free(pend); free(res_p); free(res_q); return -1; }
    npend = 0;
    for (int64_t p = 0; p < N; ++p) if (S[p] >= 2) pend[npend++] = p;

    int64_t sweeps = 0;
    for (;;) {
        if (max_sweeps >= 0 && sweeps >= max_sweeps) break;
        ++sweeps;
        /* Read phase: decide every update from the states at sweep start. */
        int64_t nres = 0;
        for (int64_t i = 0; i < npend; ++i) {
            int64_t p = pend[i];
            int n = neighbours(p, nx, ny, nz, conn, nb);
            for (int k = 0; k < n; ++k) {
                int64_t q = nb[k];
                if (S[q] == 0 && I[q] == I[p]) { res_p[nres] = p; res_q[nres] = q; ++nres; break; }
            }
        }
        if (nres == 0) break;  /* the sweep that changes nothing */
        /* Write phase (the swap of S and S'). */
        for (int64_t i = 0; i < nres; ++i) {
            L[res_p[i]] = (int32_t)res_q[i];
            S[res_p[i]] = 0;
            dist[res_p[i]] = (int32_t)sweeps;
        }
        int64_t w = 0;
        for (int64_t i = 0; i < npend; ++i) if (S[pend[i]] != 0) pend[w++] = pend[i];
        npend = w;
    }
    free(pend); free(res_p); free(res_q);
    return sweeps;
}

/* ------------------------------------------------------------------------ */
/* Step III (Alg. 1 third loop): every label is replaced by its label's     */
/* label up to RR times per synchronisation; the labels read are the ones   */
/* published at the previous synchronisation. Repeats until nothing         */
/* changes. Returns the number of synchronisations that changed a label.    */
/* ------------------------------------------------------------------------ */
static int64_t step3_reduce(int32_t *L, int64_t N, int RR)
{
    int32_t *old = (int32_t *)malloc(sizeof(int32_t) * (size_t)N);
    if (!old) return -1;
    int64_t changing = 0;
    for (;;) {
        memcpy(old, L, sizeof(int32_t) * (size_t)N);
        int changed = 0;
        for (int64_t p = 0; p < N; ++p) {
            int32_t cur = old[p];
            for (int i = 0; i < RR && cur != old[cur]; ++i) { cur = old[cur]; changed = 1; }
            L[p] = cur;
        }
        if (!changed) break;
        ++changing;
    }
    free(old);
    return changing;
}

/* Find / Union on the disjoint-set forest stored in L (Step IV). Union      */
/* links the larger root below the smaller one.                              */
static int32_t uf_find(const int32_t *L, int32_t x)
{
    while (L[x] != x) x = L[x];
    return x;
}

static void uf_union(int32_t *L, int32_t a, int32_t b)
{
    int32_t ra = uf_find(L, a), rb = uf_find(L, b);
    if (ra == rb) return;
    if (ra < rb) L[rb] = ra; else L[ra] = rb;
}

/* ------------------------------------------------------------------------ */
/* Full watershed: Steps I-IV of Alg. 1 in order, then canonical labels.    */
/*   S1_out   (optional) states after Step I                                 */
/*   bal_out  (optional) states after Step II in the balanced encoding of   */
/*            Section 3.4: -d for a resolved plateau pixel at distance d,   */
/*            otherwise the state (0..3)                                      */
/*   arrow_out(optional) L after Step II (the steepest-descent arrows)       */
/*   stats    (optional, 3 entries) Step II sweeps, Step III changing        */
/*            synchronisations, number of basins                              */
/* ------------------------------------------------------------------------ */
int or_watershed(const uint16_t *I, int64_t nx, int64_t ny, int64_t nz, int conn, int RR,
                 int64_t max_step2_sweeps, int32_t *labels, int32_t *S1_out, int32_t *bal_out,
                 int32_t *arrow_out, int64_t *stats)
{
    if (!valid_dims(nx, ny, nz, conn) || !I || !labels || RR < 1) return OR_EINVAL;
    int64_t N = nx * ny * nz, nb[26];
    if (N >= ((int64_t)1 << 31)) return OR_EINVAL;
    int32_t *S = (int32_t *)malloc(sizeof(int32_t) * (size_t)N);
    int32_t *L = (int32_t *)malloc(sizeof(int32_t) * (size_t)N);
    int32_t *dist = (int32_t *)malloc(sizeof(int32_t) * (size_t)N);
    if (!S || !L || !dist) { free(S); free(L); free(dist); return OR_ENOMEM; }

    /* Step I */
    or_step1(I, nx, ny, nz, conn, S, L);
    if (S1_out) memcpy(S1_out, S, sizeof(int32_t) * (size_t)N);
    OR_SAY("oracle: Step I done (%lld pixels)\n", (long long)N);

    /* Step II */
    int64_t sweeps = step2_sync(I, nx, ny, nz, conn, S, L, dist, max_step2_sweeps);
    OR_SAY("oracle: Step II done (%lld sweeps)\n", (long long)sweeps);
    if (bal_out)
        for (int64_t p = 0; p < N; ++p) bal_out[p] = dist[p] > 0 ? -dist[p] : S[p];
    if (arrow_out) memcpy(arrow_out, L, sizeof(int32_t) * (size_t)N);

    /* Step III */
    int64_t syncs = step3_reduce(L, N, RR);
    OR_SAY("oracle: Step III done (%lld synchronisations)\n", (long long)syncs);

    /* Step IV: union over neighbouring pixels that both still have S >= 2
     * (half neighbourhood, q > p), then Find for every pixel. */
    for (int64_t p = 0; p < N; ++p) {
        if (S[p] < 2) continue;
        int n = neighbours(p, nx, ny, nz, conn, nb);
        for (int k = 0; k < n; ++k)
            if (nb[k] > p && S[nb[k]] >= 2) uf_union(L, (int32_t)p, (int32_t)nb[k]);
    }
    for (int64_t p = 0; p < N; ++p) L[p] = uf_find(L, L[p]);
    OR_SAY("oracle: Step IV done\n");

    /* Canonical label: the smallest pixel index of each basin. */
    int32_t *cmin = dist;  /* reuse */
    for (int64_t p = 0; p < N; ++p) cmin[p] = INT32_MAX;
    for (int64_t p = 0; p < N; ++p) if ((int32_t)p < cmin[L[p]]) cmin[L[p]] = (int32_t)p;
    int64_t nbasins = 0;
    for (int64_t p = 0; p < N; ++p) { labels[p] = cmin[L[p]]; if (labels[p] == p) ++nbasins; }

    if (stats) { stats[0] = sweeps; stats[1] = syncs; stats[2] = nbasins; }
    free(S); free(L); free(dist);
    return OR_OK;
}

/* ------------------------------------------------------------------------ */
/* Graph waterfall (G1), NL layers. Layer 0 is the given canonical          */
/* partition. For k >= 1 every region R of layer k-1 finds                  */
/*   key(R) = min over boundary pairs (p in R, q in N(p), q not in R)       */
/*            of (max(I(p), I(q)), label(q)), lexicographically              */
/* (the height is Alg. 4 Step V's watershed height; the label is the        */
/* tie-break). Every region with a key is joined with the region its key    */
/* names; each connected group takes the smallest label in it.              */
/* `nregions` (optional, NL entries) receives the region count per layer.   */
/* ------------------------------------------------------------------------ */
int or_waterfall_g1(const int32_t *labels0, const uint16_t *I, int64_t nx, int64_t ny, int64_t nz,
                    int conn, int NL, int32_t *out, int64_t *nregions)
{
    if (!valid_dims(nx, ny, nz, conn) || !I || !labels0 || !out || NL < 1) return OR_EINVAL;
    int64_t N = nx * ny * nz, nb[26];
    if (N >= ((int64_t)1 << 31)) return OR_EINVAL;
    memcpy(out, labels0, sizeof(int32_t) * (size_t)N);
    int64_t cnt = 0;
    for (int64_t p = 0; p < N; ++p) if (labels0[p] == p) ++cnt;
    if (nregions) nregions[0] = cnt;
    if (NL == 1) return OR_OK;

    uint32_t *key_h = (uint32_t *)malloc(sizeof(uint32_t) * (size_t)N);
    int32_t *key_t = (int32_t *)malloc(sizeof(int32_t) * (size_t)N);
    int32_t *par = (int32_t *)malloc(sizeof(int32_t) * (size_t)N);
    if (!key_h || !key_t || !par) { free(key_h); free(key_t); free(par); return OR_ENOMEM; }

    for (int k = 1; k < NL; ++k) {
        const int32_t *prev = out + (size_t)(k - 1) * (size_t)N;
        int32_t *cur = out + (size_t)k * (size_t)N;
        for (int64_t p = 0; p < N; ++p) { key_h[p] = UINT32_MAX; key_t[p] = INT32_MAX; par[p] = (int32_t)p; }
        /* Lowest pass of every region (Step V), with the label across it. */
        for (int64_t p = 0; p < N; ++p) {
            int n = neighbours(p, nx, ny, nz, conn, nb);
            int32_t r = prev[p];
            for (int j = 0; j < n; ++j) {
                int64_t q = nb[j];
                if (prev[q] == r) continue;
                uint32_t h = I[p] > I[q] ? I[p] : I[q];
                if (h < key_h[r] || (h == key_h[r] && prev[q] < key_t[r])) { key_h[r] = h; key_t[r] = prev[q]; }
            }
        }
        /* Join each region with the one across its lowest pass. */
        for (int64_t p = 0; p < N; ++p)
            if (prev[p] == p && key_h[p] != UINT32_MAX) uf_union(par, (int32_t)p, key_t[p]);
        cnt = 0;
        for (int64_t p = 0; p < N; ++p) {
            cur[p] = uf_find(par, prev[p]);
            if (cur[p] == p) ++cnt;
        }
        if (nregions) nregions[k] = cnt;
    }
    free(key_h); free(key_t); free(par);
    return OR_OK;
}

/* ------------------------------------------------------------------------ */
/* Reconstruction waterfall (Alg. 4 Steps V-VI, then the watershed again,   */
/* as in Alg. 5). Layer 0 is the watershed of I. Between layers every basin */
/* is raised to its lowest pass height newmin, I(p) = max(I(p), newmin(L(p)))*/
/* (newmin initialised to M = 65535, at least the grey range's upper bound), */
/* and the watershed is recomputed on the raised image.                      */
/* ------------------------------------------------------------------------ */
int or_waterfall_recon(const uint16_t *I0, int64_t nx, int64_t ny, int64_t nz, int conn, int NL,
                       int32_t *out, int64_t *nregions)
{
    if (!valid_dims(nx, ny, nz, conn) || !I0 || !out || NL < 1) return OR_EINVAL;
    int64_t N = nx * ny * nz, nb[26];
    if (N >= ((int64_t)1 << 31)) return OR_EINVAL;
    uint16_t *I = (uint16_t *)malloc(sizeof(uint16_t) * (size_t)N);
    uint32_t *newmin = (uint32_t *)malloc(sizeof(uint32_t) * (size_t)N);
    if (!I || !newmin) { free(I); free(newmin); return OR_ENOMEM; }
    memcpy(I, I0, sizeof(uint16_t) * (size_t)N);
    for (int n = 0; n < NL; ++n) {
        int32_t *L = out + (size_t)n * (size_t)N;
        int64_t st[3];
        int rc = or_watershed(I, nx, ny, nz, conn, 6, -1, L, NULL, NULL, NULL, st);
        if (rc != OR_OK) { free(I); free(newmin); return rc; }
        if (nregions) nregions[n] = st[2];
        if (n == NL - 1) break;
        for (int64_t p = 0; p < N; ++p) newmin[p] = 65535u;  /* M */
        for (int64_t p = 0; p < N; ++p) {                      /* Step V */
            int k = neighbours(p, nx, ny, nz, conn, nb);
            for (int j = 0; j < k; ++j) {
                int64_t q = nb[j];
                if (L[q] == L[p]) continue;
                uint32_t h = I[p] > I[q] ? I[p] : I[q];
                if (h < newmin[L[p]]) newmin[L[p]] = h;
            }
        }
        for (int64_t p = 0; p < N; ++p)                        /* Step VI */
            if (I[p] < newmin[L[p]]) I[p] = (uint16_t)newmin[L[p]];
    }
    free(I); free(newmin);
    return OR_OK;
}

/* ------------------------------------------------------------------------ */
/* Gradient magnitude pre-processing (Introduction, pipeline steps 1-2).    */
/* ------------------------------------------------------------------------ */
static int64_t reflect_index(int64_t i, int64_t n)
{
    /* half-sample symmetric: ... c b a | a b c ... | c b a ... (period 2n) */
    int64_t m = 2 * n;
    i %= m;
    if (i < 0) i += m;
    return i < n ? i : m - 1 - i;
}

/* out = correlation of `in` with taps w[0..2r] (centre at r) along `axis`. */
static void correlate_axis(const double *in, double *out, int64_t nx, int64_t ny, int64_t nz,
                           int axis, const double *w, int r)
{
    int64_t n[3] = {nx, ny, nz};
    int64_t stride[3] = {1, nx, nx * ny};
    int64_t N = nx * ny * nz;
    for (int64_t p = 0; p < N; ++p) {
        int64_t c[3] = {p % nx, (p / nx) % ny, p / (nx * ny)};
        int64_t base = p - c[axis] * stride[axis];
        double s = 0.0;
        for (int k = -r; k <= r; ++k) {
            int64_t j = reflect_index(c[axis] + k, n[axis]);
            s += w[k + r] * in[base + j * stride[axis]];
        }
        out[p] = s;
    }
}

/*
 * img (float32, N) -> mag (double, N, optional) and q (uint16, N): the
 * quantised gradient magnitude with Q levels (255 for 8-bit, 65535 for
 * 16-bit output). sigma <= 0 skips the blur. 2D when nz == 1, else 3D.
 */
int or_gradient(const float *img, int64_t nx, int64_t ny, int64_t nz, double sigma, int Q,
                double *mag_out, uint16_t *q_out)
{
    if (nx < 1 || ny < 1 || nz < 1 || !img || !q_out || Q < 1 || Q > 65535) return OR_EINVAL;
    int64_t N = nx * ny * nz;
    int nd = nz > 1 ? 3 : 2;
    double *a = (double *)malloc(sizeof(double) * (size_t)N);
    double *b = (double *)malloc(sizeof(double) * (size_t)N);
    double *mag = (double *)calloc((size_t)N, sizeof(double));
    if (!a || !b || !mag) { free(a); free(b); free(mag); return OR_ENOMEM; }
    for (int64_t p = 0; p < N; ++p) a[p] = (double)img[p];

    if (sigma > 0.0) {
        int r = (int)(4.0 * sigma + 0.5);
        double *w = (double *)malloc(sizeof(double) * (size_t)(2 * r + 1));
        double sum = 0.0;
        for (int k = -r; k <= r; ++k) { w[k + r] = exp(-0.5 * (double)k * (double)k / (sigma * sigma)); sum += w[k + r]; }
        for (int k = 0; k <= 2 * r; ++k) w[k] /= sum;
        for (int ax = 0; ax < nd; ++ax) {
            correlate_axis(a, b, nx, ny, nz, ax, w, r);
            double *t = a; a = b; b = t;
        }
        free(w);
    }

    /* Sobel: derivative taps [-1, 0, 1] along one axis, smoothing taps
     * [1, 2, 1] along every other axis; magnitude over the axes. */
    static const double dtap[3] = {-1.0, 0.0, 1.0};
    static const double stap[3] = {1.0, 2.0, 1.0};
    double *t1 = (double *)malloc(sizeof(double) * (size_t)N);
    if (!t1) { free(a); free(b); free(mag); return OR_ENOMEM; }
    for (int ax = 0; ax < nd; ++ax) {
        correlate_axis(a, b, nx, ny, nz, ax, dtap, 1);
        double *src = b, *dst = t1;
        for (int o = 0; o < nd; ++o) {
            if (o == ax) continue;
            correlate_axis(src, dst, nx, ny, nz, o, stap, 1);
            double *t = src; src = dst; dst = t;
        }
        for (int64_t p = 0; p < N; ++p) mag[p] += src[p] * src[p];
    }
    free(t1);
    double mx = 0.0;
    for (int64_t p = 0; p < N; ++p) { mag[p] = sqrt(mag[p]); if (mag[p] > mx) mx = mag[p]; }
    for (int64_t p = 0; p < N; ++p) {
        double v = mx > 0.0 ? nearbyint(mag[p] * (double)Q / mx) : 0.0;
        q_out[p] = (uint16_t)v;
    }
    if (mag_out) memcpy(mag_out, mag, sizeof(double) * (size_t)N);
    free(a); free(b); free(mag);
    return OR_OK;
}
