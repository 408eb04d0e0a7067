/*
 * UoI_LASSO / UoI_VAR CPU oracle -- TEST INFRASTRUCTURE ONLY.
 *
 * Plain, slow, FP64 C written from the paper (Balasubramanian et al., "Optimizing
 * the Union of Intersections LASSO and Vector Autoregressive algorithms", arXiv
 * 1808.06992): Eq. (1)-(2) (linear model, LASSO), Sec. II-C Eq. (intersection),
 * Sec. II-D Eq. (union), Algorithm 1 (UoI_LASSO), Eq. (5)-(8) and Algorithm 2
 * (UoI_VAR).  Only tests/, the smoke check and the benchmark's CPU-baseline leg
 * may load this library.  It shares no code, header, table or constant
 * generator with the HIP library; the only thing the two have in common is the
 * published definition of SplitMix64 that both implement on their own.
 *
 * Readings of points the paper leaves open (each one is listed in the design
 * notes of the repository):
 *   - LASSO objective scaled as (1/(2m)) sum (y - x'b)^2 + lam*|b|_1 over the m
 *     rows of a sample (same minimiser as Eq. (2) with lam2 = 2*m*lam), i.e.
 *     0.5 b'Gb - c'b + lam*|b|_1 with G = X'X/m and c = X'y/m.
 *   - Bootstrap = m draws with replacement; estimation split = train/eval
 *     partition without replacement (train = floor(m*num/den) rows).
 *   - VAR bootstrap = moving blocks of regression rows.
 *   - Support = coordinates of the LASSO estimate that are exactly nonzero.
 *   - OLS on a support = the least-squares minimiser on the training rows
 *     (the paper runs ADMM with lam = 0; both reach the same minimiser).
 *   - Loss = mean squared residual on the evaluation rows; VAR sums it over
 *     equations and picks one support index per bootstrap; ties pick the
 *     smallest index j (largest lambda).
 *
 * The LASSO minimiser is found by cyclic coordinate descent (not ADMM), then
 * confirmed exactly: on the current support A with signs s the stationarity
 * equations G_AA b_A = c_A - lam*s_A are solved by Cholesky and accepted when
 * the KKT residual of the result is below the requested tolerance.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#include "uoi_oracle.h"

/* ------------------------------------------------------------------------ */
/* Random indices.  Alg. 1 leaves the resampling scheme open; here the      */
/* index stream is a counter-based SplitMix64 (Steele, Lea, Flood 2014)      */
/* keyed by (seed, tag, bootstrap, position), mapped to [0, m) by Lemire's   */
/* multiply-shift.                                                            */
/* ------------------------------------------------------------------------ */
uint64_t orc_mix64(uint64_t x)
{
    x += 0x9E3779B97F4A7C15ULL;
    x = (x ^ (x >> 30)) * 0xBF58476D1CE4E5B9ULL;
    x = (x ^ (x >> 27)) * 0x94D049BB133111EBULL;
    return x ^ (x >> 31);
}

uint64_t orc_key(uint64_t seed, uint32_t tag, uint32_t k, uint32_t i)
{
    uint64_t base = orc_mix64(seed ^ ((uint64_t)tag << 56));
    return orc_mix64(base ^ (((uint64_t)k << 32) | (uint64_t)i));
}

uint32_t orc_index(uint64_t r, uint32_t m)
{
    return (uint32_t)(((unsigned __int128)r * (unsigned __int128)m) >> 64);
}

/* Alg. 1 selection loop, the sample T^k: n row draws with replacement. */
void orc_boot_rows(uint64_t seed, int k, int n, int32_t *rows)
{
    for (int i = 0; i < n; ++i)
        rows[i] = (int32_t)orc_index(orc_key(seed, ORC_TAG_LASSO_BOOT, (uint32_t)k, (uint32_t)i),
                                     (uint32_t)n);
}

typedef struct { uint64_t key; int32_t idx; } keyed_t;

static int keyed_cmp(const void *a, const void *b)
{
    const keyed_t *x = (const keyed_t *)a, *y = (const keyed_t *)b;
    if (x->key != y->key) return x->key < y->key ? -1 : 1;
    return x->idx < y->idx ? -1 : (x->idx > y->idx);
}

static int int_cmp(const void *a, const void *b)
{
    int32_t x = *(const int32_t *)a, y = *(const int32_t *)b;
    return x < y ? -1 : (x > y);
}

/* Order items 0..cnt-1 by (key(seed,tag,k,i), i); the first ntrain are the
 * training items.  Both lists are returned in ascending item order. */
static void keyed_split(uint64_t seed, uint32_t tag, int k, int cnt, int ntrain,
                        int32_t *train, int32_t *eval)
{
    keyed_t *a = (keyed_t *)malloc(sizeof(keyed_t) * (size_t)cnt);
    for (int i = 0; i < cnt; ++i) {
        a[i].key = orc_key(seed, tag, (uint32_t)k, (uint32_t)i);
        a[i].idx = i;
    }
    qsort(a, (size_t)cnt, sizeof(keyed_t), keyed_cmp);
    for (int i = 0; i < ntrain; ++i) train[i] = a[i].idx;
    for (int i = ntrain; i < cnt; ++i) eval[i - ntrain] = a[i].idx;
    qsort(train, (size_t)ntrain, sizeof(int32_t), int_cmp);
    qsort(eval, (size_t)(cnt - ntrain), sizeof(int32_t), int_cmp);
    free(a);
}

int orc_split_count(int n, int num, int den)
{
    return (int)(((int64_t)n * num) / den);
}

/* Alg. 1 estimation loop: the training and evaluation samples, read here as a
 * partition of the n rows without replacement, training = floor(n*num/den) rows. */
void orc_split_rows(uint64_t seed, int k, int n, int num, int den, int32_t *train, int32_t *eval)
{
    keyed_split(seed, ORC_TAG_LASSO_SPLIT, k, n, orc_split_count(n, num, den), train, eval);
}

/* Smallest L with L^3 >= N (the block length used when none is given). */
int orc_var_block_len(int N)
{
    int L = 1;
    while ((int64_t)L * L * L < (int64_t)N) ++L;
    return L;
}

int orc_var_nblocks(int N, int L) { return (N + L - 1) / L; }

/* Alg. 2 block bootstrap (Sec. III-A.2): moving blocks of L consecutive
 * regression rows at random starts, nb = ceil(N/L) blocks, truncated to N rows. */
void orc_var_boot_rows(uint64_t seed, int k, int N, int L, int32_t *rows)
{
    int nb = orc_var_nblocks(N, L);
    int pos = 0;
    for (int b = 0; b < nb && pos < N; ++b) {
        int s = (int)orc_index(orc_key(seed, ORC_TAG_VAR_BOOT, (uint32_t)k, (uint32_t)b),
                               (uint32_t)(N - L + 1));
        for (int t = 0; t < L && pos < N; ++t) rows[pos++] = s + t;
    }
}

/* Alg. 2 estimation samples: natural blocks [bL, min((b+1)L, N)) split into
 * train/eval blocks; returns the row counts through *ntr / *nev. */
void orc_var_split_rows(uint64_t seed, int k, int N, int L, int num, int den,
                        int32_t *train, int *ntr, int32_t *eval, int *nev)
{
    int nb = orc_var_nblocks(N, L);
    int nbt = orc_split_count(nb, num, den);
    int32_t *tb = (int32_t *)malloc(sizeof(int32_t) * (size_t)nb);
    int32_t *eb = (int32_t *)malloc(sizeof(int32_t) * (size_t)nb);
    keyed_split(seed, ORC_TAG_VAR_SPLIT, k, nb, nbt, tb, eb);
    int a = 0, e = 0;
    for (int i = 0; i < nbt; ++i)
        for (int t = tb[i] * L; t < (tb[i] + 1) * L && t < N; ++t) train[a++] = t;
    for (int i = 0; i < nb - nbt; ++i)
        for (int t = eb[i] * L; t < (eb[i] + 1) * L && t < N; ++t) eval[e++] = t;
    *ntr = a;
    *nev = e;
    free(tb);
    free(eb);
}

/* ------------------------------------------------------------------------ */
/* Normal-equation statistics of a row sample (rows counted with            */
/* multiplicity): G = (1/m) sum x_r x_r',  C = (1/m) sum x_r y_r'.          */
/* Row r of the design is X + r*ldx (p values), of the response Y + r*ldy   */
/* (pe values).  G is p x p, C is p x pe, both row-major.                   */
/* ------------------------------------------------------------------------ */
void orc_gram(int m, const int32_t *rows, int p, const double *X, int ldx,
              int pe, const double *Y, int ldy, double *G, double *C)
{
    memset(G, 0, sizeof(double) * (size_t)p * p);
    if (C) memset(C, 0, sizeof(double) * (size_t)p * pe);
    for (int i = 0; i < m; ++i) {
        const double *x = X + (size_t)rows[i] * ldx;
        for (int a = 0; a < p; ++a) {
            double xa = x[a];
            double *Ga = G + (size_t)a * p;
            for (int b = 0; b < p; ++b) Ga[b] += xa * x[b];
        }
        if (C) {
            const double *yv = Y + (size_t)rows[i] * ldy;
            for (int a = 0; a < p; ++a)
                for (int e = 0; e < pe; ++e) C[(size_t)a * pe + e] += x[a] * yv[e];
        }
    }
    double inv = 1.0 / (double)m;
    for (size_t t = 0; t < (size_t)p * p; ++t) G[t] *= inv;
    if (C)
        for (size_t t = 0; t < (size_t)p * pe; ++t) C[t] *= inv;
}

/* ------------------------------------------------------------------------ */
/* KKT residual of Eq. (2) in the 1/(2m) scaling: g = c - G b;              */
/* v_i = |g_i - lam*sign(b_i)| if b_i != 0, else max(0, |g_i| - lam);        */
/* returns ||v||_inf / ||c||_inf (||v||_inf when c = 0).                     */
/* ------------------------------------------------------------------------ */
double orc_kkt(int p, const double *G, const double *c, int ldc, double lam, const double *b)
{
    double vmax = 0.0, cmax = 0.0;
    for (int i = 0; i < p; ++i) {
        double g = c[(size_t)i * ldc];
        const double *Gi = G + (size_t)i * p;
        for (int l = 0; l < p; ++l) g -= Gi[l] * b[l];
        double v;
        if (b[i] != 0.0) v = fabs(g - (b[i] > 0 ? lam : -lam));
        else v = fabs(g) - lam > 0.0 ? fabs(g) - lam : 0.0;
        if (v > vmax) vmax = v;
        double ca = fabs(c[(size_t)i * ldc]);
        if (ca > cmax) cmax = ca;
    }
    return cmax > 0.0 ? vmax / cmax : vmax;
}

static double soft(double a, double t)
{
    if (a > t) return a - t;
    if (a < -t) return a + t;
    return 0.0;
}

/* Cholesky of an s x s SPD matrix in place (lower triangle); 0 on success. */
static int chol(int s, double *A)
{
    for (int j = 0; j < s; ++j) {
        double d = A[(size_t)j * s + j];
        for (int k = 0; k < j; ++k) d -= A[(size_t)j * s + k] * A[(size_t)j * s + k];
        if (!(d > 0.0)) return -1;
        d = sqrt(d);
        A[(size_t)j * s + j] = d;
        for (int i = j + 1; i < s; ++i) {
            double v = A[(size_t)i * s + j];
            for (int k = 0; k < j; ++k) v -= A[(size_t)i * s + k] * A[(size_t)j * s + k];
            A[(size_t)i * s + j] = v / d;
        }
    }
    return 0;
}

/* Solve L L' x = b in place. */
static void chol_solve(int s, const double *L, double *x)
{
    for (int i = 0; i < s; ++i) {
        double v = x[i];
        for (int k = 0; k < i; ++k) v -= L[(size_t)i * s + k] * x[k];
        x[i] = v / L[(size_t)i * s + i];
    }
    for (int i = s - 1; i >= 0; --i) {
        double v = x[i];
        for (int k = i + 1; k < s; ++k) v -= L[(size_t)k * s + i] * x[k];
        x[i] = v / L[(size_t)i * s + i];
    }
}

/* Exact stationary point on the support of b with the signs of b:
 * G_AA b_A = c_A - lam*s_A.  Writes the candidate to out; returns -1 if the
 * solve fails or a sign flips (then the candidate is not a LASSO solution). */
static int active_set_solve(int p, const double *G, const double *c, int ldc, double lam,
                            const double *b, double *out, int *idx, double *work)
{
    int s = 0;
    for (int i = 0; i < p; ++i)
        if (b[i] != 0.0) idx[s++] = i;
    double *A = work, *r = work + (size_t)s * s;
    for (int a = 0; a < s; ++a) {
        for (int t = 0; t < s; ++t) A[(size_t)a * s + t] = G[(size_t)idx[a] * p + idx[t]];
        r[a] = c[(size_t)idx[a] * ldc] - (b[idx[a]] > 0 ? lam : -lam);
    }
    if (s > 0) {
        if (chol(s, A) != 0) return -1;
        chol_solve(s, A, r);
    }
    for (int i = 0; i < p; ++i) out[i] = 0.0;
    for (int a = 0; a < s; ++a) {
        if ((r[a] > 0) != (b[idx[a]] > 0) || r[a] == 0.0) return -1;
        out[idx[a]] = r[a];
    }
    return 0;
}

/* LASSO on (G, c): minimise 0.5 b'Gb - c'b + lam*|b|_1 (Eq. (2), 1/(2m)
 * scaling) by cyclic coordinate descent, b_i <- S_lam(c_i - sum_{l!=i} G_il b_l)/G_ii,
 * started from the value in b.  Stops when the KKT residual is <= tol; after
 * every round the exact solve on the current support is tried and kept if it
 * meets the tolerance.  Returns the number of full sweeps, or -1 if max_sweeps
 * was reached (b then holds the last iterate). */
int orc_lasso_cd(int p, const double *G, const double *c, int ldc, double lam, double tol,
                 int max_sweeps, double *b)
{
    double *g = (double *)malloc(sizeof(double) * (size_t)p);
    double *cand = (double *)malloc(sizeof(double) * (size_t)p);
    int *idx = (int *)malloc(sizeof(int) * (size_t)p);
    double *work = (double *)malloc(sizeof(double) * ((size_t)p * p + p));
    int sweeps = 0, status = -1;
    for (;;) {
        if (orc_kkt(p, G, c, ldc, lam, b) <= tol) { status = sweeps; break; }
        if (sweeps >= max_sweeps) break;
        /* gradient residual g = c - G b, refreshed every round */
        for (int i = 0; i < p; ++i) {
            double v = c[(size_t)i * ldc];
            for (int l = 0; l < p; ++l) v -= G[(size_t)i * p + l] * b[l];
            g[i] = v;
        }
        /* one full sweep followed by sweeps over the nonzero coordinates */
        for (int pass = 0; pass < 64; ++pass) {
            double change = 0.0, scale = 0.0;
            for (int i = 0; i < p; ++i) {
                if (pass > 0 && b[i] == 0.0) continue;
                double Gii = G[(size_t)i * p + i];
                double a = g[i] + Gii * b[i];
                double nb = soft(a, lam) / Gii;
                double d = nb - b[i];
                if (d != 0.0) {
                    const double *Gi = G + (size_t)i * p; /* column i == row i */
                    for (int l = 0; l < p; ++l) g[l] -= d * Gi[l];
                    b[i] = nb;
                    if (fabs(d) > change) change = fabs(d);
                }
                if (fabs(b[i]) > scale) scale = fabs(b[i]);
            }
            if (pass == 0) ++sweeps;
            if (change <= 1e-15 * (scale > 0 ? scale : 1.0)) break;
        }
        /* exact stationary point on the current support, kept if it is a solution */
        if (active_set_solve(p, G, c, ldc, lam, b, cand, idx, work) == 0 &&
            orc_kkt(p, G, c, ldc, lam, cand) <= tol) {
            memcpy(b, cand, sizeof(double) * (size_t)p);
            status = sweeps;
            break;
        }
    }
    free(g);
    free(cand);
    free(idx);
    free(work);
    return status;
}

/* ------------------------------------------------------------------------ */
/* Least squares.                                                           */
/* ------------------------------------------------------------------------ */

/* Householder QR least squares: A is m x s column-major (destroyed), yv is m
 * (destroyed); solution in b (s).  Returns -1 on an exactly singular R. */
int orc_lstsq_qr(int m, int s, double *A, double *yv, double *b)
{
    for (int j = 0; j < s; ++j) {
        double *aj = A + (size_t)j * m;
        double nrm = 0.0;
        for (int i = j; i < m; ++i) nrm += aj[i] * aj[i];
        nrm = sqrt(nrm);
        if (nrm == 0.0) return -1;
        double alpha = aj[j] > 0 ? -nrm : nrm;
        double v0 = aj[j] - alpha;
        /* v = (v0, a_{j+1..m-1}); H = I - 2 vv'/(v'v) */
        double vtv = v0 * v0;
        for (int i = j + 1; i < m; ++i) vtv += aj[i] * aj[i];
        aj[j] = v0;
        for (int t = j + 1; t < s; ++t) {
            double *at = A + (size_t)t * m;
            double d = 0.0;
            for (int i = j; i < m; ++i) d += aj[i] * at[i];
            d = 2.0 * d / vtv;
            for (int i = j; i < m; ++i) at[i] -= d * aj[i];
        }
        double d = 0.0;
        for (int i = j; i < m; ++i) d += aj[i] * yv[i];
        d = 2.0 * d / vtv;
        for (int i = j; i < m; ++i) yv[i] -= d * aj[i];
        aj[j] = alpha; /* R_jj; entries below are the reflector, no longer needed */
    }
    for (int j = s - 1; j >= 0; --j) {
        double v = yv[j];
        for (int t = j + 1; t < s; ++t) v -= A[(size_t)t * m + j] * b[t];
        b[j] = v / A[(size_t)j * m + j];
    }
    return 0;
}

/* OLS on the columns idx[0..s-1] from the normal equations of a row sample:
 * G[S,S] b = c[S] (Cholesky).  Returns -1 if G[S,S] is not positive definite. */
int orc_ols_normal(int p, const double *G, const double *c, int ldc, int s, const int *idx,
                   double *b, double *work)
{
    for (int a = 0; a < s; ++a) {
        for (int t = 0; t < s; ++t) work[(size_t)a * s + t] = G[(size_t)idx[a] * p + idx[t]];
        b[a] = c[(size_t)idx[a] * ldc];
    }
    if (s == 0) return 0;
    if (chol(s, work) != 0) return -1;
    chol_solve(s, work, b);
    return 0;
}

/* ------------------------------------------------------------------------ */
/* Support bitmasks: bit i of word i/64 is set when coefficient i is nonzero */
/* ------------------------------------------------------------------------ */
static void set_support(int p, const double *b, uint64_t *w)
{
    int W = (p + 63) / 64;
    for (int t = 0; t < W; ++t) w[t] = 0;
    for (int i = 0; i < p; ++i)
        if (b[i] != 0.0) w[i >> 6] |= (uint64_t)1 << (i & 63);
}

static int support_list(int p, const uint64_t *w, int *idx)
{
    int s = 0;
    for (int i = 0; i < p; ++i)
        if ((w[i >> 6] >> (i & 63)) & 1) idx[s++] = i;
    return s;
}

/* ------------------------------------------------------------------------ */
/* Algorithm 1: UoI_LASSO.                                                   */
/* ------------------------------------------------------------------------ */
int orc_uoi_lasso(int n, int p, const double *X, const double *y,
                  int B1, int B2, int q, const double *lam, uint64_t seed,
                  int num, int den, double tol, int max_sweeps,
                  double *beta_star, uint64_t *supp, int32_t *jstar, double *losses,
                  double *sel_beta, double *sel_kkt, double *ols_beta)
{
    int W = (p + 63) / 64;
    int bad = 0;
    /* Model selection: for every bootstrap k and every lambda_j, the LASSO
     * estimate and its support; S_j = intersection over k (Eq. (intersection)). */
    for (size_t t = 0; t < (size_t)q * W; ++t) supp[t] = ~(uint64_t)0;
    if (p % 64)
        for (int j = 0; j < q; ++j) supp[(size_t)j * W + W - 1] = ((uint64_t)1 << (p % 64)) - 1;
#pragma omp parallel for schedule(dynamic, 1) reduction(+ : bad)
    for (int k = 0; k < B1; ++k) {
        int32_t *rows = (int32_t *)malloc(sizeof(int32_t) * (size_t)n);
        double *G = (double *)malloc(sizeof(double) * (size_t)p * p);
        double *c = (double *)malloc(sizeof(double) * (size_t)p);
        double *b = (double *)calloc((size_t)p, sizeof(double));
        uint64_t *w = (uint64_t *)malloc(sizeof(uint64_t) * (size_t)W);
        orc_boot_rows(seed, k, n, rows);
        orc_gram(n, rows, p, X, p, 1, y, 1, G, c);
        for (int j = 0; j < q; ++j) {
            /* warm start from the previous lambda: the minimiser is unique, so the
             * start only changes the number of sweeps */
            if (orc_lasso_cd(p, G, c, 1, lam[j], tol, max_sweeps, b) < 0) ++bad;
            if (sel_beta) memcpy(sel_beta + ((size_t)k * q + j) * p, b, sizeof(double) * (size_t)p);
            if (sel_kkt) sel_kkt[(size_t)k * q + j] = orc_kkt(p, G, c, 1, lam[j], b);
            set_support(p, b, w);
#pragma omp critical
            for (int t = 0; t < W; ++t) supp[(size_t)j * W + t] &= w[t];
        }
        free(rows); free(G); free(c); free(b); free(w);
    }
    /* Model estimation: OLS of every S_j on the training rows of bootstrap k,
     * loss on its evaluation rows, best j per bootstrap, average (Eq. (union)). */
    int ntr = orc_split_count(n, num, den), nev = n - ntr;
    double *acc = (double *)calloc((size_t)B2 * p, sizeof(double));
#pragma omp parallel for schedule(dynamic, 1) reduction(+ : bad)
    for (int k = 0; k < B2; ++k) {
        int32_t *tr = (int32_t *)malloc(sizeof(int32_t) * (size_t)(ntr > 0 ? ntr : 1));
        int32_t *ev = (int32_t *)malloc(sizeof(int32_t) * (size_t)(nev > 0 ? nev : 1));
        double *G = (double *)malloc(sizeof(double) * (size_t)p * p);
        double *c = (double *)malloc(sizeof(double) * (size_t)p);
        double *work = (double *)malloc(sizeof(double) * (size_t)p * p);
        double *bs = (double *)malloc(sizeof(double) * (size_t)p);
        double *fit = (double *)malloc(sizeof(double) * (size_t)q * p);
        double *Lk = (double *)malloc(sizeof(double) * (size_t)q);
        int *idx = (int *)malloc(sizeof(int) * (size_t)p);
        orc_split_rows(seed, k, n, num, den, tr, ev);
        orc_gram(ntr, tr, p, X, p, 1, y, 1, G, c);
        for (int j = 0; j < q; ++j) {
            int s = support_list(p, supp + (size_t)j * W, idx);
            if (orc_ols_normal(p, G, c, 1, s, idx, bs, work) != 0) ++bad;
            double *f = fit + (size_t)j * p;
            memset(f, 0, sizeof(double) * (size_t)p);
            for (int a = 0; a < s; ++a) f[idx[a]] = bs[a];
            double L = 0.0;
            for (int r = 0; r < nev; ++r) {
                const double *x = X + (size_t)ev[r] * p;
                double e = y[ev[r]];
                for (int a = 0; a < s; ++a) e -= x[idx[a]] * bs[a];
                L += e * e;
            }
            Lk[j] = nev > 0 ? L / nev : 0.0;
            if (losses) losses[(size_t)k * q + j] = Lk[j];
            if (ols_beta) memcpy(ols_beta + ((size_t)k * q + j) * p, f, sizeof(double) * (size_t)p);
        }
        int best = 0;
        for (int j = 1; j < q; ++j)
            if (Lk[j] < Lk[best]) best = j;
        jstar[k] = best;
        memcpy(acc + (size_t)k * p, fit + (size_t)best * p, sizeof(double) * (size_t)p);
        free(tr); free(ev); free(G); free(c); free(work); free(bs); free(fit); free(Lk); free(idx);
    }
    for (int i = 0; i < p; ++i) {
        double s = 0.0;
        for (int k = 0; k < B2; ++k) s += acc[(size_t)k * p + i];
        beta_star[i] = s / B2;
    }
    free(acc);
    return bad ? -1 : 0;
}

/* ------------------------------------------------------------------------ */
/* Algorithm 2: UoI_VAR for d = 1.  Regression row r (0 <= r < N = T-1) has  */
/* design x = series[r] and response y = series[r+1] (Eq. (6)-(7)).  The    */
/* vectorised LASSO of Eq. (8) with design I (x) X separates into p LASSOs,  */
/* one per equation e (column e of Y), sharing G = X'X/m and one lambda.     */
/* Output A[e][l] = coefficient of x_{t-1,l} in equation e.                 */
/* ------------------------------------------------------------------------ */
int orc_uoi_var(int T, int p, const double *series, int L, int B1, int B2, int q,
                const double *lam, uint64_t seed, int num, int den, double tol, int max_sweeps,
                double *A_out, uint64_t *supp, int32_t *jstar, double *losses)
{
    int N = T - 1;
    int W = (p + 63) / 64;
    if (L <= 0) L = orc_var_block_len(N);
    int bad = 0;
    const double *Xd = series, *Yd = series + p;
    size_t sw = (size_t)q * p * W;
    for (size_t t = 0; t < sw; ++t) supp[t] = ~(uint64_t)0;
    if (p % 64)
        for (size_t t = 0; t < (size_t)q * p; ++t) supp[t * W + W - 1] = ((uint64_t)1 << (p % 64)) - 1;
    int32_t *rows = (int32_t *)malloc(sizeof(int32_t) * (size_t)N);
    double *G = (double *)malloc(sizeof(double) * (size_t)p * p);
    double *C = (double *)malloc(sizeof(double) * (size_t)p * p);
    /* Model selection */
    for (int k = 0; k < B1; ++k) {
        orc_var_boot_rows(seed, k, N, L, rows);
        orc_gram(N, rows, p, Xd, p, p, Yd, p, G, C);
#pragma omp parallel for schedule(dynamic, 1) reduction(+ : bad)
        for (int e = 0; e < p; ++e) {
            double *b = (double *)calloc((size_t)p, sizeof(double));
            uint64_t *w = (uint64_t *)malloc(sizeof(uint64_t) * (size_t)W);
            for (int j = 0; j < q; ++j) {
                if (orc_lasso_cd(p, G, C + e, p, lam[j], tol, max_sweeps, b) < 0) ++bad;
                set_support(p, b, w);
                uint64_t *S = supp + ((size_t)j * p + e) * W;
                for (int t = 0; t < W; ++t) S[t] &= w[t];
            }
            free(b); free(w);
        }
    }
    /* Model estimation */
    int32_t *tr = (int32_t *)malloc(sizeof(int32_t) * (size_t)N);
    int32_t *ev = (int32_t *)malloc(sizeof(int32_t) * (size_t)N);
    double *fit = (double *)malloc(sizeof(double) * (size_t)q * p * p);
    double *Lk = (double *)malloc(sizeof(double) * (size_t)q * p);
    double *acc = (double *)calloc((size_t)p * p, sizeof(double));
    for (int k = 0; k < B2; ++k) {
        int ntr = 0, nev = 0;
        orc_var_split_rows(seed, k, N, L, num, den, tr, &ntr, ev, &nev);
        orc_gram(ntr, tr, p, Xd, p, p, Yd, p, G, C);
#pragma omp parallel for schedule(dynamic, 1) reduction(+ : bad)
        for (int e = 0; e < p; ++e) {
            double *work = (double *)malloc(sizeof(double) * (size_t)p * p);
            double *bs = (double *)malloc(sizeof(double) * (size_t)p);
            int *idx = (int *)malloc(sizeof(int) * (size_t)p);
            for (int j = 0; j < q; ++j) {
                int s = support_list(p, supp + ((size_t)j * p + e) * W, idx);
                if (orc_ols_normal(p, G, C + e, p, s, idx, bs, work) != 0) ++bad;
                double *f = fit + ((size_t)j * p + e) * p;
                memset(f, 0, sizeof(double) * (size_t)p);
                for (int a = 0; a < s; ++a) f[idx[a]] = bs[a];
                double Ls = 0.0;
                for (int r = 0; r < nev; ++r) {
                    const double *x = Xd + (size_t)ev[r] * p;
                    double res = Yd[(size_t)ev[r] * p + e];
                    for (int a = 0; a < s; ++a) res -= x[idx[a]] * bs[a];
                    Ls += res * res;
                }
                Lk[(size_t)j * p + e] = nev > 0 ? Ls / nev : 0.0;
            }
            free(work); free(bs); free(idx);
        }
        int best = 0;
        double bestL = 0.0;
        for (int j = 0; j < q; ++j) {
            double s = 0.0;
            for (int e = 0; e < p; ++e) s += Lk[(size_t)j * p + e];
            if (losses) losses[(size_t)k * q + j] = s;
            if (j == 0 || s < bestL) { bestL = s; best = j; }
        }
        jstar[k] = best;
        for (size_t t = 0; t < (size_t)p * p; ++t) acc[t] += fit[(size_t)best * p * p + t];
    }
    for (size_t t = 0; t < (size_t)p * p; ++t) A_out[t] = acc[t] / B2;
    free(rows); free(G); free(C); free(tr); free(ev); free(fit); free(Lk); free(acc);
    return bad ? -1 : 0;
}

/* ------------------------------------------------------------------------ */
/* Alg. 2 for a VAR(d) series (Eq. (5)-(8)), with an optional intercept.     */
/*                                                                            */
/* Regression row r = 0..N-1 (N = T - d) has the response x_{r+d} and, as in */
/* Eq. (7), the design [x_{r+d-1}, x_{r+d-2}, ..., x_r] (lag 1 first), built  */
/* here explicitly as an N x (d p) matrix.  Equation e's coefficient vector  */
/* b_e (length d p) holds A_l[e][m] at position (l-1) p + m (vec B of Eq. (8) */
/* stacks these per equation); supports use the same bit positions.          */
/*                                                                            */
/* Intercept (Alg. 2 returns mu-hat; Eq. (5) as printed has none): the model */
/* x_t = mu + sum_l A_l x_{t-l} + u_t with mu unpenalised.  Every sample --   */
/* each bootstrap sample of the selection, each training set of the          */
/* estimation -- is centred by its own column means (counting repeated rows  */
/* with their multiplicity), which profiles mu out of the least-squares term.*/
/* A refit's intercept is mu_e = ybar_T[e] - xbar_T' b_e, its loss uses the   */
/* residuals y - mu - x'b on the evaluation rows, and mu-hat averages the     */
/* chosen refits' intercepts like every other coefficient of beta*.          */
/*                                                                            */
/* per_eq: every equation chooses its own support index per split (the argmin */
/* over lambda of that equation's loss) instead of one index for all          */
/* equations from the summed loss; losses are then reported per equation     */
/* ([B2][q][p]) and jstar per equation ([B2][p]).                             */
/* ------------------------------------------------------------------------ */

/* Centred copy of the sampled rows: out row a = src[rows[a]] - mean over the sample. */
static void centred_sample(int m, const int32_t *rows, int w, const double *src, double *out,
                           double *mean, int centre)
{
    for (int c = 0; c < w; ++c) mean[c] = 0.0;
    if (centre) {
        for (int a = 0; a < m; ++a)
            for (int c = 0; c < w; ++c) mean[c] += src[(size_t)rows[a] * w + c];
        for (int c = 0; c < w; ++c) mean[c] /= m;
    }
    for (int a = 0; a < m; ++a)
        for (int c = 0; c < w; ++c) out[(size_t)a * w + c] = src[(size_t)rows[a] * w + c] - mean[c];
}

int orc_uoi_var_d(int T, int p, int d, int intercept, int per_eq, const double *series, int L,
                  int B1, int B2, int q, const double *lam, uint64_t seed, int num, int den,
                  double tol, int max_sweeps, double *A_out, double *mu_out, uint64_t *supp,
                  int32_t *jstar, double *losses)
{
    const int N = T - d, P = d * p;
    const int W = (P + 63) / 64;
    if (L <= 0) L = orc_var_block_len(N);
    int bad = 0;
    /* the lagged design (Eq. (7), lag 1 first) and the responses (Eq. (6)) */
    double *Xl = (double *)malloc(sizeof(double) * (size_t)N * P);
    double *Yl = (double *)malloc(sizeof(double) * (size_t)N * p);
    for (int r = 0; r < N; ++r) {
        for (int l = 0; l < d; ++l)
            for (int m = 0; m < p; ++m)
                Xl[(size_t)r * P + (size_t)l * p + m] = series[(size_t)(r + d - 1 - l) * p + m];
        for (int e = 0; e < p; ++e) Yl[(size_t)r * p + e] = series[(size_t)(r + d) * p + e];
    }
    size_t sw = (size_t)q * p * W;
    for (size_t t = 0; t < sw; ++t) supp[t] = ~(uint64_t)0;
    if (P % 64)
        for (size_t t = 0; t < (size_t)q * p; ++t) supp[t * W + W - 1] = ((uint64_t)1 << (P % 64)) - 1;
    int32_t *rows = (int32_t *)malloc(sizeof(int32_t) * (size_t)N);
    int32_t *iden = (int32_t *)malloc(sizeof(int32_t) * (size_t)N);
    for (int r = 0; r < N; ++r) iden[r] = r;
    double *Xs = (double *)malloc(sizeof(double) * (size_t)N * P);
    double *Ys = (double *)malloc(sizeof(double) * (size_t)N * p);
    double *xm = (double *)malloc(sizeof(double) * (size_t)P);
    double *ym = (double *)malloc(sizeof(double) * (size_t)p);
    double *G = (double *)malloc(sizeof(double) * (size_t)P * P);
    double *C = (double *)malloc(sizeof(double) * (size_t)P * p);
    /* Model selection */
    for (int k = 0; k < B1; ++k) {
        orc_var_boot_rows(seed, k, N, L, rows);
        centred_sample(N, rows, P, Xl, Xs, xm, intercept);
        centred_sample(N, rows, p, Yl, Ys, ym, intercept);
        orc_gram(N, iden, P, Xs, P, p, Ys, p, G, C);
#pragma omp parallel for schedule(dynamic, 1) reduction(+ : bad)
        for (int e = 0; e < p; ++e) {
            double *b = (double *)calloc((size_t)P, sizeof(double));
            uint64_t *w = (uint64_t *)malloc(sizeof(uint64_t) * (size_t)W);
            for (int j = 0; j < q; ++j) {
                if (orc_lasso_cd(P, G, C + e, p, lam[j], tol, max_sweeps, b) < 0) ++bad;
                set_support(P, b, w);
                uint64_t *S = supp + ((size_t)j * p + e) * W;
                for (int t = 0; t < W; ++t) S[t] &= w[t];
            }
            free(b); free(w);
        }
    }
    /* Model estimation */
    int32_t *tr = (int32_t *)malloc(sizeof(int32_t) * (size_t)N);
    int32_t *ev = (int32_t *)malloc(sizeof(int32_t) * (size_t)N);
    double *fit = (double *)malloc(sizeof(double) * (size_t)q * p * P);
    double *fmu = (double *)malloc(sizeof(double) * (size_t)q * p);
    double *Lk = (double *)malloc(sizeof(double) * (size_t)q * p);
    double *acc = (double *)calloc((size_t)p * P, sizeof(double));
    double *macc = (double *)calloc((size_t)p, sizeof(double));
    for (int k = 0; k < B2; ++k) {
        int ntr = 0, nev = 0;
        orc_var_split_rows(seed, k, N, L, num, den, tr, &ntr, ev, &nev);
        centred_sample(ntr, tr, P, Xl, Xs, xm, intercept);
        centred_sample(ntr, tr, p, Yl, Ys, ym, intercept);
        orc_gram(ntr, iden, P, Xs, P, p, Ys, p, G, C);
#pragma omp parallel for schedule(dynamic, 1) reduction(+ : bad)
        for (int e = 0; e < p; ++e) {
            double *work = (double *)malloc(sizeof(double) * (size_t)P * P);
            double *bs = (double *)malloc(sizeof(double) * (size_t)P);
            int *idx = (int *)malloc(sizeof(int) * (size_t)P);
            for (int j = 0; j < q; ++j) {
                int s = support_list(P, supp + ((size_t)j * p + e) * W, idx);
                if (orc_ols_normal(P, G, C + e, p, s, idx, bs, work) != 0) ++bad;
                double *f = fit + ((size_t)j * p + e) * P;
                memset(f, 0, sizeof(double) * (size_t)P);
                double mu = ym[e];
                for (int a = 0; a < s; ++a) {
                    f[idx[a]] = bs[a];
                    mu -= xm[idx[a]] * bs[a];
                }
                fmu[(size_t)j * p + e] = intercept ? mu : 0.0;
                double Ls = 0.0;
                for (int r = 0; r < nev; ++r) {
                    const double *x = Xl + (size_t)ev[r] * P;
                    double res = Yl[(size_t)ev[r] * p + e] - fmu[(size_t)j * p + e];
                    for (int a = 0; a < s; ++a) res -= x[idx[a]] * bs[a];
                    Ls += res * res;
                }
                Lk[(size_t)j * p + e] = nev > 0 ? Ls / nev : 0.0;
            }
            free(work); free(bs); free(idx);
        }
        if (per_eq) {
            for (int e = 0; e < p; ++e) {
                int best = 0;
                for (int j = 0; j < q; ++j) {
                    const double Le = Lk[(size_t)j * p + e];
                    if (losses) losses[((size_t)k * q + j) * p + e] = Le;
                    if (Le < Lk[(size_t)best * p + e]) best = j;
                }
                jstar[(size_t)k * p + e] = best;
                for (int c = 0; c < P; ++c) acc[(size_t)e * P + c] += fit[((size_t)best * p + e) * P + c];
                macc[e] += fmu[(size_t)best * p + e];
            }
            continue;
        }
        int best = 0;
        double bestL = 0.0;
        for (int j = 0; j < q; ++j) {
            double s = 0.0;
            for (int e = 0; e < p; ++e) s += Lk[(size_t)j * p + e];
            if (losses) losses[(size_t)k * q + j] = s;
            if (j == 0 || s < bestL) { bestL = s; best = j; }
        }
        jstar[k] = best;
        for (size_t t = 0; t < (size_t)p * P; ++t) acc[t] += fit[(size_t)best * p * P + t];
        for (int e = 0; e < p; ++e) macc[e] += fmu[(size_t)best * p + e];
    }
    /* A_l[e][m] = beta*_e[(l-1) p + m] (Alg. 2, last steps) */
    for (int l = 0; l < d; ++l)
        for (int e = 0; e < p; ++e)
            for (int m = 0; m < p; ++m)
                A_out[((size_t)l * p + e) * p + m] = acc[(size_t)e * P + (size_t)l * p + m] / B2;
    for (int e = 0; e < p; ++e) mu_out[e] = macc[e] / B2;
    free(Xl); free(Yl); free(rows); free(iden); free(Xs); free(Ys); free(xm); free(ym); free(G);
    free(C); free(tr); free(ev); free(fit); free(fmu); free(Lk); free(acc); free(macc);
    return bad ? -1 : 0;
}
