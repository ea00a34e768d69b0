/*
 * oracle.c -- plain, slow, CPU FP64 reference ("oracle") for the
 * tridiagonal-to-banded eigenvector back-transformation of the two-stage
 * Hermitian eigensolver (Yu et al., "GPU-Acceleration of the ELPA2
 * Distributed Eigensolver ...", Sec. 2.2), and for the pipeline that
 * produces its inputs.
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product path links, loads or
 * calls this file; only the test-suite, the smoke check and the CPU-baseline
 * leg of the benchmark do.  It shares no source, header, table or helper
 * with the GPU library.
 *
 * Conventions (all 0-based):
 *   n      matrix order (paper: N), b semi-bandwidth (paper: b)
 *   stage  s = 0 .. n-3           (paper: stage i = s+1, Sec. 2.2.1)
 *   slot   j = 0 .. S_s - 1       (paper: sweep j+1 of stage i)
 *   S_s    = ceil((n-s-2)/b)      sweeps of stage s
 *   reflector (s,j) acts on rows [r0, r0+len) with r0 = s+1+j*b,
 *   len = min(b, n-r0) (>= 2 for every existing reflector).
 *   Generation order is stage-major, slot-minor; the back-transformation
 *   applies the reflectors in exactly the reverse order (Sec. 2.2.2).
 *
 *   Householder reflector H = I - tau v v^H, v[0] = 1 (Eq. householder);
 *   hh_v is K x b, reflector-contiguous, zero padded beyond len;
 *   hh_tau has K entries.
 *
 * Complex arithmetic uses C99 double complex.  Every routine is written for
 * clarity, not speed; the only parallelism is OpenMP over independent
 * eigenvector columns (Sec. 2.2.2: eigenvectors are back-transformed
 * independently) and over independent rows of the QL eigenvector matrix.
 */
#include <complex.h>
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#include <omp.h>

typedef double complex zc;

/* threads the OpenMP loops below use */
int orc_num_threads(void) { return omp_get_max_threads(); }

#define ORC_OK 0
#define ORC_EARG (-1)
#define ORC_ENOMEM (-2)
#define ORC_ENOCONV (-3)

/* ------------------------------------------------------------------------
 * Reflector geometry (Sec. 2.2.1, Figs. step2 and step4).
 * ---------------------------------------------------------------------- */

/* Number of sweeps in stage s (0-based).  The paper writes (N-i)/b for
 * stage i; every sweep must produce a reflector of length >= 2 and the
 * last sweep of a stage may be shorter than b, which gives
 * ceil((n-s-2)/b) with s = i-1 (the fourth stage of N=17, b=4 has 3). */
int64_t orc_sweeps_in_stage(int64_t n, int64_t b, int64_t s)
{
    /* b = 1: the band matrix is already tridiagonal; no reflector has the
     * length >= 2 that every sweep needs, so there are none. */
    if (n < 3 || b < 2 || s < 0 || s > n - 3) return 0;
    return (n - s - 2 + b - 1) / b;
}

int64_t orc_num_reflectors(int64_t n, int64_t b)
{
    int64_t K = 0;
    for (int64_t s = 0; s <= n - 3; ++s) K += orc_sweeps_in_stage(n, b, s);
    return K;
}

/* Fill per-reflector (stage, slot, first row, length) in generation order. */
int orc_reflector_table(int64_t n, int64_t b, int64_t *stage, int64_t *slot,
                        int64_t *row0, int64_t *len)
{
    if (n < 0 || b < 1) return ORC_EARG;
    int64_t k = 0;
    for (int64_t s = 0; s <= n - 3; ++s) {
        int64_t S = orc_sweeps_in_stage(n, b, s);
        for (int64_t j = 0; j < S; ++j) {
            int64_t r0 = s + 1 + j * b;
            int64_t l = n - r0 < b ? n - r0 : b;
            if (stage) stage[k] = s;
            if (slot) slot[k] = j;
            if (row0) row0[k] = r0;
            if (len) len[k] = l;
            ++k;
        }
    }
    return ORC_OK;
}

/* ------------------------------------------------------------------------
 * Householder vector generation, LAPACK "larfg" convention (the standard
 * Householder method the paper cites for Eq. householder).
 * Given x = (alpha, x2) of length m, find beta (real), tau and v = (1, w)
 * such that  (I - tau v v^H)^H x = beta e1.
 * On exit x is overwritten by v.
 * ---------------------------------------------------------------------- */
void orc_larfg_d(int64_t m, double *x, double *tau, double *beta)
{
    double alpha = x[0], xn2 = 0.0;
    for (int64_t i = 1; i < m; ++i) xn2 += x[i] * x[i];
    if (xn2 == 0.0) {            /* nothing to annihilate: H = I */
        *tau = 0.0;
        *beta = alpha;
        x[0] = 1.0;
        return;
    }
    double nrm = sqrt(alpha * alpha + xn2);
    double bt = alpha >= 0.0 ? -nrm : nrm;    /* beta = -sign(alpha) ||x|| */
    *tau = (bt - alpha) / bt;
    double scale = 1.0 / (alpha - bt);
    for (int64_t i = 1; i < m; ++i) x[i] *= scale;
    x[0] = 1.0;
    *beta = bt;
}

void orc_larfg_z(int64_t m, zc *x, zc *tau, double *beta)
{
    zc alpha = x[0];
    double xn2 = 0.0;
    for (int64_t i = 1; i < m; ++i) xn2 += creal(x[i] * conj(x[i]));
    if (xn2 == 0.0 && cimag(alpha) == 0.0) {
        *tau = 0.0;
        *beta = creal(alpha);
        x[0] = 1.0;
        return;
    }
    double ar = creal(alpha), ai = cimag(alpha);
    double nrm = sqrt(ar * ar + ai * ai + xn2);
    double bt = ar >= 0.0 ? -nrm : nrm;
    *tau = ((bt - ar) - I * ai) / bt;          /* (beta - alpha) / beta */
    zc scale = 1.0 / (alpha - bt);
    for (int64_t i = 1; i < m; ++i) x[i] *= scale;
    x[0] = 1.0;
    *beta = bt;
}

/* ------------------------------------------------------------------------
 * Hermitian band matrix in lower band storage with W stored subdiagonals:
 * element (i,k), i >= k, i-k <= W lives at ab[(i-k) + k*(W+1)].
 * ---------------------------------------------------------------------- */
typedef struct {
    int64_t n, W;
    double *re;     /* real case storage */
    zc *cz;         /* complex case storage */
    double dropped; /* largest |value| that fell outside the stored band */
} band_t;

static int in_band(const band_t *B, int64_t i, int64_t k)
{
    return i >= k && i - k <= B->W && i < B->n && k >= 0;
}

/* full Hermitian access: returns B(i,k) for any (i,k); zero outside band */
static double bget_d(const band_t *B, int64_t i, int64_t k)
{
    if (i < k) { int64_t t = i; i = k; k = t; }
    return in_band(B, i, k) ? B->re[(i - k) + k * (B->W + 1)] : 0.0;
}

static zc bget_z(const band_t *B, int64_t i, int64_t k)
{
    if (i >= k) return in_band(B, i, k) ? B->cz[(i - k) + k * (B->W + 1)] : 0.0;
    return in_band(B, k, i) ? conj(B->cz[(k - i) + i * (B->W + 1)]) : 0.0;
}

/* store into the lower triangle (i >= k required); outside the stored band
 * the value must vanish: its magnitude is recorded in B->dropped */
static void bset_d(band_t *B, int64_t i, int64_t k, double v)
{
    if (in_band(B, i, k)) B->re[(i - k) + k * (B->W + 1)] = v;
    else if (fabs(v) > B->dropped) B->dropped = fabs(v);
}

static void bset_z(band_t *B, int64_t i, int64_t k, zc v)
{
    if (in_band(B, i, k)) B->cz[(i - k) + k * (B->W + 1)] = v;
    else if (cabs(v) > B->dropped) B->dropped = cabs(v);
}

/* ------------------------------------------------------------------------
 * Banded-to-tridiagonal reduction by bulge chasing (Sec. 2.2.1, Eq.
 * 2stage_fwd2, Fig. step2).  Stage s, sweep j annihilates column c of the
 * current matrix over rows [r0, r0+len): c = s for the first sweep (the
 * stage's own column), and c = r0 - b for later sweeps (the first column of
 * the bulge created by the previous sweep).  Each step is the similarity
 * B <- H^H B H with H = I - tau v v^H, applied to every stored entry of
 * rows/columns [r0, r0+len).  Every (v, tau) is stored in generation order
 * in a separate array (Fig. step4 caption).
 *
 * ab_in: input band, LAPACK lower layout ab_in[d + k*ldab] = B(k+d, k),
 *        d = 0..b.
 * d_out: n real diagonal entries of T; e_out: n-1 subdiagonal entries
 *        (real case: double; complex case: zc -- only e[n-2] stays complex).
 * offband: on exit, the largest |T(i,k)| with i-k >= 2 (should be ~eps).
 * dropped: on exit, the largest value that fell outside the 2b work band.
 * ---------------------------------------------------------------------- */
static void apply_left_d(int64_t len, const double *v, double tau, double *y)
{   /* y <- H^H y = y - tau v (v^T y) */
    double dot = 0.0;
    for (int64_t i = 0; i < len; ++i) dot += v[i] * y[i];
    for (int64_t i = 0; i < len; ++i) y[i] -= tau * dot * v[i];
}

static void apply_right_d(int64_t len, const double *v, double tau, double *y)
{   /* row vector y <- y H = y - tau (y v) v^T */
    double dot = 0.0;
    for (int64_t i = 0; i < len; ++i) dot += y[i] * v[i];
    for (int64_t i = 0; i < len; ++i) y[i] -= tau * dot * v[i];
}

static void apply_left_z(int64_t len, const zc *v, zc tau, zc *y)
{   /* y <- H^H y = y - conj(tau) v (v^H y) */
    zc dot = 0.0;
    for (int64_t i = 0; i < len; ++i) dot += conj(v[i]) * y[i];
    for (int64_t i = 0; i < len; ++i) y[i] -= conj(tau) * dot * v[i];
}

static void apply_right_z(int64_t len, const zc *v, zc tau, zc *y)
{   /* row vector y <- y H = y - tau (y v) v^H */
    zc dot = 0.0;
    for (int64_t i = 0; i < len; ++i) dot += y[i] * v[i];
    for (int64_t i = 0; i < len; ++i) y[i] -= tau * dot * conj(v[i]);
}

int orc_band_to_tridi_d(int64_t n, int64_t b, const double *ab_in, int64_t ldab,
                        double *d_out, double *e_out, double *hh_v,
                        double *hh_tau, double *offband, double *dropped)
{
    if (n < 1 || b < 1 || ldab < b + 1) return ORC_EARG;
    band_t B = {n, 2 * b, NULL, NULL, 0.0};
    B.re = calloc((size_t)n * (B.W + 1), sizeof(double));
    double *x = malloc(sizeof(double) * (b + 1));
    double *blk = malloc(sizeof(double) * b * b);
    if (!B.re || !x || !blk) { free(B.re); free(x); free(blk); return ORC_ENOMEM; }
    for (int64_t k = 0; k < n; ++k)
        for (int64_t dd = 0; dd <= b && k + dd < n; ++dd)
            B.re[dd + k * (B.W + 1)] = ab_in[dd + k * ldab];

    int64_t kref = 0;
    for (int64_t s = 0; s <= n - 3; ++s) {
        int64_t S = orc_sweeps_in_stage(n, b, s);
        for (int64_t j = 0; j < S; ++j, ++kref) {
            int64_t r0 = s + 1 + j * b;
            int64_t len = n - r0 < b ? n - r0 : b;
            int64_t c = (j == 0) ? s : r0 - b;
            double tau, beta;
            for (int64_t i = 0; i < len; ++i) x[i] = bget_d(&B, r0 + i, c);
            orc_larfg_d(len, x, &tau, &beta);
            double *v = hh_v + kref * b;
            for (int64_t i = 0; i < b; ++i) v[i] = i < len ? x[i] : 0.0;
            hh_tau[kref] = tau;
            /* the annihilated column */
            bset_d(&B, r0, c, beta);
            for (int64_t i = 1; i < len; ++i) bset_d(&B, r0 + i, c, 0.0);
            /* left update of the other columns left of the block */
            for (int64_t k = r0 - B.W > 0 ? r0 - B.W : 0; k < r0; ++k) {
                if (k == c) continue;
                for (int64_t i = 0; i < len; ++i) x[i] = bget_d(&B, r0 + i, k);
                apply_left_d(len, v, tau, x);
                for (int64_t i = 0; i < len; ++i) bset_d(&B, r0 + i, k, x[i]);
            }
            /* two-sided update of the diagonal block */
            for (int64_t p = 0; p < len; ++p)
                for (int64_t q = 0; q < len; ++q)
                    blk[p + q * len] = bget_d(&B, r0 + p, r0 + q);
            for (int64_t q = 0; q < len; ++q) apply_left_d(len, v, tau, blk + q * len);
            for (int64_t p = 0; p < len; ++p) {
                for (int64_t q = 0; q < len; ++q) x[q] = blk[p + q * len];
                apply_right_d(len, v, tau, x);
                for (int64_t q = 0; q < len; ++q) blk[p + q * len] = x[q];
            }
            for (int64_t q = 0; q < len; ++q)
                for (int64_t p = q; p < len; ++p)
                    bset_d(&B, r0 + p, r0 + q, blk[p + q * len]);
            /* right update of the rows below the block */
            for (int64_t i = r0 + len; i < n && i < r0 + len + B.W; ++i) {
                for (int64_t q = 0; q < len; ++q) x[q] = bget_d(&B, i, r0 + q);
                apply_right_d(len, v, tau, x);
                for (int64_t q = 0; q < len; ++q) bset_d(&B, i, r0 + q, x[q]);
            }
        }
    }
    double off = 0.0;
    for (int64_t k = 0; k < n; ++k) {
        d_out[k] = bget_d(&B, k, k);
        if (k + 1 < n) e_out[k] = bget_d(&B, k + 1, k);
        for (int64_t dd = 2; dd <= B.W && k + dd < n; ++dd) {
            double a = fabs(B.re[dd + k * (B.W + 1)]);
            if (a > off) off = a;
        }
    }
    if (offband) *offband = off;
    if (dropped) *dropped = B.dropped;
    free(B.re); free(x); free(blk);
    return ORC_OK;
}

int orc_band_to_tridi_z(int64_t n, int64_t b, const zc *ab_in, int64_t ldab,
                        double *d_out, zc *e_out, zc *hh_v, zc *hh_tau,
                        double *offband, double *dropped)
{
    if (n < 1 || b < 1 || ldab < b + 1) return ORC_EARG;
    band_t B = {n, 2 * b, NULL, NULL, 0.0};
    B.cz = calloc((size_t)n * (B.W + 1), sizeof(zc));
    zc *x = malloc(sizeof(zc) * (b + 1));
    zc *blk = malloc(sizeof(zc) * b * b);
    if (!B.cz || !x || !blk) { free(B.cz); free(x); free(blk); return ORC_ENOMEM; }
    for (int64_t k = 0; k < n; ++k)
        for (int64_t dd = 0; dd <= b && k + dd < n; ++dd)
            B.cz[dd + k * (B.W + 1)] = ab_in[dd + k * ldab];

    int64_t kref = 0;
    for (int64_t s = 0; s <= n - 3; ++s) {
        int64_t S = orc_sweeps_in_stage(n, b, s);
        for (int64_t j = 0; j < S; ++j, ++kref) {
            int64_t r0 = s + 1 + j * b;
            int64_t len = n - r0 < b ? n - r0 : b;
            int64_t c = (j == 0) ? s : r0 - b;
            zc tau;
            double beta;
            for (int64_t i = 0; i < len; ++i) x[i] = bget_z(&B, r0 + i, c);
            orc_larfg_z(len, x, &tau, &beta);
            zc *v = hh_v + kref * b;
            for (int64_t i = 0; i < b; ++i) v[i] = i < len ? x[i] : 0.0;
            hh_tau[kref] = tau;
            bset_z(&B, r0, c, beta);
            for (int64_t i = 1; i < len; ++i) bset_z(&B, r0 + i, c, 0.0);
            for (int64_t k = r0 - B.W > 0 ? r0 - B.W : 0; k < r0; ++k) {
                if (k == c) continue;
                for (int64_t i = 0; i < len; ++i) x[i] = bget_z(&B, r0 + i, k);
                apply_left_z(len, v, tau, x);
                for (int64_t i = 0; i < len; ++i) bset_z(&B, r0 + i, k, x[i]);
            }
            for (int64_t p = 0; p < len; ++p)
                for (int64_t q = 0; q < len; ++q)
                    blk[p + q * len] = bget_z(&B, r0 + p, r0 + q);
            for (int64_t q = 0; q < len; ++q) apply_left_z(len, v, tau, blk + q * len);
            for (int64_t p = 0; p < len; ++p) {
                for (int64_t q = 0; q < len; ++q) x[q] = blk[p + q * len];
                apply_right_z(len, v, tau, x);
                for (int64_t q = 0; q < len; ++q) blk[p + q * len] = x[q];
            }
            for (int64_t q = 0; q < len; ++q)
                for (int64_t p = q; p < len; ++p)
                    bset_z(&B, r0 + p, r0 + q, blk[p + q * len]);
            for (int64_t i = r0 + len; i < n && i < r0 + len + B.W; ++i) {
                for (int64_t q = 0; q < len; ++q) x[q] = bget_z(&B, i, r0 + q);
                apply_right_z(len, v, tau, x);
                for (int64_t q = 0; q < len; ++q) bset_z(&B, i, r0 + q, x[q]);
            }
        }
    }
    double off = 0.0;
    for (int64_t k = 0; k < n; ++k) {
        d_out[k] = creal(bget_z(&B, k, k));
        if (k + 1 < n) e_out[k] = bget_z(&B, k + 1, k);
        for (int64_t dd = 2; dd <= B.W && k + dd < n; ++dd) {
            double a = cabs(B.cz[dd + k * (B.W + 1)]);
            if (a > off) off = a;
        }
    }
    if (offband) *offband = off;
    if (dropped) *dropped = B.dropped;
    free(B.cz); free(x); free(blk);
    return ORC_OK;
}

/* ------------------------------------------------------------------------
 * Tridiagonal-to-banded back-transformation, Eq. 2stage_bkwd1 (Y = Q^* X),
 * Sec. 2.2.2.  One reflector at a time, in exactly the reverse of the
 * generation order, each applied to every column by Eq. kernel:
 *     x <- x - tau v (v^H x)      on rows [r0, r0+len).
 * Columns [c0, c1) of Z (column-major, leading dimension ldz) are updated in
 * place.  Columns are independent, so they are spread over OpenMP threads.
 * ---------------------------------------------------------------------- */
int orc_back_transform_d(int64_t n, int64_t b, int64_t c0, int64_t c1,
                         const double *hh_v, const double *hh_tau, double *Z,
                         int64_t ldz)
{
    if (n < 0 || b < 1 || c0 < 0 || c1 < c0 || ldz < (n > 1 ? n : 1)) return ORC_EARG;
    int64_t K = orc_num_reflectors(n, b);
    int64_t *r0 = malloc(sizeof(int64_t) * (K + 1));
    int64_t *ln = malloc(sizeof(int64_t) * (K + 1));
    if (!r0 || !ln) { free(r0); free(ln); return ORC_ENOMEM; }
    orc_reflector_table(n, b, NULL, NULL, r0, ln);
#pragma omp parallel for schedule(dynamic, 1)
    for (int64_t c = c0; c < c1; ++c) {
        double *z = Z + c * ldz;
        for (int64_t k = K - 1; k >= 0; --k) {
            const double *v = hh_v + k * b;
            double *zz = z + r0[k];
            double d = 0.0;
            for (int64_t i = 0; i < ln[k]; ++i) d += v[i] * zz[i];
            double a = hh_tau[k] * d;
            for (int64_t i = 0; i < ln[k]; ++i) zz[i] -= a * v[i];
        }
    }
    free(r0); free(ln);
    return ORC_OK;
}

int orc_back_transform_z(int64_t n, int64_t b, int64_t c0, int64_t c1,
                         const zc *hh_v, const zc *hh_tau, zc *Z, int64_t ldz)
{
    if (n < 0 || b < 1 || c0 < 0 || c1 < c0 || ldz < (n > 1 ? n : 1)) return ORC_EARG;
    int64_t K = orc_num_reflectors(n, b);
    int64_t *r0 = malloc(sizeof(int64_t) * (K + 1));
    int64_t *ln = malloc(sizeof(int64_t) * (K + 1));
    if (!r0 || !ln) { free(r0); free(ln); return ORC_ENOMEM; }
    orc_reflector_table(n, b, NULL, NULL, r0, ln);
#pragma omp parallel for schedule(dynamic, 1)
    for (int64_t c = c0; c < c1; ++c) {
        zc *z = Z + c * ldz;
        for (int64_t k = K - 1; k >= 0; --k) {
            const zc *v = hh_v + k * b;
            zc *zz = z + r0[k];
            zc d = 0.0;
            for (int64_t i = 0; i < ln[k]; ++i) d += conj(v[i]) * zz[i];
            zc a = hh_tau[k] * d;
            for (int64_t i = 0; i < ln[k]; ++i) zz[i] -= a * v[i];
        }
    }
    free(r0); free(ln);
    return ORC_OK;
}

/* Same reflectors applied conjugate-transposed, in generation order:
 * Z <- Q Z = H_{K-1}^H ... H_0^H Z.  Undoes orc_back_transform_*. */
int orc_apply_q_z(int64_t n, int64_t b, int64_t c0, int64_t c1, const zc *hh_v,
                  const zc *hh_tau, zc *Z, int64_t ldz)
{
    if (n < 0 || b < 1 || c0 < 0 || c1 < c0 || ldz < (n > 1 ? n : 1)) return ORC_EARG;
    int64_t K = orc_num_reflectors(n, b);
    int64_t *r0 = malloc(sizeof(int64_t) * (K + 1));
    int64_t *ln = malloc(sizeof(int64_t) * (K + 1));
    if (!r0 || !ln) { free(r0); free(ln); return ORC_ENOMEM; }
    orc_reflector_table(n, b, NULL, NULL, r0, ln);
#pragma omp parallel for schedule(dynamic, 1)
    for (int64_t c = c0; c < c1; ++c) {
        zc *z = Z + c * ldz;
        for (int64_t k = 0; k < K; ++k) {
            const zc *v = hh_v + k * b;
            zc *zz = z + r0[k];
            zc d = 0.0;
            for (int64_t i = 0; i < ln[k]; ++i) d += conj(v[i]) * zz[i];
            zc a = conj(hh_tau[k]) * d;
            for (int64_t i = 0; i < ln[k]; ++i) zz[i] -= a * v[i];
        }
    }
    free(r0); free(ln);
    return ORC_OK;
}

/* ------------------------------------------------------------------------
 * Adjoint (reverse-mode derivative) of the real back-transformation
 *     Z_out = H_0 H_1 ... H_{K-1} Z_in,   H_k = I - tau_k v_k v_k^T
 * (Eq. 2stage_bkwd1 with real reflectors).  Given G = dL/dZ_out, return
 * dL/dZ_in (in G), dL/dv (K x b, zero beyond len) and dL/dtau (K).
 *
 * Plain reverse mode, one column at a time (columns are independent in Z;
 * only dv and dtau sum over them):
 *   forward  k = K-1 .. 0: record the rows [r0, r0+len) of the column as
 *            they enter H_k (the tape), then apply H_k;
 *   reverse  k = 0 .. K-1, with z = tape entry k, g = current gradient rows:
 *              gk = v.g,  wk = v.z
 *              dtau_k += -gk wk
 *              dv_k   += -tau_k (wk g + gk z)
 *              g      <- g - tau_k gk v        (= H_k^T g)
 * Derivation: the column update z' = z - tau v (v.z) has
 *   dL/dz = g - tau v (v.g),  dL/dtau = -(v.z)(v.g),
 *   dL/dv = -tau ((v.z) g + (v.g) z).
 * Per-thread accumulators are summed in thread order at the end.
 * ---------------------------------------------------------------------- */
int orc_adjoint_d(int64_t n, int64_t b, int64_t nev, const double *hh_v,
                  const double *hh_tau, const double *Zin, int64_t ldz, double *G,
                  int64_t ldg, double *dv, double *dtau)
{
    if (n < 0 || b < 1 || nev < 0 || ldz < (n > 1 ? n : 1) || ldg < (n > 1 ? n : 1))
        return ORC_EARG;
    const int64_t K = orc_num_reflectors(n, b);
    for (int64_t i = 0; i < K * b; ++i) dv[i] = 0.0;
    for (int64_t k = 0; k < K; ++k) dtau[k] = 0.0;
    if (K == 0 || nev == 0) return ORC_OK;
    int64_t *r0 = malloc(sizeof(int64_t) * K);
    int64_t *ln = malloc(sizeof(int64_t) * K);
    int64_t *toff = malloc(sizeof(int64_t) * (K + 1));
    if (!r0 || !ln || !toff) { free(r0); free(ln); free(toff); return ORC_ENOMEM; }
    orc_reflector_table(n, b, NULL, NULL, r0, ln);
    toff[0] = 0;
    for (int64_t k = 0; k < K; ++k) toff[k + 1] = toff[k] + ln[k];
    const int nt = omp_get_max_threads();
    double *acc_v = calloc((size_t)nt * K * b, sizeof(double));
    double *acc_t = calloc((size_t)nt * K, sizeof(double));
    int fail = !acc_v || !acc_t;
    if (!fail) {
#pragma omp parallel num_threads(nt)
        {
            const int me = omp_get_thread_num();
            double *av = acc_v + (size_t)me * K * b, *at = acc_t + (size_t)me * K;
            double *tape = malloc(sizeof(double) * toff[K]);
            double *z = malloc(sizeof(double) * (n > 0 ? n : 1));
            if (!tape || !z) {
#pragma omp atomic write
                fail = 1;
            } else {
#pragma omp for schedule(static)
                for (int64_t c = 0; c < nev; ++c) {
                    for (int64_t i = 0; i < n; ++i) z[i] = Zin[c * ldz + i];
                    for (int64_t k = K - 1; k >= 0; --k) {
                        const double *v = hh_v + k * b;
                        double *zz = z + r0[k];
                        double d = 0.0;
                        for (int64_t i = 0; i < ln[k]; ++i) {
                            tape[toff[k] + i] = zz[i];
                            d += v[i] * zz[i];
                        }
                        const double a = hh_tau[k] * d;
                        for (int64_t i = 0; i < ln[k]; ++i) zz[i] -= a * v[i];
                    }
                    double *g = G + c * ldg;
                    for (int64_t k = 0; k < K; ++k) {
                        const double *v = hh_v + k * b, *zk = tape + toff[k];
                        double *gg = g + r0[k];
                        double gk = 0.0, wk = 0.0;
                        for (int64_t i = 0; i < ln[k]; ++i) {
                            gk += v[i] * gg[i];
                            wk += v[i] * zk[i];
                        }
                        const double t = hh_tau[k];
                        at[k] -= gk * wk;
                        for (int64_t i = 0; i < ln[k]; ++i) av[k * b + i] -= t * (wk * gg[i] + gk * zk[i]);
                        for (int64_t i = 0; i < ln[k]; ++i) gg[i] -= t * gk * v[i];
                    }
                }
            }
            free(tape);
            free(z);
        }
    }
    if (!fail) {
        for (int th = 0; th < nt; ++th) {
            for (int64_t i = 0; i < K * b; ++i) dv[i] += acc_v[(size_t)th * K * b + i];
            for (int64_t k = 0; k < K; ++k) dtau[k] += acc_t[(size_t)th * K + k];
        }
    }
    free(acc_v); free(acc_t); free(r0); free(ln); free(toff);
    return fail ? ORC_ENOMEM : ORC_OK;
}

/* ------------------------------------------------------------------------
 * Adjoint of the complex back-transformation
 *     Z_out = H_0 H_1 ... H_{K-1} Z_in,   H_k = I - tau_k v_k v_k^H
 * (Eq. 2stage_bkwd1 with complex reflectors), for a real loss L, in the
 * convention of the conjugate Wirtinger derivative that PyTorch uses: the
 * gradient of x is grad_x with  dL = Re sum conj(grad_x) dx  for every
 * complex perturbation dx (the steepest-ascent direction).
 * Chain rule for y = f(x, conj x):  grad_x = J^H grad_y + J'^T conj(grad_y)
 * with J = dy/dx, J' = dy/d(conj x).  For one column update
 *     z' = z - tau v (v^H z),   w = v^H z,  gamma = v^H g  (g = grad_z'):
 *   grad_z   = g - conj(tau) v gamma              (= H^H g)
 *   grad_tau = -conj(w) gamma
 *   grad_v   = -conj(tau) conj(w) g - tau conj(gamma) z
 *     (the first term from v itself, the second from v^H, through which
 *     conj(v) enters).
 * The real adjoint is the special case with every imaginary part zero.
 * Same sweep structure as orc_adjoint_d: per column a forward pass that
 * records the rows entering each reflector (the tape), then the reflectors
 * in generation order; dv, dtau summed over columns, per thread, threads in
 * order.
 * ---------------------------------------------------------------------- */
int orc_adjoint_z(int64_t n, int64_t b, int64_t nev, const zc *hh_v, const zc *hh_tau,
                  const zc *Zin, int64_t ldz, zc *G, int64_t ldg, zc *dv, zc *dtau)
{
    if (n < 0 || b < 1 || nev < 0 || ldz < (n > 1 ? n : 1) || ldg < (n > 1 ? n : 1))
        return ORC_EARG;
    const int64_t K = orc_num_reflectors(n, b);
    for (int64_t i = 0; i < K * b; ++i) dv[i] = 0.0;
    for (int64_t k = 0; k < K; ++k) dtau[k] = 0.0;
    if (K == 0 || nev == 0) return ORC_OK;
    int64_t *r0 = malloc(sizeof(int64_t) * K);
    int64_t *ln = malloc(sizeof(int64_t) * K);
    int64_t *toff = malloc(sizeof(int64_t) * (K + 1));
    if (!r0 || !ln || !toff) { free(r0); free(ln); free(toff); return ORC_ENOMEM; }
    orc_reflector_table(n, b, NULL, NULL, r0, ln);
    toff[0] = 0;
    for (int64_t k = 0; k < K; ++k) toff[k + 1] = toff[k] + ln[k];
    const int nt = omp_get_max_threads();
    zc *acc_v = calloc((size_t)nt * K * b, sizeof(zc));
    zc *acc_t = calloc((size_t)nt * K, sizeof(zc));
    int fail = !acc_v || !acc_t;
    if (!fail) {
#pragma omp parallel num_threads(nt)
        {
            const int me = omp_get_thread_num();
            zc *av = acc_v + (size_t)me * K * b, *at = acc_t + (size_t)me * K;
            zc *tape = malloc(sizeof(zc) * toff[K]);
            zc *z = malloc(sizeof(zc) * (n > 0 ? n : 1));
            if (!tape || !z) {
#pragma omp atomic write
                fail = 1;
            } else {
#pragma omp for schedule(static)
                for (int64_t c = 0; c < nev; ++c) {
                    for (int64_t i = 0; i < n; ++i) z[i] = Zin[c * ldz + i];
                    for (int64_t k = K - 1; k >= 0; --k) {
                        const zc *v = hh_v + k * b;
                        zc *zz = z + r0[k];
                        zc d = 0.0;
                        for (int64_t i = 0; i < ln[k]; ++i) {
                            tape[toff[k] + i] = zz[i];
                            d += conj(v[i]) * zz[i];
                        }
                        const zc a = hh_tau[k] * d;
                        for (int64_t i = 0; i < ln[k]; ++i) zz[i] -= a * v[i];
                    }
                    zc *g = G + c * ldg;
                    for (int64_t k = 0; k < K; ++k) {
                        const zc *v = hh_v + k * b, *zk = tape + toff[k];
                        zc *gg = g + r0[k];
                        zc gam = 0.0, w = 0.0;
                        for (int64_t i = 0; i < ln[k]; ++i) {
                            gam += conj(v[i]) * gg[i];
                            w += conj(v[i]) * zk[i];
                        }
                        const zc t = hh_tau[k];
                        at[k] -= conj(w) * gam;
                        for (int64_t i = 0; i < ln[k]; ++i)
                            av[k * b + i] -= conj(t) * conj(w) * gg[i] + t * conj(gam) * zk[i];
                        for (int64_t i = 0; i < ln[k]; ++i) gg[i] -= conj(t) * gam * v[i];
                    }
                }
            }
            free(tape);
            free(z);
        }
    }
    if (!fail) {
        for (int th = 0; th < nt; ++th) {
            for (int64_t i = 0; i < K * b; ++i) dv[i] += acc_v[(size_t)th * K * b + i];
            for (int64_t k = 0; k < K; ++k) dtau[k] += acc_t[(size_t)th * K + k];
        }
    }
    free(acc_v); free(acc_t); free(r0); free(ln); free(toff);
    return fail ? ORC_ENOMEM : ORC_OK;
}

/* ------------------------------------------------------------------------
 * Symmetric tridiagonal eigensolver, Eq. 2stage_solve, by the implicit QL
 * algorithm with Wilkinson shift, in the published formulation of
 * Bowdler, Martin, Reinsch and Wilkinson ("The QR and QL algorithms for
 * symmetric matrices", Numer. Math. 11, 1968: the Handbook routine tql2, as
 * restated in textbook form, e.g. Numerical Recipes' tqli): a small
 * subdiagonal splits the matrix, the shift is the eigenvalue of the leading
 * 2x2 block nearer d[l], and one sweep of plane rotations runs from the
 * bottom of the unreduced block up (theory: Golub & Van Loan, Sec. 8.3).
 * The paper itself uses divide and conquer, which reaches the same
 * eigenpairs.
 * d (n) diagonal, e (n-1) subdiagonal (e[i] couples rows i and i+1).
 * On exit d holds the eigenvalues in ascending order and X (n x n,
 * column-major, ldx) the orthonormal eigenvectors in the same order.
 * The plane rotations of each QL sweep are recorded and then applied to
 * the rows of the eigenvector matrix in parallel (each row is independent).
 * ---------------------------------------------------------------------- */
int orc_tridi_ql(int64_t n, double *d, const double *e_in, double *X, int64_t ldx)
{
    if (n < 1 || ldx < n) return ORC_EARG;
    double *e = calloc(n, sizeof(double));
    double *R = calloc((size_t)n * n, sizeof(double)); /* row-major work copy */
    double *rc = malloc(sizeof(double) * n), *rs = malloc(sizeof(double) * n);
    int64_t *ri = malloc(sizeof(int64_t) * n);
    if (!e || !R || !rc || !rs || !ri) {
        free(e); free(R); free(rc); free(rs); free(ri);
        return ORC_ENOMEM;
    }
    for (int64_t i = 0; i + 1 < n; ++i) e[i] = e_in[i];
    for (int64_t i = 0; i < n; ++i) R[i * n + i] = 1.0;
    const double eps = 0x1p-52;
    int status = ORC_OK;

    for (int64_t l = 0; l < n && status == ORC_OK; ++l) {
        for (int iter = 0;; ++iter) {
            /* the unreduced block starting at l ends at m */
            int64_t m = l;
            while (m + 1 < n) {
                double dd = fabs(d[m]) + fabs(d[m + 1]);
                if (fabs(e[m]) <= eps * dd) break;
                ++m;
            }
            if (m == l) break;
            if (iter == 100) { status = ORC_ENOCONV; break; }
            /* Wilkinson shift from the leading 2x2 block */
            double g = (d[l + 1] - d[l]) / (2.0 * e[l]);
            double r = hypot(g, 1.0);
            g = d[m] - d[l] + e[l] / (g + (g >= 0.0 ? r : -r));
            double sn = 1.0, cs = 1.0, p = 0.0;
            int64_t nrot = 0;
            int early = 0;
            /* chase the bulge from the bottom of the block up to row l;
             * e has a spare slot e[n-1] so that e[i+1] is always valid */
            for (int64_t i = m - 1; i >= l; --i) {
                double f = sn * e[i], h = cs * e[i];
                r = hypot(f, g);
                e[i + 1] = r;
                if (r == 0.0) {          /* the block splits: deflate */
                    d[i + 1] -= p;
                    e[m] = 0.0;
                    early = 1;
                    break;
                }
                sn = f / r;
                cs = g / r;
                g = d[i + 1] - p;
                r = (d[i] - g) * sn + 2.0 * cs * h;
                p = sn * r;
                d[i + 1] = g + p;
                g = cs * r - h;
                rc[nrot] = cs; rs[nrot] = sn; ri[nrot] = i; ++nrot;
            }
            /* rotate eigenvector columns (i, i+1) in recorded order */
#pragma omp parallel for schedule(static)
            for (int64_t row = 0; row < n; ++row) {
                double *zr = R + row * n;
                for (int64_t q = 0; q < nrot; ++q) {
                    int64_t c = ri[q];
                    double f = zr[c + 1];
                    zr[c + 1] = rs[q] * zr[c] + rc[q] * f;
                    zr[c] = rc[q] * zr[c] - rs[q] * f;
                }
            }
            if (early) continue;
            d[l] -= p;
            e[l] = g;
            e[m] = 0.0;
        }
    }
    if (status == ORC_OK) {
        /* sort ascending (selection sort; n is modest) */
        int64_t *perm = malloc(sizeof(int64_t) * n);
        for (int64_t i = 0; i < n; ++i) perm[i] = i;
        for (int64_t i = 0; i < n; ++i) {
            int64_t best = i;
            for (int64_t k = i + 1; k < n; ++k)
                if (d[perm[k]] < d[perm[best]]) best = k;
            int64_t t = perm[i]; perm[i] = perm[best]; perm[best] = t;
        }
        double *dw = malloc(sizeof(double) * n);
        for (int64_t i = 0; i < n; ++i) dw[i] = d[perm[i]];
#pragma omp parallel for schedule(static)
        for (int64_t c = 0; c < n; ++c)
            for (int64_t row = 0; row < n; ++row)
                X[row + c * ldx] = R[row * n + perm[c]];
        memcpy(d, dw, sizeof(double) * n);
        free(dw); free(perm);
    }
    free(e); free(R); free(rc); free(rs); free(ri);
    return status;
}

/* ------------------------------------------------------------------------
 * Cyclic Jacobi eigenvalue method for a small dense real symmetric matrix
 * (brute force; used only to pin the other routines at n <= 64).
 * A (n x n column-major) is destroyed; w ascending; V eigenvectors.
 * ---------------------------------------------------------------------- */
int orc_jacobi_d(int64_t n, double *A, double *w, double *V)
{
    if (n < 1) return ORC_EARG;
    for (int64_t i = 0; i < n * n; ++i) V[i] = 0.0;
    for (int64_t i = 0; i < n; ++i) V[i + i * n] = 1.0;
    for (int sweep = 0; sweep < 100; ++sweep) {
        double off = 0.0, tot = 0.0;
        for (int64_t q = 0; q < n; ++q)
            for (int64_t p = 0; p < n; ++p) {
                tot += A[p + q * n] * A[p + q * n];
                if (p != q) off += A[p + q * n] * A[p + q * n];
            }
        if (off <= 1e-30 * tot) break;
        for (int64_t p = 0; p < n - 1; ++p)
            for (int64_t q = p + 1; q < n; ++q) {
                double apq = A[p + q * n];
                if (apq == 0.0) continue;
                /* rotation angle zeroing A(p,q): t = tan(theta) */
                double theta = (A[q + q * n] - A[p + p * n]) / (2.0 * apq);
                double t = (theta >= 0.0 ? 1.0 : -1.0) /
                           (fabs(theta) + sqrt(theta * theta + 1.0));
                double c = 1.0 / sqrt(t * t + 1.0), s = t * c;
                for (int64_t k = 0; k < n; ++k) {   /* A <- A J (columns) */
                    double akp = A[k + p * n], akq = A[k + q * n];
                    A[k + p * n] = c * akp - s * akq;
                    A[k + q * n] = s * akp + c * akq;
                }
                for (int64_t k = 0; k < n; ++k) {   /* A <- J^T A (rows) */
                    double apk = A[p + k * n], aqk = A[q + k * n];
                    A[p + k * n] = c * apk - s * aqk;
                    A[q + k * n] = s * apk + c * aqk;
                }
                for (int64_t k = 0; k < n; ++k) {   /* V <- V J */
                    double vkp = V[k + p * n], vkq = V[k + q * n];
                    V[k + p * n] = c * vkp - s * vkq;
                    V[k + q * n] = s * vkp + c * vkq;
                }
            }
    }
    /* sort ascending */
    for (int64_t i = 0; i < n; ++i) w[i] = A[i + i * n];
    for (int64_t i = 0; i < n; ++i) {
        int64_t best = i;
        for (int64_t k = i + 1; k < n; ++k) if (w[k] < w[best]) best = k;
        if (best != i) {
            double t = w[i]; w[i] = w[best]; w[best] = t;
            for (int64_t r = 0; r < n; ++r) {
                double u = V[r + i * n]; V[r + i * n] = V[r + best * n]; V[r + best * n] = u;
            }
        }
    }
    return ORC_OK;
}

/* ------------------------------------------------------------------------
 * Full -> band reduction (Sec. 2.1, Eq. 2stage_fwd1): B = P A P^*.
 *
 * The paper states what this step produces -- a Hermitian band matrix of
 * semi-bandwidth b similar to A -- and that it is done with BLAS-3
 * operations, not how.  The plain definition written here takes one
 * Householder reflector per column (the column-at-a-time form of successive
 * band reduction, Bischof, Lang and Sun): for j = 0, 1, ..., n-b-2 the
 * reflector H_j = I - tau_j v_j v_j^H with H_j^H x = beta e1 (the standard
 * method of Eq. householder) is built from x = A[j+b : n, j], and
 * A <- H_j^H A H_j acts on rows and columns [j+b, n).  Column j is then
 * beta e1 below row j+b-1 and stays so: later reflectors act on rows
 * >= j+1+b only.  A blocked implementation groups consecutive reflectors
 * into panels and yields the same reflectors up to rounding, because a
 * column of a panel only ever sees the left updates of the panel's earlier
 * reflectors (their right updates touch columns >= j+b).
 *
 * With J = max(0, n-b-1) reflectors, B = H_{J-1}^H ... H_0^H A H_0 ... H_{J-1},
 * i.e. P = H_{J-1}^H ... H_0^H and P^* = H_0 H_1 ... H_{J-1}.
 *
 * A  n x n Hermitian, both triangles stored, column-major (lda >= n);
 *    overwritten with B (entries outside the band are set to exact zeros
 *    for the annihilated columns; nothing else is touched).
 * V  n x J column-major (ldv >= n): column j holds v_j in rows [j+b, n)
 *    with v_j[0] = 1 at row j+b; every other entry is set to zero.
 * tau J entries.
 * Lengths n-j-b of 1 (j = n-b-1) carry no reflector: there is nothing to
 * annihilate (the complex case would only rotate the phase of one entry,
 * which the band form does not require).
 * ---------------------------------------------------------------------- */
int64_t orc_full_reflectors(int64_t n, int64_t b)
{
    return (b >= 1 && n - b - 1 > 0) ? n - b - 1 : 0;
}

int orc_full_to_band_d(int64_t n, int64_t b, double *A, int64_t lda, double *V,
                       int64_t ldv, double *tau)
{
    if (n < 0 || b < 1 || lda < (n > 1 ? n : 1) || ldv < (n > 1 ? n : 1)) return ORC_EARG;
    const int64_t J = orc_full_reflectors(n, b);
    for (int64_t j = 0; j < J; ++j) {
        const int64_t r = j + b, m = n - r;
        double *v = V + j * ldv;
        for (int64_t i = 0; i < n; ++i) v[i] = 0.0;
        double beta;
        for (int64_t i = 0; i < m; ++i) v[r + i] = A[(r + i) + j * lda];
        orc_larfg_d(m, v + r, &tau[j], &beta);
        const double t = tau[j];
        /* left: A[r:n, k] <- H^H A[r:n, k] for every column k != j */
#pragma omp parallel for schedule(static)
        for (int64_t k = 0; k < n; ++k) {
            if (k == j) continue;
            double *y = A + r + k * lda;
            double d = 0.0;
            for (int64_t i = 0; i < m; ++i) d += v[r + i] * y[i];
            for (int64_t i = 0; i < m; ++i) y[i] -= t * d * v[r + i];
        }
        /* right: A[k, r:n] <- A[k, r:n] H for every row k != j */
#pragma omp parallel for schedule(static)
        for (int64_t k = 0; k < n; ++k) {
            if (k == j) continue;
            double d = 0.0;
            for (int64_t i = 0; i < m; ++i) d += A[k + (r + i) * lda] * v[r + i];
            for (int64_t i = 0; i < m; ++i) A[k + (r + i) * lda] -= t * d * v[r + i];
        }
        /* column j and row j: beta e1 */
        for (int64_t i = 0; i < m; ++i) {
            A[(r + i) + j * lda] = i == 0 ? beta : 0.0;
            A[j + (r + i) * lda] = i == 0 ? beta : 0.0;
        }
    }
    return ORC_OK;
}

int orc_full_to_band_z(int64_t n, int64_t b, zc *A, int64_t lda, zc *V, int64_t ldv, zc *tau)
{
    if (n < 0 || b < 1 || lda < (n > 1 ? n : 1) || ldv < (n > 1 ? n : 1)) return ORC_EARG;
    const int64_t J = orc_full_reflectors(n, b);
    for (int64_t j = 0; j < J; ++j) {
        const int64_t r = j + b, m = n - r;
        zc *v = V + j * ldv;
        for (int64_t i = 0; i < n; ++i) v[i] = 0.0;
        double beta;
        for (int64_t i = 0; i < m; ++i) v[r + i] = A[(r + i) + j * lda];
        orc_larfg_z(m, v + r, &tau[j], &beta);
        const zc t = tau[j];
        /* left: H^H y = y - conj(tau) v (v^H y) */
#pragma omp parallel for schedule(static)
        for (int64_t k = 0; k < n; ++k) {
            if (k == j) continue;
            zc *y = A + r + k * lda;
            zc d = 0.0;
            for (int64_t i = 0; i < m; ++i) d += conj(v[r + i]) * y[i];
            for (int64_t i = 0; i < m; ++i) y[i] -= conj(t) * d * v[r + i];
        }
        /* right: y H = y - tau (y v) v^H for the rows y */
#pragma omp parallel for schedule(static)
        for (int64_t k = 0; k < n; ++k) {
            if (k == j) continue;
            zc d = 0.0;
            for (int64_t i = 0; i < m; ++i) d += A[k + (r + i) * lda] * v[r + i];
            for (int64_t i = 0; i < m; ++i) A[k + (r + i) * lda] -= t * d * conj(v[r + i]);
        }
        for (int64_t i = 0; i < m; ++i) {
            A[(r + i) + j * lda] = i == 0 ? beta : 0.0;
            A[j + (r + i) * lda] = i == 0 ? beta : 0.0;
        }
    }
    return ORC_OK;
}

/* ------------------------------------------------------------------------
 * Band -> full back-transformation (Sec. 2.1, Eq. 2stage_bkwd2):
 * C = P^* Y = H_0 (H_1 ( ... (H_{J-1} Y))), i.e. the stage-1 reflectors
 * applied one at a time in reverse generation order, each as
 * y <- y - tau_j v_j (v_j^H y) on rows [j+b, n) (the operation of Eq.
 * kernel).  v_j[0] is read from V (not assumed 1); entries of V outside
 * rows [j+b, n) of column j are not read.  Columns c0 .. c1-1 of Z only;
 * OpenMP over the independent columns.
 * ---------------------------------------------------------------------- */
int orc_back_transform_full_d(int64_t n, int64_t b, int64_t c0, int64_t c1, const double *V,
                              int64_t ldv, const double *tau, double *Z, int64_t ldz)
{
    if (n < 0 || b < 1 || c0 < 0 || c1 < c0 || ldz < (n > 1 ? n : 1) || ldv < (n > 1 ? n : 1))
        return ORC_EARG;
    const int64_t J = orc_full_reflectors(n, b);
#pragma omp parallel for schedule(dynamic, 1)
    for (int64_t c = c0; c < c1; ++c) {
        double *z = Z + c * ldz;
        for (int64_t j = J - 1; j >= 0; --j) {
            const int64_t r = j + b, m = n - r;
            const double *v = V + j * ldv + r;
            double d = 0.0;
            for (int64_t i = 0; i < m; ++i) d += v[i] * z[r + i];
            const double a = tau[j] * d;
            for (int64_t i = 0; i < m; ++i) z[r + i] -= a * v[i];
        }
    }
    return ORC_OK;
}

int orc_back_transform_full_z(int64_t n, int64_t b, int64_t c0, int64_t c1, const zc *V,
                              int64_t ldv, const zc *tau, zc *Z, int64_t ldz)
{
    if (n < 0 || b < 1 || c0 < 0 || c1 < c0 || ldz < (n > 1 ? n : 1) || ldv < (n > 1 ? n : 1))
        return ORC_EARG;
    const int64_t J = orc_full_reflectors(n, b);
#pragma omp parallel for schedule(dynamic, 1)
    for (int64_t c = c0; c < c1; ++c) {
        zc *z = Z + c * ldz;
        for (int64_t j = J - 1; j >= 0; --j) {
            const int64_t r = j + b, m = n - r;
            const zc *v = V + j * ldv + r;
            zc d = 0.0;
            for (int64_t i = 0; i < m; ++i) d += conj(v[i]) * z[r + i];
            const zc a = tau[j] * d;
            for (int64_t i = 0; i < m; ++i) z[r + i] -= a * v[i];
        }
    }
    return ORC_OK;
}
