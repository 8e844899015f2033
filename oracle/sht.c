/*
 * Oracle: plain FP64 spherical harmonic synthesis and its adjoint on the
 * HEALPix ring grid, written from the definitions.
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing on the product path may include, link,
 * load or call this file; only the test-suite, the smoke check and the CPU
 * baseline leg of the benchmark use it.  It shares no code with the GPU
 * library.
 *
 * What it computes
 *   synthesis  s(p) = sum_{l,m} a_lm Y_lm(theta_p, phi_p)     (real field,
 *              a_{l,-m} = (-1)^m conj(a_lm), so s = F_0 + 2 Re sum_{m>0} F_m e^{i m phi})
 *   adjoint    b_lm = sum_p r(p) conj(Y_lm(theta_p, phi_p))
 * with orthonormal Y_lm = lambda_lm(cos theta) e^{i m phi} (Condon-Shortley
 * phase).  The adjoint is the transpose of the synthesis for the inner
 * product on a_lm that counts m > 0 twice.  In the method these play the
 * roles of the inverse and forward basis changes F^-1 and F of the paper's
 * Algorithm 2, transplanted from the flat-sky FFT to the sphere.
 *
 * Plain evaluation:
 *   - lambda_lm at each ring from the textbook three-term recurrence in l,
 *     seeded by lambda_mm evaluated in logarithms, carried as
 *     mantissa * 2^exponent so that polar values far below the FP64 range
 *     are exact until they re-enter it;
 *   - the phi sum as a direct sum over pixels (no FFT), with e^{i m phi_j}
 *     formed as e^{i m phi_0} times the exact root of unity w^{(m j) mod n}.
 *
 * Layout: alm[idx(l,m)][2] with idx(l,m) = m(2 lmax + 1 - m)/2 + l (m-major),
 * maps in HEALPix RING order.
 */
#include <math.h>
#include <stdlib.h>
#include <string.h>
#include <omp.h>

#define TWO_PI 6.283185307179586476925286766559
#define PI     3.141592653589793238462643383280

static long alm_index(int l, int m, int lmax) {
    return (long)m * (2L * lmax + 1 - m) / 2 + l;
}

/* HEALPix RING geometry for ring r = 1..4N-1: cos(theta), sin(theta),
 * pixel count, phi of the first pixel and the first pixel's index. */
void or_ring(int nside, int r, double* z, double* sint, long* nph, double* phi0, long* start) {
    long n = nside;
    long npix = 12 * n * n;
    if (r < n) {                      /* north polar cap */
        double onemz = (double)r * r / (3.0 * n * n);
        *z = 1.0 - onemz;
        *sint = sqrt(onemz * (2.0 - onemz));
        *nph = 4L * r;
        *phi0 = PI / (4.0 * r);
        *start = 2L * r * (r - 1);
    } else if (r <= 3 * n) {          /* equatorial belt */
        *z = (4.0 / 3.0) - 2.0 * r / (3.0 * n);
        *sint = sqrt((1.0 - *z) * (1.0 + *z));
        *nph = 4L * n;
        int s = (int)((r - n + 1) % 2);
        *phi0 = PI / (2.0 * n) * (0.5 * s);
        *start = 2L * n * (n - 1) + 4L * n * (r - n);
    } else {                          /* south polar cap, mirror of the north */
        long j = 4 * n - r;
        double onemz = (double)j * j / (3.0 * n * n);
        *z = -(1.0 - onemz);
        *sint = sqrt(onemz * (2.0 - onemz));
        *nph = 4L * j;
        *phi0 = PI / (4.0 * j);
        *start = npix - 2L * j * (j + 1);
    }
}

/* log lambda_mm(x) without the sin(theta) factor:
 *   1/2 log((2m+1)/(4 pi)) + 1/2 sum_{k=1..m} log((2k-1)/(2k)). */
double or_lognorm(int m) {
    double lg = 0.5 * log((2.0 * m + 1.0) / (4.0 * PI));
    for (int k = 1; k <= m; ++k) lg += 0.5 * log1p(-1.0 / (2.0 * k));
    return lg;
}

/* The same for every m = 0..lmax as one running sum. */
static void lognorm_table(int lmax, double* out) {
    double s = 0.0;
    for (int m = 0; m <= lmax; ++m) {
        if (m > 0) s += 0.5 * log1p(-1.0 / (2.0 * m));
        out[m] = 0.5 * log((2.0 * m + 1.0) / (4.0 * PI)) + s;
    }
}

/* lambda_lm(x) for l = m..lmax as mant[l-m] * 2^expo[l-m], given lognorm = or_lognorm(m).
 *   log|lambda_mm| = lognorm + m log(sin theta), sign (-1)^m;
 *   lambda_lm = a_lm (x lambda_{l-1,m} - b_lm lambda_{l-2,m}),
 *   a_lm = sqrt((4l^2-1)/(l^2-m^2)), b_lm = sqrt(((l-1)^2-m^2)/(4(l-1)^2-1)).
 * The two carried values share one binary exponent, reduced by 2^-256 whenever
 * the newest value exceeds 2^256 in magnitude. */
static void lambda_scaled(int m, double x, double sint, int lmax, double lognorm,
                          double* mant, int* expo) {
    if (lmax < m) return;
    if (m > 0 && sint <= 0.0) {       /* pole: lambda_lm = 0 for m > 0 */
        for (int l = m; l <= lmax; ++l) { mant[l - m] = 0.0; expo[l - m] = 0; }
        return;
    }
    double lg = lognorm + (m > 0 ? m * log(sint) : 0.0);
    double l2 = lg / log(2.0);
    int e = (int)floor(l2);
    double cur = exp2(l2 - e);
    if (m & 1) cur = -cur;
    double prev = 0.0;
    mant[0] = cur; expo[0] = e;
    for (int l = m + 1; l <= lmax; ++l) {
        double dl = l, dm = m;
        double a = sqrt((4.0 * dl * dl - 1.0) / (dl * dl - dm * dm));
        double b = sqrt(((dl - 1.0) * (dl - 1.0) - dm * dm) / (4.0 * (dl - 1.0) * (dl - 1.0) - 1.0));
        double nxt = a * (x * cur - b * prev);
        prev = cur; cur = nxt;
        if (fabs(cur) > 0x1p256) { cur = ldexp(cur, -256); prev = ldexp(prev, -256); e += 256; }
        mant[l - m] = cur; expo[l - m] = e;
    }
}

void or_lambda_scaled(int m, double x, double sint, int lmax, double* mant, int* expo) {
    lambda_scaled(m, x, sint, lmax, or_lognorm(m), mant, expo);
}

/* True values lambda_lm(x), l = m..lmax (values below the FP64 range flush to 0). */
static void lambda_true(int m, double x, double sint, int lmax, double lognorm,
                        double* out, double* mt, int* ex) {
    int cnt = lmax - m + 1;
    if (cnt <= 0) return;
    lambda_scaled(m, x, sint, lmax, lognorm, mt, ex);
    for (int i = 0; i < cnt; ++i) out[i] = ldexp(mt[i], ex[i]);
}

void or_lambda(int m, double x, double sint, int lmax, double* out) {
    int cnt = lmax - m + 1;
    if (cnt <= 0) return;
    double* mt = (double*)malloc(sizeof(double) * cnt);
    int* ex = (int*)malloc(sizeof(int) * cnt);
    lambda_true(m, x, sint, lmax, or_lognorm(m), out, mt, ex);
    free(mt); free(ex);
}

/* Per-thread scratch for one ring or one m. */
typedef struct {
    double *lam, *mt, *Fre, *Fim, *wc, *ws;
    int* ex;
} scratch_t;

static void scratch_init(scratch_t* s, int nside, int lmax) {
    long nmax = 4L * nside;
    s->lam = (double*)malloc(sizeof(double) * (lmax + 1));
    s->mt = (double*)malloc(sizeof(double) * (lmax + 1));
    s->ex = (int*)malloc(sizeof(int) * (lmax + 1));
    s->Fre = (double*)malloc(sizeof(double) * (lmax + 1));
    s->Fim = (double*)malloc(sizeof(double) * (lmax + 1));
    s->wc = (double*)malloc(sizeof(double) * nmax);
    s->ws = (double*)malloc(sizeof(double) * nmax);
}

static void scratch_free(scratch_t* s) {
    free(s->lam); free(s->mt); free(s->ex); free(s->Fre); free(s->Fim); free(s->wc); free(s->ws);
}

/* Synthesis of one ring r into out[0..nph-1]. */
static void synth_ring(int nside, int lmax, const double* alm, const double* lognorm, int r,
                       double* out, scratch_t* sc) {
    double z, st, phi0; long n, start;
    or_ring(nside, r, &z, &st, &n, &phi0, &start);
    for (int m = 0; m <= lmax; ++m) {
        lambda_true(m, z, st, lmax, lognorm[m], sc->lam, sc->mt, sc->ex);
        double re = 0.0, im = 0.0;
        for (int l = m; l <= lmax; ++l) {
            long k = alm_index(l, m, lmax);
            re += alm[2 * k] * sc->lam[l - m];
            if (m > 0) im += alm[2 * k + 1] * sc->lam[l - m];
        }
        /* E_m = F_m e^{i m phi0} */
        double c = cos(m * phi0), s = sin(m * phi0);
        sc->Fre[m] = re * c - im * s;
        sc->Fim[m] = re * s + im * c;
    }
    for (long t = 0; t < n; ++t) { sc->wc[t] = cos(TWO_PI * t / n); sc->ws[t] = sin(TWO_PI * t / n); }
    for (long j = 0; j < n; ++j) {
        double acc = 0.0;
        long t = 0;
        for (int m = 1; m <= lmax; ++m) {
            t += j; if (t >= n) t -= n;           /* t = (m j) mod n */
            acc += sc->Fre[m] * sc->wc[t] - sc->Fim[m] * sc->ws[t];
        }
        out[j] = sc->Fre[0] + 2.0 * acc;
    }
}

static void set_threads(int nthreads) {
    if (nthreads > 0) omp_set_num_threads(nthreads);
}

int or_max_threads(void) { return omp_get_max_threads(); }

/* Synthesis restricted to a list of rings; outputs concatenated in list order. */
void or_alm2map_rings(int nside, int lmax, const double* alm, const int* rings, int nrings,
                      double* out, int nthreads) {
    long* off = (long*)malloc(sizeof(long) * (nrings + 1));
    double* lognorm = (double*)malloc(sizeof(double) * (lmax + 1));
    lognorm_table(lmax, lognorm);
    off[0] = 0;
    for (int i = 0; i < nrings; ++i) {
        double z, st, phi0; long n, start;
        or_ring(nside, rings[i], &z, &st, &n, &phi0, &start);
        off[i + 1] = off[i] + n;
    }
    set_threads(nthreads);
#pragma omp parallel
    {
        scratch_t sc;
        scratch_init(&sc, nside, lmax);
#pragma omp for schedule(dynamic, 1)
        for (int i = 0; i < nrings; ++i)
            synth_ring(nside, lmax, alm, lognorm, rings[i], out + off[i], &sc);
        scratch_free(&sc);
    }
    free(lognorm);
    free(off);
}

void or_alm2map(int nside, int lmax, const double* alm, double* map, int nthreads) {
    int nr = 4 * nside - 1;
    int* rings = (int*)malloc(sizeof(int) * nr);
    for (int r = 1; r <= nr; ++r) rings[r - 1] = r;
    /* rings in order are contiguous in RING ordering */
    or_alm2map_rings(nside, lmax, alm, rings, nr, map, nthreads);
    free(rings);
}

/* R_m(r) = sum_j map_j e^{-i m phi_j} for m in ms[], every ring.  R[(r-1)*nm + k][2]. */
static void ring_fourier(int nside, const double* map, const int* ms, int nm, double* R) {
    int nr = 4 * nside - 1;
#pragma omp parallel
    {
        long nmax = 4L * nside;
        double* wc = (double*)malloc(sizeof(double) * nmax);
        double* ws = (double*)malloc(sizeof(double) * nmax);
#pragma omp for schedule(dynamic, 1)
        for (int r = 1; r <= nr; ++r) {
            double z, st, phi0; long n, start;
            or_ring(nside, r, &z, &st, &n, &phi0, &start);
            for (long t = 0; t < n; ++t) { wc[t] = cos(TWO_PI * t / n); ws[t] = sin(TWO_PI * t / n); }
            const double* v = map + start;
            for (int k = 0; k < nm; ++k) {
                long m = ms[k];
                long mr = m % n;
                double re = 0.0, im = 0.0;
                long t = 0;
                for (long j = 0; j < n; ++j) {       /* t = (m j) mod n */
                    re += v[j] * wc[t];
                    im -= v[j] * ws[t];
                    t += mr; if (t >= n) t -= n;
                }
                /* times e^{-i m phi0} */
                double c = cos(m * phi0), s = sin(m * phi0);
                R[2 * ((long)(r - 1) * nm + k)] = re * c + im * s;
                R[2 * ((long)(r - 1) * nm + k) + 1] = im * c - re * s;
            }
        }
        free(wc); free(ws);
    }
}

/* b_lm = sum_p map_p conj(Y_lm(p)) for the m listed in ms[]; out holds, one m
 * after another, b_lm for l = m..lmax as [re, im] pairs. */
void or_adjoint_m(int nside, int lmax, const double* map, const int* ms, int nm,
                  double* out, int nthreads) {
    int nr = 4 * nside - 1;
    set_threads(nthreads);
    double* R = (double*)malloc(sizeof(double) * 2 * (size_t)nr * nm);
    ring_fourier(nside, map, ms, nm, R);
    double* lognorm = (double*)malloc(sizeof(double) * (lmax + 1));
    lognorm_table(lmax, lognorm);
    long* off = (long*)malloc(sizeof(long) * (nm + 1));
    off[0] = 0;
    for (int k = 0; k < nm; ++k) off[k + 1] = off[k] + (lmax - ms[k] + 1);
#pragma omp parallel
    {
        scratch_t sc;
        scratch_init(&sc, nside, lmax);
#pragma omp for schedule(dynamic, 1)
        for (int k = 0; k < nm; ++k) {
            int m = ms[k];
            double* o = out + 2 * off[k];
            memset(o, 0, sizeof(double) * 2 * (lmax - m + 1));
            for (int r = 1; r <= nr; ++r) {
                double z, st, phi0; long n, start;
                or_ring(nside, r, &z, &st, &n, &phi0, &start);
                lambda_true(m, z, st, lmax, lognorm[m], sc.lam, sc.mt, sc.ex);
                double re = R[2 * ((long)(r - 1) * nm + k)], im = R[2 * ((long)(r - 1) * nm + k) + 1];
                for (int l = m; l <= lmax; ++l) {
                    o[2 * (l - m)] += sc.lam[l - m] * re;
                    o[2 * (l - m) + 1] += sc.lam[l - m] * im;
                }
            }
        }
        scratch_free(&sc);
    }
    free(off);
    free(lognorm);
    free(R);
}

/* Full adjoint into alm[n_alm][2] (m-major). */
void or_adjoint(int nside, int lmax, const double* map, double* alm, int nthreads) {
    int* ms = (int*)malloc(sizeof(int) * (lmax + 1));
    for (int m = 0; m <= lmax; ++m) ms[m] = m;
    or_adjoint_m(nside, lmax, map, ms, lmax + 1, alm, nthreads);
    free(ms);
}
