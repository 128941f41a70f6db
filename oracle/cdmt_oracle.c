/*
 * FP64 CPU oracle for coherent dedispersion of channelised dual-polarisation
 * voltages to many DM trials (Bassa, Pleunis & Hessels, "Enabling pulsar and
 * fast transient searches using coherent dedispersion", 2016).
 *
 * TEST INFRASTRUCTURE ONLY.  This file is the plain, slow, obviously correct
 * definition that the GPU library is checked against.  Only the test suite,
 * the smoke check and the CPU-baseline leg of the benchmark load it.  It shares
 * no source, header, table or helper with the HIP library and includes nothing
 * from it.
 *
 * Everything is double precision.  The steps follow the paper's order:
 *   Sec. 3 / Alg. 1: segment a block of N_bin samples (overlap n_d*n_c),
 *   forward FFT, swap halves per subband, multiply by the transfer function of
 *   each channel (Sec. 2, Eq. 1), swap halves per channel, backward FFT of
 *   M_bin = N_bin/n_c, discard n_d/2 samples at each edge, detect (|X|^2+|Y|^2)
 *   and pack channels in decreasing frequency.  Time downsampling by summing
 *   ndec consecutive kept samples follows detection.
 *
 * Readings of points the paper leaves open (each is listed in the design
 * notes): forward transform e^{-2 pi i kn/N}, backward e^{+}; the transfer
 * function of Eq. 1 with a + sign is the dispersing response, so
 * dedispersion multiplies by exp(sign * 2 pi i Phi) with sign = -1; the 1/N_bin
 * normalisation is applied with the transfer function; k_DM = 1/2.41e-4
 * exactly; upper sideband, subbands given in increasing frequency.
 */
#include <complex.h>
#include <math.h>
#include <pthread.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define ORC_PI 3.14159265358979323846264338327950288

/* Sec. 2, text after Eq. 1: k_DM^{-1} = 2.41e-4 (s MHz^2 per pc cm^-3)^{-1}. */
static const double ORC_KDM = 1.0 / 2.41e-4;

typedef double complex cplx;

/* ------------------------------------------------------------------ */
/* Discrete Fourier transforms                                          */
/* ------------------------------------------------------------------ */

/* The DFT by its definition, O(n^2): y[k] = sum_n x[n] exp(sign 2 pi i k n / n).
 * The exponent k*n is reduced mod n before the trigonometric call so that the
 * argument stays small. */
void orc_dft(const double *x_ri, double *y_ri, long n, int sign)
{
    const cplx *x = (const cplx *)x_ri;
    cplx *y = (cplx *)y_ri;
    for (long k = 0; k < n; ++k) {
        cplx acc = 0;
        for (long j = 0; j < n; ++j) {
            long e = (long)(((unsigned long long)k * (unsigned long long)j) % (unsigned long long)n);
            double a = sign * 2.0 * ORC_PI * (double)e / (double)n;
            acc += x[j] * (cos(a) + I * sin(a));
        }
        y[k] = acc;
    }
}

/* In-place iterative radix-2 Cooley-Tukey FFT (decimation in time) of a
 * power-of-two length n:  x[k] <- sum_j x[j] exp(sign 2 pi i j k / n).
 * Unnormalised.  Every twiddle factor is evaluated directly with cos/sin (no
 * recurrence).  Returns -1 if n is not a power of two. */
int orc_fft_inplace(cplx *x, long n, int sign)
{
    if (n < 1 || (n & (n - 1)))
        return -1;
    /* bit-reversal permutation */
    for (long i = 1, j = 0; i < n; ++i) {
        long bit = n >> 1;
        for (; j & bit; bit >>= 1)
            j ^= bit;
        j ^= bit;
        if (i < j) {
            cplx t = x[i];
            x[i] = x[j];
            x[j] = t;
        }
    }
    cplx *w = (cplx *)malloc(sizeof(cplx) * (size_t)(n > 1 ? n / 2 : 1));
    if (!w)
        return -2;
    for (long len = 2; len <= n; len <<= 1) {
        long half = len / 2;
        for (long k = 0; k < half; ++k) {
            double a = sign * 2.0 * ORC_PI * (double)k / (double)len;
            w[k] = cos(a) + I * sin(a);
        }
        for (long s = 0; s < n; s += len) {
            for (long k = 0; k < half; ++k) {
                cplx u = x[s + k];
                cplx v = x[s + k + half] * w[k];
                x[s + k] = u + v;
                x[s + k + half] = u - v;
            }
        }
    }
    free(w);
    return 0;
}

/* Out-of-place wrapper on interleaved (re, im) doubles, for the tests. */
int orc_fft(const double *x_ri, double *y_ri, long n, int sign)
{
    memcpy(y_ri, x_ri, sizeof(double) * 2 * (size_t)n);
    return orc_fft_inplace((cplx *)y_ri, n, sign);
}

/* ------------------------------------------------------------------ */
/* Transfer function (Sec. 2, Eq. 1) and dispersion sweep (Eq. 2)       */
/* ------------------------------------------------------------------ */

/* Phase of H(nu + nu0) in cycles: nu^2 k_DM DM / (nu0^2 (nu + nu0)), with
 * nu, nu0 in MHz; the factor 1e6 converts s*MHz to cycles (Eq. 1). */
double orc_chirp_cycles(double nu, double nu0, double dm)
{
    return 1e6 * ORC_KDM * dm * nu * nu / (nu0 * nu0 * (nu0 + nu));
}

/* Dispersion sweep in seconds across [nu_min, nu_max] MHz (Eq. 2). */
double orc_sweep_seconds(double nu_min, double nu_max, double dm)
{
    return ORC_KDM * (1.0 / (nu_min * nu_min) - 1.0 / (nu_max * nu_max)) * dm;
}

double orc_kdm(void) { return ORC_KDM; }

/* ------------------------------------------------------------------ */
/* Plan parameters                                                      */
/* ------------------------------------------------------------------ */

typedef struct {
    int nsub;          /* n_s subbands, increasing frequency              */
    double f_centre;   /* MHz, centre of the whole band                     */
    double bw;         /* MHz, subband bandwidth = complex sample rate      */
    int nfft;          /* N_bin                                            */
    int noverlap;      /* n_d * n_c, in subband samples                     */
    int nchan;         /* n_c channels per subband                          */
    int ndec;          /* output samples summed per filterbank sample       */
    int chirp_ref;     /* 0: per-channel nu0 (Sec. 2 text), 1: per-subband  */
    int sign;          /* -1 dedisperses (default), +1 applies Eq. 1 as is  */
} orc_cfg;

/* Input sample kinds: interleaved [time][pol X,Y][re,im]. */
enum { ORC_CF32 = 0, ORC_CI8 = 1, ORC_CF64 = 2 };

static double sub_centre(const orc_cfg *c, int s)
{
    return c->f_centre + ((double)s - (c->nsub - 1) / 2.0) * c->bw;
}

static cplx load_sample(int kind, const void *x, long idx, int pol)
{
    long o = (idx * 2 + pol) * 2;
    switch (kind) {
    case ORC_CI8: {
        const int8_t *p = (const int8_t *)x;
        return (double)p[o] + I * (double)p[o + 1];
    }
    case ORC_CF32: {
        const float *p = (const float *)x;
        return (double)p[o] + I * (double)p[o + 1];
    }
    default: {
        const double *p = (const double *)x;
        return p[o] + I * p[o + 1];
    }
    }
}

/* Reference frequency nu0 and offset nu (MHz) of swapped spectrum bin j of an
 * N-bin subband spectrum (bin j is at (j - N/2) * bw / N from the subband
 * centre, Sec. 3).  CHANNEL mode: nu0 is the centre of the channel holding j
 * and nu the offset from it (Sec. 2, last paragraph); SUBBAND mode: nu0 is the
 * subband centre (Eq. 1 allows either). */
static void bin_frequency(const orc_cfg *c, int s, long j, long n, double *nu0, double *nu)
{
    double fs = sub_centre(c, s);
    double rel = ((double)j - n / 2.0) * c->bw / (double)n;
    if (c->chirp_ref == 0) {
        long m = n / c->nchan;
        long ch = j / m;
        double centre = fs - c->bw / 2.0 + (ch + 0.5) * c->bw / c->nchan;
        *nu0 = centre;
        *nu = rel - (centre - fs);
    } else {
        *nu0 = fs;
        *nu = rel;
    }
}

int orc_validate(const orc_cfg *c)
{
    if (c->nsub < 1 || c->nfft < 2 || (c->nfft & (c->nfft - 1)))
        return -1;
    if (c->nchan < 1 || (c->nchan & (c->nchan - 1)) || c->nfft % c->nchan)
        return -1;
    if (c->noverlap < 0 || c->noverlap >= c->nfft || c->noverlap % (2 * c->nchan))
        return -1;
    int m = c->nfft / c->nchan, nd = c->noverlap / c->nchan;
    if (c->ndec < 1 || (m - nd) % c->ndec)
        return -1;
    if (!(c->bw > 0) || !(c->f_centre - c->nsub * c->bw / 2.0 > 0))
        return -1;
    if (c->sign != 1 && c->sign != -1)
        return -1;
    if (c->chirp_ref != 0 && c->chirp_ref != 1)
        return -1;
    return 0;
}

/* Output samples per block and per channel. */
int orc_tblk(const orc_cfg *c)
{
    int m = c->nfft / c->nchan, nd = c->noverlap / c->nchan;
    return (m - nd) / c->ndec;
}

/*
 * One subband s, one block b:  F[d][t][ch] for ch = 0 .. nchan-1 in
 * INCREASING frequency (the caller packs decreasing frequency).
 * x_sub points at subband s's stream [ntime][2][2] of the given kind.
 */
int orc_subband_block(const orc_cfg *c, int kind, const void *x_sub, long ntime, int s, int b,
                      const double *dms, int ndm, double *F)
{
    if (orc_validate(c))
        return -1;
    const long n = c->nfft, m = n / c->nchan;
    const long nd = c->noverlap / c->nchan;
    const long tb = (m - nd) / c->ndec;
    const long start = (long)b * (n - c->noverlap);
    if (start + n > ntime)
        return -2;

    cplx *spec = (cplx *)malloc(sizeof(cplx) * 2 * n);   /* swapped spectra, 2 pols */
    cplx *seg = (cplx *)malloc(sizeof(cplx) * n);
    cplx *z = (cplx *)malloc(sizeof(cplx) * m);
    double *inten = (double *)malloc(sizeof(double) * m);
    cplx *h = (cplx *)malloc(sizeof(cplx) * n);
    if (!spec || !seg || !z || !inten || !h) {
        free(spec); free(seg); free(z); free(inten); free(h);
        return -3;
    }

    /* Sec. 3: segment, forward FFT, swap halves per subband. */
    for (int p = 0; p < 2; ++p) {
        for (long i = 0; i < n; ++i)
            seg[i] = load_sample(kind, x_sub, start + i, p);
        orc_fft_inplace(seg, n, -1);
        for (long j = 0; j < n; ++j)
            spec[p * n + j] = seg[(j + n / 2) % n];
    }

    for (int d = 0; d < ndm; ++d) {
        /* Eq. 1 for every bin; one transfer function serves both pols. */
        for (long j = 0; j < n; ++j) {
            double nu0, nu;
            bin_frequency(c, s, j, n, &nu0, &nu);
            double cyc = orc_chirp_cycles(nu, nu0, dms[d]);
            h[j] = cexp(I * (double)c->sign * 2.0 * ORC_PI * cyc) / (double)n;
        }
        for (long ch = 0; ch < c->nchan; ++ch) {
            for (long i = 0; i < m; ++i)
                inten[i] = 0.0;
            for (int p = 0; p < 2; ++p) {
                /* swap halves per channel, then backward FFT of M_bin */
                for (long i = 0; i < m; ++i) {
                    long j = ch * m + (i + m / 2) % m;
                    z[i] = spec[p * n + j] * h[j];
                }
                orc_fft_inplace(z, m, +1);
                for (long i = 0; i < m; ++i)
                    inten[i] += creal(z[i]) * creal(z[i]) + cimag(z[i]) * cimag(z[i]);
            }
            /* unpad n_d/2 per edge, then sum ndec kept samples */
            for (long t = 0; t < tb; ++t) {
                double acc = 0.0;
                for (long q = 0; q < c->ndec; ++q)
                    acc += inten[nd / 2 + t * c->ndec + q];
                F[((long)d * tb + t) * c->nchan + ch] = acc;
            }
        }
    }
    free(spec); free(seg); free(z); free(inten); free(h);
    return 0;
}

/* ------------------------------------------------------------------ */
/* Whole filterbank, threads over (subband, block) pairs                */
/* ------------------------------------------------------------------ */

typedef struct {
    const orc_cfg *c;
    int kind;
    const void *x;
    long ntime;
    int nblock;
    const double *dms;
    int ndm;
    double *out;
    int next;            /* next (s, b) work item */
    int status;
    pthread_mutex_t mu;
} orc_job;

/*
 * Derivative with respect to DM of L = sum_{d,t,ch} G[d][t][ch] F[d][t][ch]
 * for one subband s and block b, one value per DM trial (F as produced by
 * orc_subband_block, G in the same layout).  Not a step of the paper: the
 * adjoint of its per-DM chain, for refining a candidate's DM by gradient
 * ascent.  Each forward step of orc_subband_block is followed, then its
 * adjoint in reverse order (complex gradients as dL = Re sum conj(g) dv):
 *   F = sum of ndec kept samples of I       -> dL/dI[i] = G[t(i)] (0 if dropped)
 *   I = |y_X|^2 + |y_Y|^2                   -> g_y = 2 (dL/dI) y
 *   y = backward transform (e^{+}) of z     -> g_z = forward transform (e^{-}) of g_y
 *   z = channel-swapped S' (a permutation)  -> g_S' = the inverse permutation of g_z
 *   S'_j = S_j h_j, h_j = exp(sign 2 pi i Phi_j) / N, Phi_j = DM phi_j (Eq. 1
 *   is linear in DM)                        -> dS'_j/dDM = sign 2 pi i phi_j S'_j
 *   dL/dDM = sum_j Re(conj(g_S'_j) dS'_j/dDM), both polarisations.
 * absterms (may be NULL) receives, per DM, the sum of the absolute values of
 * those terms, sum_j |Re(conj(g_S'_j) dS'_j/dDM)|: the scale that rounding
 * errors of a floating-point evaluation of the same sum are measured against.
 */
int orc_dm_gradient(const orc_cfg *c, int kind, const void *x_sub, long ntime, int s, int b,
                    const double *dms, int ndm, const double *G, double *dldm,
                    double *absterms)
{
    if (orc_validate(c))
        return -1;
    const long n = c->nfft, m = n / c->nchan;
    const long nd = c->noverlap / c->nchan;
    const long tb = (m - nd) / c->ndec;
    const long start = (long)b * (n - c->noverlap);
    if (start + n > ntime)
        return -2;

    cplx *spec = (cplx *)malloc(sizeof(cplx) * 2 * n);
    cplx *seg = (cplx *)malloc(sizeof(cplx) * n);
    cplx *z = (cplx *)malloc(sizeof(cplx) * 2 * m);
    cplx *h = (cplx *)malloc(sizeof(cplx) * n);
    double *phi = (double *)malloc(sizeof(double) * n);
    double *gi = (double *)malloc(sizeof(double) * m);
    if (!spec || !seg || !z || !h || !phi || !gi) {
        free(spec); free(seg); free(z); free(h); free(phi); free(gi);
        return -3;
    }
    for (int p = 0; p < 2; ++p) {
        for (long i = 0; i < n; ++i)
            seg[i] = load_sample(kind, x_sub, start + i, p);
        orc_fft_inplace(seg, n, -1);
        for (long j = 0; j < n; ++j)
            spec[p * n + j] = seg[(j + n / 2) % n];
    }
    for (long j = 0; j < n; ++j) {
        double nu0, nu;
        bin_frequency(c, s, j, n, &nu0, &nu);
        phi[j] = orc_chirp_cycles(nu, nu0, 1.0);          /* Eq. 1 cycles per unit DM */
    }
    for (int d = 0; d < ndm; ++d) {
        for (long j = 0; j < n; ++j)
            h[j] = cexp(I * (double)c->sign * 2.0 * ORC_PI * phi[j] * dms[d]) / (double)n;
        double acc = 0.0, abs_acc = 0.0;
        for (long ch = 0; ch < c->nchan; ++ch) {
            /* dL/dI over the channel's M samples */
            for (long i = 0; i < m; ++i)
                gi[i] = 0.0;
            for (long t = 0; t < tb; ++t)
                for (long q = 0; q < c->ndec; ++q)
                    gi[nd / 2 + t * c->ndec + q] = G[((long)d * tb + t) * c->nchan + ch];
            for (int p = 0; p < 2; ++p) {
                cplx *zp = z + p * m;
                for (long i = 0; i < m; ++i) {
                    long j = ch * m + (i + m / 2) % m;
                    zp[i] = spec[p * n + j] * h[j];
                }
                orc_fft_inplace(zp, m, +1);                 /* y */
                for (long i = 0; i < m; ++i)
                    zp[i] = 2.0 * gi[i] * zp[i];             /* g_y */
                orc_fft_inplace(zp, m, -1);                 /* g_z */
                for (long i = 0; i < m; ++i) {
                    long j = ch * m + (i + m / 2) % m;       /* g_S' at bin j */
                    cplx sp = spec[p * n + j] * h[j];
                    cplx ds = (double)c->sign * 2.0 * ORC_PI * phi[j] * I * sp;
                    const double term = creal(conj(zp[i]) * ds);
                    acc += term;
                    abs_acc += fabs(term);
                }
            }
        }
        dldm[d] = acc;
        if (absterms)
            absterms[d] = abs_acc;
    }
    free(spec); free(seg); free(z); free(h); free(phi); free(gi);
    return 0;
}

/*
 * Gradient of the same L with respect to the voltages of subband s, from
 * block b and one DM: the adjoint continued through the per-DM multiply and
 * the forward stage (Sec. 3 order reversed).  With g_S' as in
 * orc_dm_gradient:
 *   S'_j = spec_j h_j                        -> g_spec_j = g_S'_j conj(h_j)
 *   spec_j = X[(j + N/2) mod N] (swap)       -> g_X[k] = g_spec[(k + N/2) mod N]
 *   X = forward transform (e^{-}) of seg     -> g_seg = backward transform (e^{+}) of g_X
 *   seg[n] = x[b (N - n_d n_c) + n]          -> g_x[b (N - n_d n_c) + n] += g_seg[n]
 * gx is complex128 [ntime][2 pol] (re, im interleaved) and is ADDED to; for
 * a real loss dL = Re sum conj(gx) dx, i.e. dL/dRe x = Re gx, dL/dIm x = Im gx.
 */
int orc_voltage_gradient(const orc_cfg *c, int kind, const void *x_sub, long ntime, int s, int b,
                         double dm, const double *G, double *gx)
{
    if (orc_validate(c))
        return -1;
    const long n = c->nfft, m = n / c->nchan;
    const long nd = c->noverlap / c->nchan;
    const long tb = (m - nd) / c->ndec;
    const long start = (long)b * (n - c->noverlap);
    if (start + n > ntime)
        return -2;
    cplx *spec = (cplx *)malloc(sizeof(cplx) * 2 * n);
    cplx *seg = (cplx *)malloc(sizeof(cplx) * n);
    cplx *z = (cplx *)malloc(sizeof(cplx) * m);
    cplx *h = (cplx *)malloc(sizeof(cplx) * n);
    cplx *gspec = (cplx *)malloc(sizeof(cplx) * n);
    double *gi = (double *)malloc(sizeof(double) * m);
    if (!spec || !seg || !z || !h || !gspec || !gi) {
        free(spec); free(seg); free(z); free(h); free(gspec); free(gi);
        return -3;
    }
    for (int p = 0; p < 2; ++p) {
        for (long i = 0; i < n; ++i)
            seg[i] = load_sample(kind, x_sub, start + i, p);
        orc_fft_inplace(seg, n, -1);
        for (long j = 0; j < n; ++j)
            spec[p * n + j] = seg[(j + n / 2) % n];
    }
    for (long j = 0; j < n; ++j) {
        double nu0, nu;
        bin_frequency(c, s, j, n, &nu0, &nu);
        double cyc = orc_chirp_cycles(nu, nu0, dm);
        h[j] = cexp(I * (double)c->sign * 2.0 * ORC_PI * cyc) / (double)n;
    }
    for (int p = 0; p < 2; ++p) {
        for (long ch = 0; ch < c->nchan; ++ch) {
            for (long i = 0; i < m; ++i)
                gi[i] = 0.0;
            for (long t = 0; t < tb; ++t)
                for (long q = 0; q < c->ndec; ++q)
                    gi[nd / 2 + t * c->ndec + q] = G[t * c->nchan + ch];
            for (long i = 0; i < m; ++i) {
                long j = ch * m + (i + m / 2) % m;
                z[i] = spec[p * n + j] * h[j];
            }
            orc_fft_inplace(z, m, +1);                      /* y */
            for (long i = 0; i < m; ++i)
                z[i] = 2.0 * gi[i] * z[i];                   /* g_y */
            orc_fft_inplace(z, m, -1);                      /* g_z */
            for (long i = 0; i < m; ++i) {
                long j = ch * m + (i + m / 2) % m;
                gspec[j] = z[i] * conj(h[j]);                /* g_spec */
            }
        }
        for (long k = 0; k < n; ++k)
            seg[k] = gspec[(k + n / 2) % n];                 /* g_X */
        orc_fft_inplace(seg, n, +1);                        /* g_seg */
        for (long i = 0; i < n; ++i) {
            gx[((start + i) * 2 + p) * 2] += creal(seg[i]);
            gx[((start + i) * 2 + p) * 2 + 1] += cimag(seg[i]);
        }
    }
    free(spec); free(seg); free(z); free(h); free(gspec); free(gi);
    return 0;
}

static size_t sample_bytes(int kind)
{
    return kind == ORC_CI8 ? 4 : (kind == ORC_CF32 ? 16 : 32);
}

static void *orc_worker(void *arg)
{
    orc_job *jb = (orc_job *)arg;
    const orc_cfg *c = jb->c;
    const long tb = orc_tblk(c);
    const long nch_out = (long)c->nsub * c->nchan;
    const long ntout = tb * jb->nblock;
    double *F = (double *)malloc(sizeof(double) * (size_t)jb->ndm * tb * c->nchan);
    if (!F) {
        pthread_mutex_lock(&jb->mu);
        jb->status = -3;
        pthread_mutex_unlock(&jb->mu);
        return NULL;
    }
    for (;;) {
        pthread_mutex_lock(&jb->mu);
        int item = jb->next++;
        pthread_mutex_unlock(&jb->mu);
        if (item >= c->nsub * jb->nblock)
            break;
        int s = item / jb->nblock, b = item % jb->nblock;
        const char *xs = (const char *)jb->x + (size_t)s * jb->ntime * sample_bytes(jb->kind);
        int st = orc_subband_block(c, jb->kind, xs, jb->ntime, s, b, jb->dms, jb->ndm, F);
        if (st) {
            pthread_mutex_lock(&jb->mu);
            jb->status = st;
            pthread_mutex_unlock(&jb->mu);
            break;
        }
        /* Sec. 3: pack channels in decreasing frequency order. */
        for (long d = 0; d < jb->ndm; ++d)
            for (long t = 0; t < tb; ++t)
                for (long ch = 0; ch < c->nchan; ++ch) {
                    long col = (long)(c->nsub - 1 - s) * c->nchan + (c->nchan - 1 - ch);
                    jb->out[(d * ntout + (long)b * tb + t) * nch_out + col] =
                        F[(d * tb + t) * c->nchan + ch];
                }
    }
    free(F);
    return NULL;
}

/* x: [nsub][ntime][2][2] of the given kind; out: [ndm][nblock*tblk][nsub*nchan]. */
int orc_dedisperse(const orc_cfg *c, int kind, const void *x, long ntime, int nblock,
                   const double *dms, int ndm, double *out, int nthreads)
{
    if (orc_validate(c))
        return -1;
    if ((long)nblock * (c->nfft - c->noverlap) + c->noverlap > ntime)
        return -2;
    orc_job jb = {c, kind, x, ntime, nblock, dms, ndm, out, 0, 0, PTHREAD_MUTEX_INITIALIZER};
    if (nthreads < 1)
        nthreads = 1;
    pthread_t *th = (pthread_t *)malloc(sizeof(pthread_t) * (size_t)nthreads);
    int started = 0;
    for (int i = 0; i < nthreads; ++i)
        if (pthread_create(&th[i], NULL, orc_worker, &jb) == 0)
            ++started;
    if (started == 0)
        orc_worker(&jb);
    for (int i = 0; i < started; ++i)
        pthread_join(th[i], NULL);
    free(th);
    return jb.status;
}

/* ------------------------------------------------------------------ */
/* Test-signal synthesis: an impulse dispersed by the inverse operator  */
/* ------------------------------------------------------------------ */

/*
 * Adds to subband s of a complex double stream x [ntime][2 pol] a real impulse
 * of amplitude amp at sample n0 in both polarisations, dispersed by the
 * inverse of the dedispersion transfer function at DM dm: on a grid of L
 * samples (power of two) centred on n0, the impulse spectrum is multiplied by
 * exp(-sign * 2 pi i Phi(nu)) with Phi from Eq. 1 and the same nu0 convention
 * as the plan (per channel or per subband), then transformed back.  Samples
 * of the window outside [0, ntime) are dropped.
 */
int orc_inject_impulse(const orc_cfg *c, int s, double *x_ri, long ntime, double dm, long n0,
                       double amp, long L)
{
    if (orc_validate(c) || L < 2 || (L & (L - 1)) || L % c->nchan)
        return -1;
    cplx *x = (cplx *)x_ri;
    cplx *w = (cplx *)malloc(sizeof(cplx) * L);
    if (!w)
        return -3;
    for (long i = 0; i < L; ++i)
        w[i] = 0;
    w[L / 2] = amp;
    orc_fft_inplace(w, L, -1);
    for (long k = 0; k < L; ++k) {
        long j = (k + L / 2) % L;        /* swapped index of FFT bin k */
        double nu0, nu;
        bin_frequency(c, s, j, L, &nu0, &nu);
        double cyc = orc_chirp_cycles(nu, nu0, dm);
        w[k] *= cexp(-I * (double)c->sign * 2.0 * ORC_PI * cyc);
    }
    orc_fft_inplace(w, L, +1);
    long w0 = n0 - L / 2;
    for (long i = 0; i < L; ++i) {
        long t = w0 + i;
        if (t < 0 || t >= ntime)
            continue;
        cplx v = w[i] / (double)L;
        x[t * 2 + 0] += v;
        x[t * 2 + 1] += v;
    }
    free(w);
    return 0;
}
