/* Host-sanitizer driver for the C oracle (test infrastructure): runs every
 * exported oracle routine on small inputs in buffers of exactly the documented
 * sizes, plus its error paths, so that AddressSanitizer and UBSan see any
 * out-of-bounds access, overflow or undefined operation.  Exit status 0 when
 * every call returned what it documents. */
#include <math.h>
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>

typedef struct {
    int nsub;
    double f_centre;
    double bw;
    int nfft;
    int noverlap;
    int nchan;
    int ndec;
    int chirp_ref;
    int sign;
} orc_cfg;

void orc_dft(const double *x_ri, double *y_ri, long n, int sign);
int orc_fft(const double *x_ri, double *y_ri, long n, int sign);
int orc_tblk(const orc_cfg *c);
int orc_subband_block(const orc_cfg *c, int kind, const void *x_sub, long ntime, int s, int b,
                      const double *dms, int ndm, double *F);
int orc_dm_gradient(const orc_cfg *c, int kind, const void *x_sub, long ntime, int s, int b,
                    const double *dms, int ndm, const double *G, double *dldm,
                    double *absterms);
int orc_voltage_gradient(const orc_cfg *c, int kind, const void *x_sub, long ntime, int s, int b,
                         double dm, const double *G, double *gx);
int orc_dedisperse(const orc_cfg *c, int kind, const void *x, long ntime, int nblock,
                   const double *dms, int ndm, double *out, int nthreads);
int orc_inject_impulse(const orc_cfg *c, int s, double *x_ri, long ntime, double dm, long n0,
                       double amp, long L);

static int failures = 0;
#define EXPECT(cond)                                                   \
    do {                                                               \
        if (!(cond)) {                                                 \
            fprintf(stderr, "FAILED %s:%d: %s\n", __FILE__, __LINE__, #cond); \
            ++failures;                                                \
        }                                                              \
    } while (0)

static double urand(unsigned *s) {
    *s = *s * 1664525u + 1013904223u;
    return (*s >> 8) * (1.0 / 16777216.0) - 0.5;
}

static void run_cfg(int chirp_ref, int sign) {
    const orc_cfg c = {2, 120.0, 0.1953125, 1024, 256, 8, 4, chirp_ref, sign};
    const int nblock = 3, ndm = 3;
    const long ntime = (long)nblock * (c.nfft - c.noverlap) + c.noverlap;
    const int tblk = orc_tblk(&c);
    EXPECT(tblk == (1024 / 8 - 256 / 8) / 4);
    const double dms[3] = {0.0, 2.5, -4.0};
    unsigned seed = 7u + (unsigned)chirp_ref;

    /* complex double stream, impulse injected into it */
    double *x64 = malloc(sizeof(double) * (size_t)c.nsub * ntime * 4);
    for (long i = 0; i < (long)c.nsub * ntime * 4; ++i)
        x64[i] = urand(&seed);
    for (int s = 0; s < c.nsub; ++s)
        EXPECT(orc_inject_impulse(&c, s, x64 + (size_t)s * ntime * 4, ntime, 2.5, 600, 20.0,
                                  2048) == 0);
    /* the window may reach past both ends of the stream */
    EXPECT(orc_inject_impulse(&c, 0, x64, ntime, 2.5, 3, 1.0, 1024) == 0);
    EXPECT(orc_inject_impulse(&c, 0, x64, ntime, 2.5, ntime - 2, 1.0, 1024) == 0);
    EXPECT(orc_inject_impulse(&c, 0, x64, ntime, 2.5, 10, 1.0, 1000) == -1);

    /* the same stream as cf32 and ci8 */
    float *x32 = malloc(sizeof(float) * (size_t)c.nsub * ntime * 4);
    int8_t *x8 = malloc((size_t)c.nsub * ntime * 4);
    for (long i = 0; i < (long)c.nsub * ntime * 4; ++i) {
        x32[i] = (float)x64[i];
        double q = rint(16.0 * x64[i]);
        x8[i] = (int8_t)(q > 127 ? 127 : q < -127 ? -127 : q);
    }
    const long nout = (long)ndm * nblock * tblk * c.nsub * c.nchan;
    double *out = malloc(sizeof(double) * nout);
    const void *xs[3] = {x32, x8, x64};
    for (int kind = 0; kind < 3; ++kind) {
        EXPECT(orc_dedisperse(&c, kind, xs[kind], ntime, nblock, dms, ndm, out, 3) == 0);
        for (long i = 0; i < nout; ++i)
            EXPECT(isfinite(out[i]) && out[i] >= 0.0);
    }
    /* stream too short for the blocks asked for */
    EXPECT(orc_dedisperse(&c, 2, x64, ntime - 1, nblock, dms, ndm, out, 1) == -2);

    double *F = malloc(sizeof(double) * ndm * tblk * c.nchan);
    double *G = malloc(sizeof(double) * ndm * tblk * c.nchan);
    for (long i = 0; i < (long)ndm * tblk * c.nchan; ++i)
        G[i] = urand(&seed);
    EXPECT(orc_subband_block(&c, 2, x64, ntime, 0, nblock - 1, dms, ndm, F) == 0);
    EXPECT(orc_subband_block(&c, 2, x64, ntime, 0, nblock, dms, ndm, F) == -2);
    double dl[3], ab[3];
    EXPECT(orc_dm_gradient(&c, 2, x64, ntime, 1, 1, dms, ndm, G, dl, ab) == 0);
    for (int d = 0; d < ndm; ++d)
        EXPECT(ab[d] >= fabs(dl[d]));
    EXPECT(orc_dm_gradient(&c, 1, x8, ntime, 1, 0, dms, ndm, G, dl, NULL) == 0);
    EXPECT(orc_dm_gradient(&c, 0, x32, ntime, 1, nblock, dms, ndm, G, dl, ab) == -2);
    double *gx = calloc((size_t)ntime * 4, sizeof(double));
    for (int b = 0; b < nblock; ++b)
        EXPECT(orc_voltage_gradient(&c, 2, x64, ntime, 0, b, 2.5, G + 0, gx) == 0);
    EXPECT(orc_voltage_gradient(&c, 2, x64, ntime, 0, nblock, 2.5, G, gx) == -2);
    free(gx);
    free(F);
    free(G);
    free(out);
    free(x8);
    free(x32);
    free(x64);
}

int main(void) {
    /* transforms: definition and FFT on exactly-sized buffers */
    for (long n = 1; n <= 64; n *= 2) {
        double *x = malloc(sizeof(double) * 2 * n), *y = malloc(sizeof(double) * 2 * n);
        double *z = malloc(sizeof(double) * 2 * n);
        unsigned seed = (unsigned)n;
        for (long i = 0; i < 2 * n; ++i)
            x[i] = urand(&seed);
        orc_dft(x, y, n, -1);
        EXPECT(orc_fft(x, z, n, -1) == 0);
        for (long i = 0; i < 2 * n; ++i)
            EXPECT(fabs(y[i] - z[i]) <= 1e-12 * n);
        free(x);
        free(y);
        free(z);
    }
    double t[6] = {0};
    EXPECT(orc_fft(t, t, 3, 1) == -1);

    /* invalid plans are refused before any work */
    const orc_cfg bad[] = {
        {0, 120.0, 0.2, 1024, 256, 8, 4, 0, -1},      /* no subband */
        {2, 120.0, 0.2, 1000, 256, 8, 4, 0, -1},      /* N not a power of two */
        {2, 120.0, 0.2, 1024, 1024, 8, 4, 0, -1},     /* overlap = N */
        {2, 120.0, 0.2, 1024, 250, 8, 4, 0, -1},      /* overlap not a multiple of 2 n_c */
        {2, 120.0, 0.2, 1024, 256, 8, 5, 0, -1},      /* ndec does not divide M - n_d */
        {2, 0.1, 0.2, 1024, 256, 8, 4, 0, -1},        /* band below 0 Hz */
        {2, 120.0, 0.2, 1024, 256, 8, 4, 2, -1},      /* bad nu0 mode */
        {2, 120.0, 0.2, 1024, 256, 8, 4, 0, 0},       /* bad sign */
    };
    double dm = 1.0, o[1];
    for (size_t i = 0; i < sizeof(bad) / sizeof(bad[0]); ++i)
        EXPECT(orc_dedisperse(&bad[i], 2, t, 1, 1, &dm, 1, o, 1) == -1);

    for (int ref = 0; ref < 2; ++ref)
        for (int sign = -1; sign <= 1; sign += 2)
            run_cfg(ref, sign);
    if (failures)
        fprintf(stderr, "%d failures\n", failures);
    else
        printf("oracle sanitizer run: ok\n");
    return failures ? 1 : 0;
}
