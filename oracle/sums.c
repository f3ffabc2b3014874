/* Plain FP64 summation loops of the oracle (test infrastructure only; never
 * linked into the product library).
 *
 * Each routine is a direct sum written out from its definition, one output at
 * a time, OpenMP over outputs, with Neumaier-compensated accumulation so that
 * the sums are accurate to a few ulps of the largest term even for 10^6 terms.
 *
 *   osum_dft_bins   S_k = sum_j z_j exp(-2 pi i (j k mod nfft) / nfft)
 *                   (the DFT of Sec. VI B with the data zero-padded to nfft)
 *   osum_dft_freqs  S(f) = sum_j z_j exp(-2 pi i f j dt)   (continuous f)
 *   osum_phase      S(f) = sum_j w_j exp(-2 pi i (f tau_j + psi_j))
 *                   (the matched-filter integrals of Eqs. Fab on the detector
 *                    grid; phase split as in Eqs. pham/phas, in cycles)
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>

typedef struct { double s, c; } nsum;   /* Neumaier accumulator */

static inline void nadd(nsum *a, double v) {
    double t = a->s + v;
    if (fabs(a->s) >= fabs(v)) a->c += (a->s - t) + v;
    else                       a->c += (v - t) + a->s;
    a->s = t;
}
static inline double nval(const nsum *a) { return a->s + a->c; }

static const double TWO_PI = 6.283185307179586476925286766559;

/* exp(-2 pi i * cyc) for a phase given in cycles: reduce to [-1/2, 1/2]. */
static inline void cis_cycles(double cyc, double *c, double *s) {
    double r = cyc - nearbyint(cyc);
    *c = cos(TWO_PI * r);
    *s = -sin(TWO_PI * r);
}

void osum_dft_bins(const double *zre, const double *zim, int64_t n, int64_t nfft,
                   const int64_t *k, int64_t nk, double *out_re, double *out_im) {
    double *ct = (double *)malloc(sizeof(double) * (size_t)nfft);
    double *st = (double *)malloc(sizeof(double) * (size_t)nfft);
    for (int64_t m = 0; m < nfft; ++m) {
        ct[m] = cos(TWO_PI * (double)m / (double)nfft);
        st[m] = -sin(TWO_PI * (double)m / (double)nfft);
    }
    #pragma omp parallel for schedule(dynamic, 4)
    for (int64_t q = 0; q < nk; ++q) {
        nsum re = {0, 0}, im = {0, 0};
        int64_t kk = ((k[q] % nfft) + nfft) % nfft;
        for (int64_t j = 0; j < n; ++j) {
            int64_t m = (int64_t)(((__int128)j * kk) % nfft);
            double c = ct[m], s = st[m];
            nadd(&re, zre[j] * c - zim[j] * s);
            nadd(&im, zre[j] * s + zim[j] * c);
        }
        out_re[q] = nval(&re);
        out_im[q] = nval(&im);
    }
    free(ct);
    free(st);
}

void osum_dft_freqs(const double *zre, const double *zim, int64_t n, double dt,
                    const double *f, int64_t nf, double *out_re, double *out_im) {
    #pragma omp parallel for schedule(dynamic, 4)
    for (int64_t q = 0; q < nf; ++q) {
        nsum re = {0, 0}, im = {0, 0};
        for (int64_t j = 0; j < n; ++j) {
            double c, s;
            cis_cycles(f[q] * ((double)j * dt), &c, &s);
            nadd(&re, zre[j] * c - zim[j] * s);
            nadd(&im, zre[j] * s + zim[j] * c);
        }
        out_re[q] = nval(&re);
        out_im[q] = nval(&im);
    }
}

/* Two real weight series share one phase: returns S_a and S_b together. */
void osum_phase(const double *wa, const double *wb, const double *tau,
                const double *psi, int64_t n, const double *f, int64_t nf,
                double *sa_re, double *sa_im, double *sb_re, double *sb_im) {
    #pragma omp parallel for schedule(dynamic, 4)
    for (int64_t q = 0; q < nf; ++q) {
        nsum ar = {0, 0}, ai = {0, 0}, br = {0, 0}, bi = {0, 0};
        for (int64_t j = 0; j < n; ++j) {
            double c, s;
            cis_cycles(f[q] * tau[j] + psi[j], &c, &s);
            nadd(&ar, wa[j] * c);
            nadd(&ai, wa[j] * s);
            nadd(&br, wb[j] * c);
            nadd(&bi, wb[j] * s);
        }
        sa_re[q] = nval(&ar);
        sa_im[q] = nval(&ai);
        sb_re[q] = nval(&br);
        sb_im[q] = nval(&bi);
    }
}
