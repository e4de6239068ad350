/*
 * simus_oracle.c -- plain, slow FP64 reference of the SIMUS radio-frequency
 * synthesis (D. Garcia, "SIMUS: an open-source simulator for medical
 * ultrasound imaging. Part I: theory & examples").
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product library links, loads or
 * calls this file; only the tests, the smoke check and the benchmark's CPU
 * baseline leg do.  It shares no header, table or helper with the HIP path.
 *
 * Every quantity is evaluated term by term, in double precision, in the order
 * the paper states it: no tiling, no tables, no recurrences, no FFT.
 *
 * Readings of points the paper leaves open (they are listed with their
 * reasons in the design notes of the repository):
 *   - sinc(x) = sin(x)/x (unnormalised), as Eq. (10) requires.
 *   - a sub-element of an element of width 2b has half-width b/nu in the
 *     directivity, and weight 1 in the sum of Eq. (22).
 *   - nu follows Eq. (21) with lambda_min = c / (fc (1 + bw/2)), the upper
 *     -6 dB edge of the pulse-echo band.
 *   - soft-baffle cos(theta) uses the azimuthal angle of sin(theta) (Eq. 23).
 *   - a sub-element does not radiate behind its own face (z_local <= 0).
 *   - convex probe: apex at the origin, centre of curvature at (0, -R),
 *     chord pitch, flat elements split along their tangent.
 *   - RF(t_q) = Re sum_j X_j exp(-i w_j t_q), t_q = q/fs, no extra scale
 *     (time convention of Eq. 1).
 *   - frequency grid and RMS-field partition: see oracle_grid/oracle_pfield.
 *   - 2-D acoustics (Section V): G = exp(i (k + i k_a) r) / sqrt(r) D with no
 *     elevation term (Eqs. 36-38), r in the x-z plane (the point's y is not
 *     used), a factor 2b on the two-way spectrum (Eq. 38) and sqrt(2b) on the
 *     one-way field (Eq. 37), b the element half-width.
 *
 * Parity pins for every function live in tests/test_oracle_*.py.
 */
#include <complex.h>
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

typedef double complex cplx;

/* Probe, medium and pulse description, in SI units.  Mirrored by a ctypes
 * Structure in oracle/oracle.py; private to the oracle. */
typedef struct {
    int32_t n_elements;     /* N */
    int32_t nu;             /* sub-elements per element, >= 1 (resolved) */
    double fc;              /* centre frequency [Hz] */
    double pitch;           /* element pitch [m] */
    double width;           /* element width 2b [m] */
    double height;          /* element height h [m] */
    double elev_focus;      /* elevation focus R_f [m], may be +inf */
    double bandwidth;       /* pulse-echo fractional -6 dB bandwidth */
    double radius;          /* 0: linear array; > 0: convex radius [m] */
    int32_t baffle;         /* 0 soft, 1 rigid, 2 finite impedance (zeta) */
    int32_t pad0;
    double zeta;            /* impedance ratio for baffle 2 */
    double c;               /* speed of sound [m/s] */
    double alpha_db;        /* attenuation [dB/cm/MHz] */
    double fs;              /* sampling frequency [Hz] */
    double n_cycles;        /* n_lambda, number of wavelengths of the pulse */
    int32_t dim2;           /* 1: 2-D acoustics of Section V */
    int32_t pad1;
    int32_t n_gauss;        /* Gaussians of Eq. (12); 0: the four of Eq. (18) */
    int32_t pad2;
    const double *gauss;    /* [n_gauss][4]: Re A_g, Im A_g, Re B_g, Im B_g */
} orc_setup;

/* ------------------------------------------------------------------ */
/* Section II-B: elementary functions                                   */
/* ------------------------------------------------------------------ */

/* Unnormalised cardinal sine, the one Eq. (10) produces. */
static double sinc(double x)
{
    if (x == 0.0) return 1.0;
    return sin(x) / x;
}

/* Derivative of sinc, with its Taylor series near 0. */
static double dsinc(double x)
{
    if (fabs(x) < 1e-3) return -x / 3.0 + x * x * x / 30.0;
    return (cos(x) - sin(x) / x) / x;
}

/* Eq. (12): the rectangle function as a sum of G complex Gaussians,
 * Pi(u) ~ sum_g A_g exp(-B_g u^2).  The set is the caller's (su->gauss),
 * or by default the four of Eq. (18), whose coefficients 3 and 4 are the
 * complex conjugates of 1 and 2.  Returns G (at most ORC_MAX_GAUSS). */
#define ORC_MAX_GAUSS 64
static int gauss_set(const orc_setup *su, cplx A[ORC_MAX_GAUSS], cplx B[ORC_MAX_GAUSS])
{
    if (su->n_gauss > 0 && su->gauss) {
        int G = su->n_gauss < ORC_MAX_GAUSS ? su->n_gauss : ORC_MAX_GAUSS;
        for (int g = 0; g < G; ++g) {
            A[g] = su->gauss[4 * g] + I * su->gauss[4 * g + 1];
            B[g] = su->gauss[4 * g + 2] + I * su->gauss[4 * g + 3];
        }
        return G;
    }
    A[0] = 0.187 + 0.275 * I;  B[0] = 4.558 - 25.59 * I;
    A[1] = 0.288 - 1.954 * I;  B[1] = 8.598 - 7.924 * I;
    A[2] = conj(A[0]);         B[2] = conj(B[0]);
    A[3] = conj(A[1]);         B[3] = conj(B[1]);
    return 4;
}

/* Eqs. (14)-(16): elevation term delta(y, r, k) of the Gaussian
 * superposition model, principal square root. */
static cplx elevation_delta(const orc_setup *su, double y, double r, double k)
{
    cplx A[ORC_MAX_GAUSS], B[ORC_MAX_GAUSS];
    int G = gauss_set(su, A, B);
    double h = su->height;
    double inv_rf = 1.0 / su->elev_focus;   /* 0 when R_f = inf */
    cplx beta = -I * k * y / r;
    cplx gamma = I * k * y * y / (2.0 * r);
    cplx sum = 0.0;
    for (int g = 0; g < G; ++g) {
        cplx alpha = B[g] / (h * h) + I * k / 2.0 * (inv_rf - 1.0 / r);
        sum += A[g] * csqrt(M_PI / alpha) * cexp(beta * beta / (4.0 * alpha) + gamma);
    }
    return sum;
}

/* Partial derivatives of delta with respect to r and y (used by the
 * adjoint only). */
static void elevation_delta_grad(const orc_setup *su, double y, double r, double k,
                                 cplx *d_dr, cplx *d_dy)
{
    cplx A[ORC_MAX_GAUSS], B[ORC_MAX_GAUSS];
    int G = gauss_set(su, A, B);
    double h = su->height;
    double inv_rf = 1.0 / su->elev_focus;
    cplx beta = -I * k * y / r;
    cplx gamma = I * k * y * y / (2.0 * r);
    cplx dbeta_dr = I * k * y / (r * r), dbeta_dy = -I * k / r;
    cplx dgamma_dr = -I * k * y * y / (2.0 * r * r), dgamma_dy = I * k * y / r;
    cplx dalpha_dr = I * k / (2.0 * r * r);
    *d_dr = 0.0;
    *d_dy = 0.0;
    for (int g = 0; g < G; ++g) {
        cplx alpha = B[g] / (h * h) + I * k / 2.0 * (inv_rf - 1.0 / r);
        cplx term = A[g] * csqrt(M_PI / alpha) * cexp(beta * beta / (4.0 * alpha) + gamma);
        /* d/dr of [alpha^{-1/2} exp(beta^2/(4 alpha) + gamma)] / itself */
        cplx dlog_dr = -0.5 * dalpha_dr / alpha
                     + 2.0 * beta * dbeta_dr / (4.0 * alpha)
                     - beta * beta * dalpha_dr / (4.0 * alpha * alpha)
                     + dgamma_dr;
        cplx dlog_dy = 2.0 * beta * dbeta_dy / (4.0 * alpha) + dgamma_dy;
        *d_dr += term * dlog_dr;
        *d_dy += term * dlog_dy;
    }
}

/* Eq. (39): element directivity for the three baffle conditions, with the
 * sub-element half-width b_sub in the sinc of Eq. (10). */
static double directivity(const orc_setup *su, double sin_t, double cos_t, double k, double b_sub)
{
    double s = sinc(k * b_sub * sin_t);
    if (su->baffle == 1) return s;
    if (su->baffle == 2) return s * cos_t / (cos_t + su->zeta);
    return s * cos_t;
}

/* Eq. (21) with lambda_min at the upper -6 dB edge of the pulse-echo band. */
int32_t oracle_nu(double width, double fc, double bandwidth, double c)
{
    double lambda_min = c / (fc * (1.0 + bandwidth / 2.0));
    int32_t nu = (int32_t)ceil(width / lambda_min);
    return nu < 1 ? 1 : nu;
}

/* ------------------------------------------------------------------ */
/* Eq. (24) and its convex counterpart: sub-element centroids, face      */
/* tangents and normals.  n runs from 0 to nu*N-1 (paper: 1 .. nu*N).  */
/* ------------------------------------------------------------------ */
void oracle_subelements(const orc_setup *su, double *xc, double *zc,
                        double *tx, double *tz, double *nx, double *nz)
{
    int N = su->n_elements, nu = su->nu;
    double b = su->width / 2.0;
    for (int n1 = 1; n1 <= nu * N; ++n1) {
        int e = (n1 + nu - 1) / nu;                      /* ceil(n/nu), 1-based */
        double offset = b / nu * (2.0 * ((n1 - 1) % nu) - nu + 1.0);
        int i = n1 - 1;
        if (su->radius <= 0.0) {
            xc[i] = su->pitch / 2.0 * (2.0 * e - N - 1.0) + offset;   /* Eq. (24) */
            zc[i] = 0.0;
            tx[i] = 1.0; tz[i] = 0.0;
            nx[i] = 0.0; nz[i] = 1.0;
        } else {
            double R = su->radius;
            double dphi = 2.0 * asin(su->pitch / (2.0 * R));
            double phi = (e - (N + 1.0) / 2.0) * dphi;
            double ex = R * sin(phi), ez = R * cos(phi) - R;  /* element centre */
            tx[i] = cos(phi);  tz[i] = -sin(phi);
            nx[i] = sin(phi);  nz[i] = cos(phi);
            xc[i] = ex + offset * tx[i];
            zc[i] = ez + offset * tz[i];
        }
    }
}

/* ------------------------------------------------------------------ */
/* Section III: transmit pulse and transducer spectra                    */
/* ------------------------------------------------------------------ */

/* Eq. (25): spectrum of the rectangularly windowed sinusoid. */
void oracle_pulse_spectrum(const orc_setup *su, double w, double out[2])
{
    double wc = 2.0 * M_PI * su->fc;
    double T = su->n_cycles / su->fc;
    cplx sp = I * (sinc(T * (w - wc) / 2.0) - sinc(T * (w + wc) / 2.0));
    out[0] = creal(sp);
    out[1] = cimag(sp);
}

/* Eq. (27): transducer (pulse-echo) spectrum, generalised Gaussian. */
double oracle_transducer_spectrum(const orc_setup *su, double w)
{
    double wc = 2.0 * M_PI * su->fc;
    double wb = su->bandwidth * wc;
    double p = log(126.0) / log(2.0 * wc / wb);
    return exp(-log(2.0) * pow(2.0 * fabs(w - wc) / wb, p));
}

/* Eqs. (28) and (34): the two-way spectral weight S_P(w) S_T(w); in 2-D
 * also the factor 2b of Eq. (38). */
static cplx spectral_weight(const orc_setup *su, double w)
{
    double sp[2];
    oracle_pulse_spectrum(su, w, sp);
    double f2 = su->dim2 ? su->width : 1.0;
    return (sp[0] + I * sp[1]) * oracle_transducer_spectrum(su, w) * f2;
}

/* ------------------------------------------------------------------ */
/* Eqs. (19)-(20), (23), (39), (40): the field of one sub-element at a  */
/* point, without P_Tx and without the transmit delay.                  */
/* ------------------------------------------------------------------ */
typedef struct { double xc, zc, tx, tz, nx, nz; } subel;

static cplx green(const orc_setup *su, const subel *se, double X, double Y, double Z,
                  double k, double ka)
{
    if (su->dim2) Y = 0.0;                      /* the x-z plane */
    double dx = X - se->xc, dz = Z - se->zc;
    double xl = dx * se->tx + dz * se->tz;     /* along the face */
    double zl = dx * se->nx + dz * se->nz;     /* along the normal */
    if (zl <= 0.0) return 0.0;
    double rho = sqrt(xl * xl + zl * zl);
    double r = sqrt(dx * dx + Y * Y + dz * dz);
    double b_sub = su->width / 2.0 / su->nu;
    double D = directivity(su, xl / rho, zl / rho, k, b_sub);
    if (su->dim2) return cexp(I * (k + I * ka) * r) / sqrt(r) * D;   /* Eqs. (36)-(38) */
    cplx d = elevation_delta(su, Y, r, k);
    return cexp(I * (k + I * ka) * r) / r * D * d;
}

/* Gradient of green() with respect to the point coordinates (X, Y, Z). */
static cplx green_grad(const orc_setup *su, const subel *se, double X, double Y, double Z,
                       double k, double ka, cplx dG[3])
{
    dG[0] = dG[1] = dG[2] = 0.0;
    if (su->dim2) Y = 0.0;
    double dx = X - se->xc, dz = Z - se->zc;
    double xl = dx * se->tx + dz * se->tz;
    double zl = dx * se->nx + dz * se->nz;
    if (zl <= 0.0) return 0.0;
    double rho = sqrt(xl * xl + zl * zl);
    double r = sqrt(dx * dx + Y * Y + dz * dz);
    double b_sub = su->width / 2.0 / su->nu;
    double s_t = xl / rho, c_t = zl / rho;
    double u = k * b_sub * s_t;
    double sn = sinc(u), dsn = dsinc(u);
    double obl, dobl_dc;                        /* baffle factor and d/dcos */
    if (su->baffle == 1)      { obl = 1.0; dobl_dc = 0.0; }
    else if (su->baffle == 2) { obl = c_t / (c_t + su->zeta);
                                dobl_dc = su->zeta / ((c_t + su->zeta) * (c_t + su->zeta)); }
    else                      { obl = c_t; dobl_dc = 1.0; }
    double D = sn * obl;
    cplx d = 1.0, d_dr = 0.0, d_dy = 0.0;
    if (!su->dim2) {
        d = elevation_delta(su, Y, r, k);
        elevation_delta_grad(su, Y, r, k, &d_dr, &d_dy);
    }
    /* amplitude 1/r (3-D) or 1/sqrt(r) (2-D) */
    double apow = su->dim2 ? 0.5 : 1.0;
    cplx E = cexp(I * (k + I * ka) * r) / pow(r, apow);
    cplx G = E * D * d;
    /* partials of the local coordinates w.r.t. X, Y, Z */
    double dxl[3] = { se->tx, 0.0, se->tz };
    double dzl[3] = { se->nx, 0.0, se->nz };
    double dY[3] = { 0.0, su->dim2 ? 0.0 : 1.0, 0.0 };
    for (int a = 0; a < 3; ++a) {
        double drho = (xl * dxl[a] + zl * dzl[a]) / rho;
        double dr = (xl * dxl[a] + zl * dzl[a] + Y * dY[a]) / r;
        double ds_t = (dxl[a] * rho - xl * drho) / (rho * rho);
        double dc_t = (dzl[a] * rho - zl * drho) / (rho * rho);
        double dD = dsn * k * b_sub * ds_t * obl + sn * dobl_dc * dc_t;
        cplx dE = E * (I * (k + I * ka) - apow / r) * dr;
        cplx dd = d_dr * dr + d_dy * dY[a];
        dG[a] = dE * D * d + E * dD * d + E * D * dd;
    }
    return G;
}

static void load_subels(const orc_setup *su, subel *se)
{
    int M = su->n_elements * su->nu;
    double *buf = malloc(sizeof(double) * 6 * M);
    oracle_subelements(su, buf, buf + M, buf + 2 * M, buf + 3 * M, buf + 4 * M, buf + 5 * M);
    for (int n = 0; n < M; ++n) {
        se[n].xc = buf[n];         se[n].zc = buf[M + n];
        se[n].tx = buf[2 * M + n]; se[n].tz = buf[3 * M + n];
        se[n].nx = buf[4 * M + n]; se[n].nz = buf[5 * M + n];
    }
    free(buf);
}

/* Eq. (40): amplitude attenuation wavenumber for angular frequency w. */
static double attenuation_k(const orc_setup *su, double w)
{
    double k = w / su->c;
    return su->alpha_db / 8.69 * k * su->c / (2.0 * M_PI * 1e4);
}

/* One-way complex field of one sub-element (test hook). */
void oracle_green(const orc_setup *su, int32_t n, double X, double Y, double Z,
                  double w, double out[2])
{
    subel *se = malloc(sizeof(subel) * su->n_elements * su->nu);
    load_subels(su, se);
    cplx g = green(su, &se[n], X, Y, Z, w / su->c, attenuation_k(su, w));
    free(se);
    out[0] = creal(g);
    out[1] = cimag(g);
}

void oracle_delta(const orc_setup *su, double y, double r, double k, double out[2])
{
    cplx d = elevation_delta(su, y, r, k);
    out[0] = creal(d);
    out[1] = cimag(d);
}

double oracle_directivity(const orc_setup *su, double sin_t, double cos_t, double k, double b_sub)
{
    return directivity(su, sin_t, cos_t, k, b_sub);
}

/* ------------------------------------------------------------------ */
/* Frequency grid (the paper does not fix one for RF; reading):          */
/*   t_max = 2 r_max / c + max delay + 10/fc, r_max = max sub-element to */
/*   scatterer distance; nfft = smallest even 2^a 3^b 5^c >= fs t_max   */
/*   and >= n_t; candidate bins 1 <= j < nfft/2 with f_j < 2 fc; the    */
/*   evaluated band is the contiguous range spanning every candidate    */
/*   with |S_P S_T| >= eps * max |S_P S_T|.                             */
/* ------------------------------------------------------------------ */
static int smooth235(long n)
{
    while (n % 2 == 0) n /= 2;
    while (n % 3 == 0) n /= 3;
    while (n % 5 == 0) n /= 5;
    return n == 1;
}

/* Band of evaluated bins for a given nfft: out = {j_lo, n_bins}. */
void oracle_band(const orc_setup *su, int32_t nfft, double eps, int32_t out[2])
{
    double df = su->fs / nfft;
    int jmax = 0;
    for (int j = 1; j < nfft / 2 && j * df < 2.0 * su->fc; ++j) jmax = j;
    double wmax = 0.0;
    for (int j = 1; j <= jmax; ++j) {
        double m = cabs(spectral_weight(su, 2.0 * M_PI * j * df));
        if (m > wmax) wmax = m;
    }
    int lo = -1, hi = -2;
    for (int j = 1; j <= jmax; ++j) {
        double m = cabs(spectral_weight(su, 2.0 * M_PI * j * df));
        if (m >= eps * wmax && m > 0.0) {
            if (lo < 0) lo = j;
            hi = j;
        }
    }
    if (lo < 0) { out[0] = 1; out[1] = 0; return; }
    out[0] = lo;
    out[1] = hi - lo + 1;
}

/* out = {nfft, n_t, j_lo, n_bins}.  delays: [n_tx][N] seconds. */
void oracle_grid(const orc_setup *su, int32_t n_t_req, int32_t nfft_req, double eps,
                 int32_t n_tx, const double *delays,
                 int64_t n_scat, const double *x, const double *y, const double *z,
                 int32_t out[4])
{
    int M = su->n_elements * su->nu;
    subel *se = malloc(sizeof(subel) * M);
    load_subels(su, se);
    double rmax = 0.0;
    for (int64_t s = 0; s < n_scat; ++s)
        for (int n = 0; n < M; ++n) {
            double dx = x[s] - se[n].xc, dz = z[s] - se[n].zc;
            double yy = su->dim2 ? 0.0 : y[s];
            double r = sqrt(dx * dx + yy * yy + dz * dz);
            if (r > rmax) rmax = r;
        }
    free(se);
    double dmax = 0.0;
    for (int i = 0; i < n_tx * su->n_elements; ++i)
        if (delays[i] > dmax) dmax = delays[i];
    long nfft = nfft_req;
    if (nfft <= 0) {
        double tmax = 2.0 * rmax / su->c + dmax + 10.0 / su->fc;
        long nmin = (long)ceil(su->fs * tmax);
        if (n_t_req > nmin) nmin = n_t_req;
        nfft = nmin < 2 ? 2 : nmin;
        while (nfft % 2 != 0 || !smooth235(nfft)) ++nfft;
    }
    int32_t band[2];
    oracle_band(su, (int32_t)nfft, eps, band);
    out[0] = (int32_t)nfft;
    out[1] = n_t_req > 0 ? n_t_req : (int32_t)nfft;
    out[2] = band[0];
    out[3] = band[1];
}

/* ------------------------------------------------------------------ */
/* Eqs. (29)-(34): received element spectra, direct sum.                 */
/*   X[t][e][b] = P(w_j) sum_s R_s a_{s,t}(w_j) B_{e,s}(w_j)             */
/*   a_{s,t} = sum_n W_{t,e(n)} exp(i w tau_{t,e(n)}) G_{n,s}  (Eq. 29)  */
/*   B_{e,s} = sum over the nu sub-elements of e of G_{m,s}  (Eq. 33)    */
/* bins[b] are absolute bin indices j (w_j = 2 pi j fs / nfft).          */
/* X is laid out [n_tx][N][n_sel][2].                                    */
/* ------------------------------------------------------------------ */
void oracle_spectrum(const orc_setup *su, int32_t nfft, int32_t n_tx,
                     const double *delays, const double *apod,
                     int64_t n_scat, const double *x, const double *y, const double *z,
                     const double *R, int32_t n_sel, const int32_t *bins, double *X)
{
    int N = su->n_elements, nu = su->nu, M = N * nu;
    subel *se = malloc(sizeof(subel) * M);
    load_subels(su, se);
    #pragma omp parallel for schedule(dynamic, 1)
    for (int b = 0; b < n_sel; ++b) {
        double w = 2.0 * M_PI * bins[b] * su->fs / nfft;
        double k = w / su->c, ka = attenuation_k(su, w);
        cplx P = spectral_weight(su, w);
        cplx *G = malloc(sizeof(cplx) * M);
        cplx *acc = calloc((size_t)n_tx * N, sizeof(cplx));
        for (int64_t s = 0; s < n_scat; ++s) {
            for (int n = 0; n < M; ++n) G[n] = green(su, &se[n], x[s], y[s], z[s], k, ka);
            for (int t = 0; t < n_tx; ++t) {
                cplx a = 0.0;                                   /* Eq. (29) */
                for (int n = 0; n < M; ++n) {
                    int e = n / nu;
                    a += apod[t * N + e] * cexp(I * w * delays[t * N + e]) * G[n];
                }
                for (int e = 0; e < N; ++e) {                   /* Eqs. (31)-(33) */
                    cplx Be = 0.0;
                    for (int m = e * nu; m < (e + 1) * nu; ++m) Be += G[m];
                    acc[t * N + e] += R[s] * a * Be;
                }
            }
        }
        for (int t = 0; t < n_tx; ++t)
            for (int e = 0; e < N; ++e) {
                cplx v = P * acc[t * N + e];                    /* Eq. (34) */
                size_t o = (((size_t)t * N + e) * n_sel + b) * 2;
                X[o] = creal(v);
                X[o + 1] = cimag(v);
            }
        free(G);
        free(acc);
    }
    free(se);
}

/* ------------------------------------------------------------------ */
/* Eq. (1), discretised: rf[c][q] = Re sum_b X[c][b] exp(-2 pi i j_b q / nfft) */
/* X: [n_chan][n_bins][2], rf: [n_chan][n_t].                            */
/* ------------------------------------------------------------------ */
void oracle_rf_from_spectrum(int32_t nfft, int32_t n_t, int32_t n_bins, const int32_t *bins,
                             int64_t n_chan, const double *X, double *rf)
{
    #pragma omp parallel for schedule(static)
    for (int64_t ch = 0; ch < n_chan; ++ch)
        for (int q = 0; q < n_t; ++q) {
            double acc = 0.0;
            for (int b = 0; b < n_bins; ++b) {
                long m = ((long)bins[b] * q) % nfft;
                double ph = -2.0 * M_PI * (double)m / nfft;
                const double *xv = X + (ch * n_bins + b) * 2;
                acc += xv[0] * cos(ph) - xv[1] * sin(ph);
            }
            rf[ch * n_t + q] = acc;
        }
}

/* Adjoint of the step above: Lam[c][b] = sum_q rho[c][q] exp(-2 pi i j_b q / nfft). */
void oracle_residual_spectrum(int32_t nfft, int32_t n_t, int32_t n_bins, const int32_t *bins,
                              int64_t n_chan, const double *rho, double *Lam)
{
    #pragma omp parallel for schedule(static)
    for (int64_t ch = 0; ch < n_chan; ++ch)
        for (int b = 0; b < n_bins; ++b) {
            double re = 0.0, im = 0.0;
            for (int q = 0; q < n_t; ++q) {
                long m = ((long)bins[b] * q) % nfft;
                double ph = -2.0 * M_PI * (double)m / nfft;
                re += rho[ch * n_t + q] * cos(ph);
                im += rho[ch * n_t + q] * sin(ph);
            }
            Lam[(ch * n_bins + b) * 2] = re;
            Lam[(ch * n_bins + b) * 2 + 1] = im;
        }
}

/* ------------------------------------------------------------------ */
/* Gradient of L = 1/2 sum (rf - obs)^2 with respect to R_s, X_s, Y_s,   */
/* Z_s for the selected scatterers, given Lam = residual spectrum        */
/* [n_tx][N][n_bins][2] over the bins in `bins`:                         */
/*   dL/dR_s  = Re sum_j P_j sum_t a_{s,t} b_{s,t}                       */
/*   dL/dxi_s = R_s Re sum_j P_j sum_t (a'_{s,t} b_{s,t} + a_{s,t} b'_{s,t}) */
/*   with b_{s,t} = sum_e Lam_{t,e} B_{e,s}; primes are d/dxi_s.         */
/* Output arrays are [n_sel_s]; any may be NULL.                         */
/* ------------------------------------------------------------------ */
void oracle_adjoint(const orc_setup *su, int32_t nfft, int32_t n_tx,
                    const double *delays, const double *apod,
                    const double *x, const double *y, const double *z, const double *R,
                    int32_t n_bins, const int32_t *bins, const double *Lam,
                    int32_t n_sel_s, const int64_t *sel_s,
                    double *dR, double *dX, double *dY, double *dZ)
{
    int N = su->n_elements, nu = su->nu, M = N * nu;
    subel *se = malloc(sizeof(subel) * M);
    load_subels(su, se);
    #pragma omp parallel for schedule(dynamic, 1)
    for (int i = 0; i < n_sel_s; ++i) {
        int64_t s = sel_s[i];
        cplx *G = malloc(sizeof(cplx) * M);
        cplx *dG = malloc(sizeof(cplx) * M * 3);
        double gR = 0.0, gx[3] = { 0.0, 0.0, 0.0 };
        for (int b = 0; b < n_bins; ++b) {
            double w = 2.0 * M_PI * bins[b] * su->fs / nfft;
            double k = w / su->c, ka = attenuation_k(su, w);
            cplx P = spectral_weight(su, w);
            for (int n = 0; n < M; ++n) G[n] = green_grad(su, &se[n], x[s], y[s], z[s], k, ka, &dG[3 * n]);
            for (int t = 0; t < n_tx; ++t) {
                cplx a = 0.0, bb = 0.0, da[3] = { 0, 0, 0 }, db[3] = { 0, 0, 0 };
                for (int n = 0; n < M; ++n) {
                    int e = n / nu;
                    cplx W = apod[t * N + e] * cexp(I * w * delays[t * N + e]);
                    const double *lv = Lam + (((size_t)t * N + e) * n_bins + b) * 2;
                    cplx L = lv[0] + I * lv[1];
                    a += W * G[n];
                    bb += L * G[n];
                    for (int c = 0; c < 3; ++c) {
                        da[c] += W * dG[3 * n + c];
                        db[c] += L * dG[3 * n + c];
                    }
                }
                gR += creal(P * a * bb);
                for (int c = 0; c < 3; ++c) gx[c] += R[s] * creal(P * (da[c] * bb + a * db[c]));
            }
        }
        if (dR) dR[i] = gR;
        if (dX) dX[i] = gx[0];
        if (dY) dY[i] = gx[1];
        if (dZ) dZ[i] = gx[2];
        free(G);
        free(dG);
    }
    free(se);
}

/* ------------------------------------------------------------------ */
/* Section VII: RMS pressure field, Eqs. (22), (28), (41), (42).         */
/* Reading: dw_max = 2 pi / max over points and sub-elements of          */
/* (r/c + delay); N_f = ceil(2 wc / dw_max); nodes w_j = 2 wc j / N_f,   */
/* j = 0..N_f; the Riemann weight is the node spacing 2 wc / N_f.        */
/* ------------------------------------------------------------------ */
int32_t oracle_pfield_nf(const orc_setup *su, const double *delays,
                         int64_t n_pts, const double *X, const double *Y, const double *Z)
{
    int N = su->n_elements, nu = su->nu, M = N * nu;
    subel *se = malloc(sizeof(subel) * M);
    load_subels(su, se);
    double tmax = 0.0;
    for (int64_t p = 0; p < n_pts; ++p)
        for (int n = 0; n < M; ++n) {
            double dx = X[p] - se[n].xc, dz = Z[p] - se[n].zc;
            double yy = su->dim2 ? 0.0 : Y[p];
            double r = sqrt(dx * dx + yy * yy + dz * dz);
            double t = r / su->c + delays[n / nu];
            if (t > tmax) tmax = t;
        }
    free(se);
    double wc = 2.0 * M_PI * su->fc;
    double dw = 2.0 * M_PI / tmax;
    return (int32_t)ceil(2.0 * wc / dw);
}

/* One-way field at points (Eq. 22 without P_Tx) for given angular
 * frequencies: out [n_pts][n_w][2]. */
void oracle_field(const orc_setup *su, const double *delays, const double *apod,
                  int32_t n_w, const double *ws,
                  int64_t n_pts, const double *X, const double *Y, const double *Z, double *out)
{
    int N = su->n_elements, nu = su->nu, M = N * nu;
    subel *se = malloc(sizeof(subel) * M);
    load_subels(su, se);
    #pragma omp parallel for schedule(dynamic, 16)
    for (int64_t p = 0; p < n_pts; ++p)
        for (int j = 0; j < n_w; ++j) {
            double w = ws[j];
            double k = w / su->c, ka = attenuation_k(su, w);
            cplx acc = 0.0;
            for (int n = 0; n < M; ++n) {
                int e = n / nu;
                acc += apod[e] * cexp(I * w * delays[e]) * green(su, &se[n], X[p], Y[p], Z[p], k, ka);
            }
            out[(p * n_w + j) * 2] = creal(acc);
            out[(p * n_w + j) * 2 + 1] = cimag(acc);
        }
    free(se);
}

void oracle_pfield(const orc_setup *su, const double *delays, const double *apod, int32_t n_f,
                   int64_t n_pts, const double *X, const double *Y, const double *Z, double *prms)
{
    int N = su->n_elements, nu = su->nu, M = N * nu;
    subel *se = malloc(sizeof(subel) * M);
    load_subels(su, se);
    double wc = 2.0 * M_PI * su->fc;
    double dw = 2.0 * wc / n_f;
    #pragma omp parallel for schedule(dynamic, 16)
    for (int64_t p = 0; p < n_pts; ++p) {
        double sum = 0.0;
        for (int j = 0; j <= n_f; ++j) {
            double w = j * dw;
            double k = w / su->c, ka = attenuation_k(su, w);
            double sp[2];
            oracle_pulse_spectrum(su, w, sp);
            cplx ptx = (sp[0] + I * sp[1]) * sqrt(oracle_transducer_spectrum(su, w));  /* Eq. (28) */
            if (su->dim2) ptx *= sqrt(su->width);                                  /* Eq. (37) */
            cplx acc = 0.0;
            for (int n = 0; n < M; ++n) {
                int e = n / nu;
                acc += apod[e] * cexp(I * w * delays[e]) * green(su, &se[n], X[p], Y[p], Z[p], k, ka);
            }
            cplx P = ptx * acc;                                                    /* Eq. (22) */
            sum += creal(P) * creal(P) + cimag(P) * cimag(P);
        }
        prms[p] = sqrt(dw * sum);                                                  /* Eq. (42) */
    }
    free(se);
}
