// Host planning for libsimus (see plan.hpp).
#include "plan.hpp"

#include "eq18.hpp"

#include <algorithm>
#include <cmath>
#include <limits>

namespace simus {

namespace {

void require(bool ok, const char* what)
{
    if (!ok) throw Error{SIMUS_EINVAL, what};
}

bool finite_pos(double v) { return std::isfinite(v) && v > 0; }

}  // namespace

int nu_from_width(double width, double fc, double bandwidth, double c)
{
    // Eq. (21); the shortest wavelength is taken at the upper -6 dB edge of
    // the pulse-echo band, fc (1 + bw / 2).
    const double lambda_min = c / (fc * (1.0 + 0.5 * bandwidth));
    const double ratio = width / lambda_min;
    int nu = static_cast<int>(std::ceil(ratio));
    return std::max(nu, 1);
}

Probe make_probe(const simus_probe* p, const simus_medium* m, const simus_options* o)
{
    require(p && m && o, "probe, medium and options must be non-NULL");
    Probe P;
    require(p->n_elements >= 1 && p->n_elements <= 4096, "probe.n_elements must be in [1, 4096]");
    require(finite_pos(p->fc), "probe.fc must be > 0");
    require(finite_pos(p->pitch), "probe.pitch must be > 0");
    require(finite_pos(p->width) && p->width <= p->pitch * (1 + 1e-12),
            "probe.width must be in (0, pitch]");
    require(finite_pos(p->height), "probe.height must be > 0");
    require(p->elev_focus > 0 && !std::isnan(p->elev_focus), "probe.elev_focus must be > 0 (inf allowed)");
    require(std::isfinite(p->bandwidth) && p->bandwidth > 0 && p->bandwidth < 2,
            "probe.bandwidth must be in (0, 2)");
    require(std::isfinite(p->radius) && p->radius >= 0, "probe.radius must be >= 0");
    require(p->baffle >= 0 && p->baffle <= 2, "probe.baffle must be 0, 1 or 2");
    require(std::isfinite(p->zeta) && p->zeta >= 0, "probe.zeta must be >= 0");
    if (p->radius > 0) require(p->pitch < 2 * p->radius, "convex probe: pitch must be < 2 radius");
    require(finite_pos(m->c), "medium.c must be > 0");
    require(std::isfinite(m->alpha_db) && m->alpha_db >= 0, "medium.alpha_db must be >= 0");
    require(finite_pos(o->fs) && o->fs > 2 * p->fc, "options.fs must be > 2 fc");
    require(finite_pos(o->n_cycles), "options.n_cycles must be > 0");
    require(std::isfinite(o->spectral_eps) && o->spectral_eps >= 0 && o->spectral_eps < 1,
            "options.spectral_eps must be in [0, 1)");
    require(o->nu >= 0 && o->nu <= 64, "options.nu must be in [0, 64]");
    require(o->nfft >= 0 && o->n_t >= 0, "options.nfft and options.n_t must be >= 0");
    require(o->nfft % 2 == 0, "options.nfft must be even");
    require(o->n_gauss >= 0 && o->n_gauss <= SIMUS_MAX_GAUSS, "options.n_gauss must be in [0, 32]");
    require(o->n_gauss == 0 || o->gauss != nullptr, "options.gauss must be non-NULL when n_gauss > 0");
    for (int g = 0; g < o->n_gauss; ++g) {
        const double* c = o->gauss + 4 * g;
        require(std::isfinite(c[0]) && std::isfinite(c[1]) && std::isfinite(c[2]) && std::isfinite(c[3]),
                "options.gauss must be finite");
        require(c[2] > 0, "options.gauss: Re B_g must be > 0");
    }
    require(o->tile_scat >= 0, "options.tile_scat must be >= 0");
    require((o->flags & ~(SIMUS_FLAG_NO_MFMA | SIMUS_FLAG_PERSISTENT | SIMUS_FLAG_NO_DELTA_TABLE |
                          SIMUS_FLAG_2D | SIMUS_FLAG_STATIC | SIMUS_FLAG_ALT_SHAPE |
                          SIMUS_FLAG_FP32_PRODUCTS)) == 0,
            "options.flags has unknown bits");

    P.N = p->n_elements;
    P.baffle = p->baffle;
    P.fc = p->fc;
    P.pitch = p->pitch;
    P.width = p->width;
    P.height = p->height;
    P.elev_focus = p->elev_focus;
    P.bandwidth = p->bandwidth;
    P.radius = p->radius;
    P.zeta = p->zeta;
    P.c = m->c;
    P.alpha_db = m->alpha_db;
    P.fs = o->fs;
    P.n_cycles = o->n_cycles;
    P.eps = o->spectral_eps;
    P.dim2 = (o->flags & SIMUS_FLAG_2D) != 0;
    if (o->n_gauss > 0) {
        for (int g = 0; g < o->n_gauss; ++g) {
            const double* c = o->gauss + 4 * g;
            P.gA.emplace_back(c[0], c[1]);
            P.gB.emplace_back(c[2], c[3]);
        }
    } else {
        // Eq. (18): coefficients 3 and 4 are the conjugates of 1 and 2
        for (int g = 0; g < 4; ++g) {
            P.gA.emplace_back(eq18::Ar[g], eq18::Ai[g]);
            P.gB.emplace_back(eq18::Br[g], eq18::Bi[g]);
        }
    }
    P.nu = o->nu > 0 ? o->nu : nu_from_width(P.width, P.fc, P.bandwidth, P.c);
    P.M = P.nu * P.N;
    require(P.M <= 1024, "nu * n_elements must be <= 1024");
    return P;
}

SubElements sub_elements(const Probe& P)
{
    SubElements S;
    const int M = P.M;
    S.xc.resize(M);
    S.zc.resize(M);
    S.tx.resize(M);
    S.tz.resize(M);
    S.nx.resize(M);
    S.nz.resize(M);
    const double half_w = 0.5 * P.width;
    const double dphi = P.convex() ? 2.0 * std::asin(P.pitch / (2.0 * P.radius)) : 0.0;
    for (int e = 0; e < P.N; ++e) {
        // element centre and face frame
        double cx, cz, tx = 1, tz = 0, nx = 0, nz = 1;
        const double idx = e - 0.5 * (P.N - 1);      // signed element index about the middle
        if (!P.convex()) {
            cx = idx * P.pitch;
            cz = 0;
        } else {
            const double phi = idx * dphi;
            cx = P.radius * std::sin(phi);
            cz = P.radius * std::cos(phi) - P.radius;
            tx = std::cos(phi);
            tz = -std::sin(phi);
            nx = std::sin(phi);
            nz = std::cos(phi);
        }
        for (int i = 0; i < P.nu; ++i) {
            // Eq. (24): sub-element i of nu sits at (2i - nu + 1) b / nu along the face
            const double off = (2.0 * i - P.nu + 1.0) * half_w / P.nu;
            const int n = e * P.nu + i;
            S.xc[n] = cx + off * tx;
            S.zc[n] = cz + off * tz;
            S.tx[n] = tx;
            S.tz[n] = tz;
            S.nx[n] = nx;
            S.nz[n] = nz;
        }
    }
    return S;
}

std::complex<double> pulse_spectrum(const Probe& P, double w)
{
    // Eq. (25) with the unnormalised sinc.
    const double wc = 2 * M_PI * P.fc;
    const double T = P.n_cycles / P.fc;
    auto sinc = [](double u) { return u == 0 ? 1.0 : std::sin(u) / u; };
    return {0.0, sinc(0.5 * T * (w - wc)) - sinc(0.5 * T * (w + wc))};
}

double transducer_spectrum(const Probe& P, double w)
{
    // Eq. (27): generalised Gaussian, -6 dB pulse-echo bandwidth bw,
    // S_T(0) = 2^-126 (Eq. 49).
    const double wc = 2 * M_PI * P.fc;
    const double wb = P.bandwidth * wc;
    const double p = std::log(126.0) / std::log(2.0 * wc / wb);
    const double u = 2.0 * std::abs(w - wc) / wb;
    return std::exp(-M_LN2 * std::pow(u, p));
}

int64_t next_fft_size(int64_t n)
{
    int64_t m = std::max<int64_t>(n, 2);
    if (m % 2) ++m;
    for (;; m += 2) {
        int64_t r = m;
        for (int f : {2, 3, 5})
            while (r % f == 0) r /= f;
        if (r == 1) return m;
    }
}

Band make_band(const Probe& P, int nfft, int n_t)
{
    Band B;
    B.nfft = nfft;
    B.n_t = n_t > 0 ? n_t : nfft;
    B.df = P.fs / nfft;
    int last = 0;
    for (int j = 1; j < nfft / 2; ++j) {
        if (j * B.df >= 2 * P.fc) break;
        last = j;
    }
    std::vector<double> mag(last + 1, 0.0);
    double peak = 0;
    for (int j = 1; j <= last; ++j) {
        const double w = 2 * M_PI * j * B.df;
        mag[j] = std::abs(pulse_spectrum(P, w)) * transducer_spectrum(P, w);
        peak = std::max(peak, mag[j]);
    }
    int lo = 0, hi = -1;
    for (int j = 1; j <= last; ++j) {
        if (mag[j] > 0 && mag[j] >= P.eps * peak) {
            if (lo == 0) lo = j;
            hi = j;
        }
    }
    if (lo == 0) {
        B.j_lo = 1;
        B.n_bins = 0;
    } else {
        B.j_lo = lo;
        B.n_bins = hi - lo + 1;
    }
    return B;
}

double max_distance(const SubElements& S, int64_t n, const float* x, const float* y,
                    const float* z)
{
    double best = 0;
    const size_t M = S.xc.size();
    for (int64_t s = 0; s < n; ++s) {
        const double yy = y ? double(y[s]) : 0.0;
        for (size_t m = 0; m < M; ++m) {
            const double dx = double(x[s]) - S.xc[m], dz = double(z[s]) - S.zc[m];
            best = std::max(best, dx * dx + dz * dz + yy * yy);
        }
    }
    return std::sqrt(best);
}

void check_domain(const Probe& P, const SubElements& S, int64_t n, const float* x,
                  const float* y, const float* z)
{
    const size_t M = S.xc.size();
    for (int64_t s = 0; s < n; ++s) {
        if (!std::isfinite(x[s]) || !std::isfinite(z[s]) || (y && !std::isfinite(y[s])))
            throw Error{SIMUS_EDOMAIN, "scatterer coordinates must be finite"};
        if (!P.convex() && !(z[s] > 0))
            throw Error{SIMUS_EDOMAIN, "scatterer at depth z <= 0 in front of a linear array"};
        const double yy = y ? double(y[s]) : 0.0;
        for (size_t m = 0; m < M; ++m) {
            const double dx = double(x[s]) - S.xc[m], dz = double(z[s]) - S.zc[m];
            if (dx * dx + dz * dz + yy * yy < 1e-18)
                throw Error{SIMUS_EDOMAIN, "scatterer within 1e-9 m of a sub-element centroid"};
        }
    }
}

void check_transmits(const Probe& P, int n_tx, const double* delays, const float* apod)
{
    require(n_tx >= 1 && n_tx <= 4096, "n_tx must be in [1, 4096]");
    require(delays != nullptr, "delays must be non-NULL");
    for (int64_t i = 0; i < int64_t(n_tx) * P.N; ++i) {
        require(std::isfinite(delays[i]) && delays[i] >= 0, "delays must be finite and >= 0");
        if (apod) require(std::isfinite(apod[i]), "apodisation must be finite");
    }
}

}  // namespace simus
