// Host-side planning for libsimus: validation, sub-element geometry,
// frequency grid and per-bin spectral weights.  Pure C++ (no HIP), so it
// also serves the host-only entry points (simus_rf_grid, simus_pfield_nf).
#pragma once

#include <complex>
#include <cstdint>
#include <string>
#include <vector>

#include "simus.h"

namespace simus {

// Error carrying a simus status code; never crosses the C ABI.
struct Error {
    int code;
    std::string msg;
};

struct Probe {
    int N = 0, nu = 0, M = 0;        // elements, sub-elements per element, nu*N
    int baffle = 0;
    double fc = 0, pitch = 0, width = 0, height = 0, elev_focus = 0, bandwidth = 0;
    double radius = 0, zeta = 0;
    double c = 0, alpha_db = 0;
    double fs = 0, n_cycles = 1, eps = 0;
    bool dim2 = false;               // 2-D acoustics (Section V)
    // Gaussians of the elevation aperture (Eq. 12): A_g, B_g; Eq. (18)'s
    // four unless the caller gives a set
    std::vector<std::complex<double>> gA, gB;
    bool convex() const { return radius > 0; }
};

// Sub-element centroids (FP64) and face frames, index n = e*nu + i.
struct SubElements {
    std::vector<double> xc, zc;      // centroid
    std::vector<double> tx, tz;      // unit tangent of the face (azimuth direction)
    std::vector<double> nx, nz;      // unit normal of the face (into the medium)
};

struct Band {
    int nfft = 0, n_t = 0, j_lo = 1, n_bins = 0;
    double df = 0;
};

// Validates probe/medium/options and resolves nu.  Throws Error.
Probe make_probe(const simus_probe* p, const simus_medium* m, const simus_options* o);

// nu from Eq. (21): ceil(width / lambda_min), lambda_min = c / (fc (1 + bw/2)).
int nu_from_width(double width, double fc, double bandwidth, double c);

SubElements sub_elements(const Probe& P);

// Evaluated band for a given nfft (see simus.h).
Band make_band(const Probe& P, int nfft, int n_t);

// Pulse spectrum S_P (Eq. 25) and transducer spectrum S_T (Eq. 27).
std::complex<double> pulse_spectrum(const Probe& P, double w);
double transducer_spectrum(const Probe& P, double w);

// Smallest even 2^a 3^b 5^c >= n.
int64_t next_fft_size(int64_t n);

// Checks the scatterer domain on host copies; throws Error(EDOMAIN).
void check_domain(const Probe& P, const SubElements& S, int64_t n, const float* x,
                  const float* y, const float* z);

// Largest sub-element-to-point distance.
double max_distance(const SubElements& S, int64_t n, const float* x, const float* y,
                    const float* z);

void check_transmits(const Probe& P, int n_tx, const double* delays, const float* apod);

}  // namespace simus
