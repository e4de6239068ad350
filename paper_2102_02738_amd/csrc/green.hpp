// Device-side evaluation of the sub-element Green's term of SIMUS
// (Eqs. 10, 14-20, 39, 40 of Garcia, SIMUS Part I):
//
//   G(f_j) = exp(i k r) exp(-k_a r) / r * D(theta, k) * delta(y, r, k)
//
// A (sub-element, scatterer) pair is set up once per tile of consecutive
// bins (struct Geo), and each next bin is then reached by recurrences:
//   - E_j = (obliquity / r) exp((i k_j - k_a,j) r) is a rotor: E_{j+1} = E_j dE.
//     Its start and step phases are reduced in FP64 from r j df / c, so the
//     only error is the FP32 rounding of the rotor over the tile's bins.
//   - s_j = sin(j theta) / theta (sinc(j theta) = s_j / j, theta = 2 pi df
//     b_sub sin(t) / c) follows the second-order recurrence
//     d_{j+1} = d_j + lambda s_j, s_{j+1} = s_j + d_{j+1}, lambda = -(theta
//     sinc(theta/2))^2, which stays accurate for small theta.
//   - delta(0, r, k) depends on r and k only through q = (k/2)(1/R_f - 1/r);
//     for y = 0 it is read from a cubic table in w = q / (|q| + L) built for
//     the call's range of q (DeltaTable); otherwise it is evaluated directly.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

#include "kernels.hpp"

namespace simus {

// bf16 pairs packed in a 32-bit word, round to nearest even: (a | b << 16)
__device__ __forceinline__ uint32_t pack_bf16(float a, float b)
{
    typedef __bf16 bf16x2_t __attribute__((ext_vector_type(2)));
    typedef float f32x2_t __attribute__((ext_vector_type(2)));
    const f32x2_t v = {a, b};
    return __builtin_bit_cast(uint32_t, __builtin_convertvector(v, bf16x2_t));
}
// the float values of a packed pair's low and high halves
__device__ __forceinline__ float bf16_lo(uint32_t p) { return __uint_as_float(p << 16); }
__device__ __forceinline__ float bf16_hi(uint32_t p) { return __uint_as_float(p & 0xffff0000u); }

// Matrix-core operands: 4 FP32 accumulators; 8 bf16 values as 4 packed words.
typedef float floatx4 __attribute__((ext_vector_type(4)));
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));

__device__ __forceinline__ floatx4 mfma_bf(u32x4 a, u32x4 b, floatx4 c)
{
    return __builtin_amdgcn_mfma_f32_16x16x32_bf16(__builtin_bit_cast(bf16x8, a), __builtin_bit_cast(bf16x8, b), c,
                                                   0, 0, 0);
}
// (re, im) -> (re, -im) and (im, re) of a packed pair
__device__ __forceinline__ uint32_t bf_conj(uint32_t p) { return p ^ 0x80000000u; }
__device__ __forceinline__ uint32_t bf_swap(uint32_t p) { return (p >> 16) | (p << 16); }

// sin(2 pi x), cos(2 pi x) with x in turns (hardware v_sin/v_cos, |x| <= 256).
__device__ __forceinline__ float sin_turns(float x) { return __builtin_amdgcn_sinf(x); }
__device__ __forceinline__ float cos_turns(float x) { return __builtin_amdgcn_cosf(x); }
__device__ __forceinline__ float exp2_fast(float x) { return __builtin_amdgcn_exp2f(x); }
__device__ __forceinline__ float rsq_fast(float x) { return __builtin_amdgcn_rsqf(x); }
__device__ __forceinline__ float rcp_fast(float x) { return __builtin_amdgcn_rcpf(x); }

// Issue priority of a wave by its progress through the synthesis between two
// barriers (step k of n, uniform): of the two waves on a SIMD, the one that
// is behind issues first, so that they reach the barrier together instead of
// one finishing alone with no other wave to hide its latencies.  In the
// split-bf16 synthesis kernels, with their GEMM phase ordered the same way
// (transmit GEMM before receive GEMM): a quarter of the uneven 16-phantom
// batch 202.8 -> 190.0 ms, 21 plane waves 88.8 -> 84.1 ms, 5 plane waves
// 30.7 -> 28.8 ms; FP32 products 312.3 -> 306.9 ms; the four-bin adjoint
// 69.6 -> 68.7 ms; results bit-identical.
__device__ __forceinline__ void prio_by_progress(int k, int n)
{
    const int p = 3 - 4 * k / n;
    if (p >= 3) __builtin_amdgcn_s_setprio(3);
    else if (p == 2) __builtin_amdgcn_s_setprio(2);
    else if (p == 1) __builtin_amdgcn_s_setprio(1);
    else __builtin_amdgcn_s_setprio(0);
}

// Fraction of a turn as a float in [0, 1), reduced in FP64.
__device__ __forceinline__ float frac_turns(double x) { return (float)(x - floor(x)); }

__device__ __forceinline__ float2 cmul(float2 a, float2 b)
{
    return make_float2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}

__device__ __forceinline__ float2 cfma(float2 a, float2 b, float2 c)
{
    c.x = fmaf(a.x, b.x, c.x);
    c.x = fmaf(-a.y, b.y, c.x);
    c.y = fmaf(a.x, b.y, c.y);
    c.y = fmaf(a.y, b.x, c.y);
    return c;
}

// sin(x)/x by its Taylor series to x^12, for |x| < 1 (remainder below 2e-10).
__device__ __forceinline__ float sinc_taylor(float x)
{
    const float x2 = x * x;
    float p = fmaf(x2, 1.6059043836821613e-10f, -2.5052108385441720e-08f);
    p = fmaf(x2, p, 2.7557319223985893e-06f);
    p = fmaf(x2, p, -1.9841269841269841e-04f);
    p = fmaf(x2, p, 8.3333333333333333e-03f);
    p = fmaf(x2, p, -1.6666666666666667e-01f);
    return fmaf(x2, p, 1.0f);
}

// sin(x)/x for the set-up: the Taylor series for |x| < 1, hardware sine above.
__device__ __forceinline__ float sinc_setup(float x)
{
    if (fabsf(x) < 1.f) return sinc_taylor(x);
    return sin_turns(x * 0.15915494309189535f) * rcp_fast(x);
}

// State of one (sub-element, scatterer) pair at the current bin.
struct Geo {
    float2 E;     // (obliquity / r) exp((i k - k_a) r)
    float2 dE;    // per-bin factor of E
    float s;      // sin(j theta) / theta
    float d;      // s_j - s_{j-1}
    float lam;    // -(theta sinc(theta/2))^2
    float kap;    // q per bin index: q_j = j kap
    float yr2;    // y^2 / r^2        (y != 0 path)
    float y2r;    // y^2 / (2 r)      (y != 0 path)
};

struct SubFrame {
    double xc, zc;
    float tx, tz, nx, nz;
};

__device__ __forceinline__ SubFrame load_frame(const SubGeo& g, int n)
{
    SubFrame f;
    f.xc = g.xc[n];
    f.zc = g.zc[n];
    f.tx = g.tx[n];
    f.tz = g.tz[n];
    f.nx = g.nx[n];
    f.nz = g.nz[n];
    return f;
}

// Frequency-independent derivative data of a pair for the adjoint, per
// scatterer coordinate xi in (X, Y, Z) (index 0, 1, 2):
//   la = d ln(obliquity / r) / d xi,  rd = dr / d xi,
//   ud = b_sub d sin(theta) / d xi  (du = k ud, u = k b_sub sin(theta)),
//   qd = (dr / d xi) / (2 r^2)     (dq = k qd for y = 0).
// c, dc carry cos(j theta) by the same recurrence as s (for sinc'(u)).
struct GeoD {
    float la[3], rd[3], ud[3];
    float hq;     // 1 / (2 r^2): dq/dr per unit wavenumber
    float c, dc;
    float inv_theta;
    float r, y;
};

// A (sub-element, scatterer) pair in the sub-element's frame: squared
// distance in FP64, the point's coordinates along the face (xl) and along
// its normal (zl), and whether the pair lies in the model's domain: in front
// of the face (zl > 0) and farther than 1e-9 m from the centroid.  Outside
// it the pair's Green's term is 0 (a flat piston does not radiate behind its
// face; Eq. 22's 1/r is undefined at r = 0).  The table of the elevation
// term covers the distances of in-domain pairs only (k_rrange), so both use
// this one test.
struct PairFrame {
    double r2;
    float xl, zl;
    bool ok;
};

template <bool HASY>
__device__ __forceinline__ PairFrame pair_frame(const SubFrame& f, float px, float py, float pz)
{
    const double dx = (double)px - f.xc;
    const double dz = (double)pz - f.zc;
    const double yy = HASY ? (double)py : 0.0;
    PairFrame p;
    p.r2 = fma(dx, dx, fma(dz, dz, yy * yy));
    const float dxf = (float)dx, dzf = (float)dz;
    p.xl = dxf * f.tx + dzf * f.tz;
    p.zl = dxf * f.nx + dzf * f.nz;
    p.ok = (p.zl > 0.f) && (p.r2 > 1e-18);
    return p;
}

// Set-up of a pair at bin j0: distance r in FP64, azimuthal angle theta of
// the point seen from the sub-element face (Eq. 23), obliquity of Eq. (39).
// With D != nullptr also the derivative data of the pair.
template <bool HASY, bool SMALL_SINC = false>
__device__ __forceinline__ Geo make_geo(const ModelConst& K, const SubFrame& f, float px, float py,
                                        float pz, int j0, GeoD* D = nullptr)
{
    const PairFrame pf = pair_frame<HASY>(f, px, py, pz);
    // r in FP64 without a double-precision root: the FP32 root of the FP64
    // square, refined by one Newton step in FP64 (relative error ~1e-14)
    const double r2 = pf.r2;
    const float xl = pf.xl, zl = pf.zl;
    const bool ok = pf.ok;
    const double r2s = ok ? r2 : 1.0;
    const float r2f = (float)r2s;
    const float inv_r0 = rsq_fast(r2f);
    const double r0 = (double)(r2f * inv_r0);
    const double r = fma(fma(-r0, r0, r2s), 0.5 * (double)inv_r0, r0);
    const float rf = (float)r;
    // 1/r: the FP32 reciprocal root above (about 1 ulp, as a division);
    // 1/rho, the in-plane distance, the same without y
    const float inv_r = inv_r0;
    const float inv_rho = ok ? (HASY ? rsq_fast(xl * xl + zl * zl) : inv_r) : 0.f;
    const float st = xl * inv_rho;
    const float ct = ok ? zl * inv_rho : 1.f;
    float obl = ct, dobl = 1.f;                            // soft baffle
    if (K.baffle == 1) {                                   // rigid
        obl = 1.f;
        dobl = 0.f;
    } else if (K.baffle == 2) {                            // finite impedance
        const float den = rcp_fast(ct + K.zeta);
        obl = ct * den;
        dobl = K.zeta * den * den;
    }
    // amplitude 1/r, or 1/sqrt(r) in 2-D (Eqs. 36-38)
    const float amp = ok ? obl * (K.dim2 ? rsq_fast(rf) : inv_r) : 0.f;
    const float apow = K.dim2 ? 0.5f : 1.f;
    const float jf0 = (float)j0;

    Geo g;
    // rotor: phase (turns) r j df / c reduced in FP64; attenuation exp2(j a1)
    const double tpb = r * K.turns_per_bin_m;
    const float t0 = frac_turns(tpb * (double)j0);
    const float dt = frac_turns(tpb);
    const float a1 = K.att_per_bin_m * rf;
    const float m0 = amp * exp2_fast(jf0 * a1);
    const float m1 = exp2_fast(a1);
    g.E = make_float2(m0 * cos_turns(t0), m0 * sin_turns(t0));
    g.dE = make_float2(m1 * cos_turns(dt), m1 * sin_turns(dt));
    // sinc recurrence, theta = 2 pi sigma, sigma = df b_sub sin(t) / c (turns per bin)
    const float sigma = K.sinc_per_bin * st;
    const float theta = 6.283185307179586f * sigma;
    // sinc(theta / 2): |theta / 2| <= pi sinc_per_bin, below 1 for any
    // practical probe and grid (a uniform branch; SMALL_SINC: known below)
    const float sh = (SMALL_SINC || K.sinc_per_bin < SINC_TAYLOR_LIMIT) ? sinc_taylor(0.5f * theta)
                                                                        : sinc_setup(0.5f * theta);
    g.s = jf0 * sinc_setup(jf0 * theta);
    g.d = cos_turns((jf0 - 0.5f) * sigma) * sh;
    g.lam = -(theta * sh) * (theta * sh);
    g.kap = K.q_per_bin * (K.inv_rf - inv_r);
    if (HASY) {
        const float yf = py;
        g.yr2 = yf * yf * inv_r * inv_r;
        g.y2r = 0.5f * yf * yf * inv_r;
    } else {
        g.yr2 = 0.f;
        g.y2r = 0.f;
    }
    if (D) {
        const float yf = HASY ? py : 0.f;
        const float dxl[3] = {f.tx, 0.f, f.tz};
        const float dzl[3] = {f.nx, 0.f, f.nz};
        const float dyy[3] = {0.f, 1.f, 0.f};
        const float inv_obl = ok ? rcp_fast(obl) : 0.f;
#pragma unroll
        for (int a = 0; a < 3; ++a) {
            const float drho = (xl * dxl[a] + zl * dzl[a]) * inv_rho;
            const float dr = (xl * dxl[a] + zl * dzl[a] + yf * dyy[a]) * inv_r;
            const float dst = (dxl[a] - st * drho) * inv_rho;
            const float dct = (dzl[a] - ct * drho) * inv_rho;
            D->la[a] = ok ? dobl * dct * inv_obl - apow * dr * inv_r : 0.f;
            D->rd[a] = ok ? dr : 0.f;
            D->ud[a] = ok ? K.b_sub * dst : 0.f;
        }
        D->hq = 0.5f * inv_r * inv_r;
        D->c = cos_turns(jf0 * sigma);
        D->dc = -theta * sin_turns((jf0 - 0.5f) * sigma) * sh;
        D->inv_theta = (theta != 0.f) ? rcp_fast(theta) : 0.f;
        D->r = rf;
        D->y = yf;
    }
    return g;
}

// Elevation term delta (Eqs. 14-16), one Gaussian of Eq. (12) at a time:
// alpha_g = a_g + i (b_g + q), evaluated directly.  alpha^{-1/2} is formed
// without trig: sqrt(alpha) = s + i b/(2 s), s = sqrt((|alpha| + a)/2),
// alpha^{-1/2} = conj(sqrt(alpha)) / |alpha|.  For y != 0 each term is
// multiplied by exp(beta^2 / (4 alpha) + gamma), beta^2 = -k^2 y^2 / r^2,
// gamma = i k y^2 / (2 r).  Accumulates A_g sqrt(pi) alpha^{-1/2} e^(...)
// into (dr, di).
template <bool HASY>
__device__ __forceinline__ void elevation_term(float a, float a2, float b, float Ar, float Ai, float q,
                                               float k, float yr2, float y2r, float& dr, float& di)
{
    const float bi = b + q;
    const float m2 = fmaf(bi, bi, a2);
    const float inv_mod = rsq_fast(m2);
    const float mod = m2 * inv_mod;
    const float x = 0.5f * (mod + a);
    const float rx = rsq_fast(x);
    float zr = x * rx * inv_mod;              // Re alpha^{-1/2}
    float zi = -0.5f * bi * rx * inv_mod;     // Im alpha^{-1/2}
    if (HASY) {
        const float ar = zr * zr - zi * zi, ai = 2.f * zr * zi;   // 1/alpha
        const float c0 = -0.25f * k * k * yr2;
        const float er = c0 * ar;
        const float ei = c0 * ai + k * y2r;   // radians
        float et = ei * 0.15915494309189535f;
        et -= rintf(et);
        const float mag = exp2_fast(er * 1.4426950408889634f);
        const float c = mag * cos_turns(et), s = mag * sin_turns(et);
        const float nr = zr * c - zi * s, ni = zr * s + zi * c;
        zr = nr;
        zi = ni;
    }
    dr = fmaf(Ar, zr, dr);
    dr = fmaf(-Ai, zi, dr);
    di = fmaf(Ar, zi, di);
    di = fmaf(Ai, zr, di);
}

// delta summed over the set: four Gaussians unrolled from the constants,
// any other count from the device table.
template <bool HASY>
__device__ __forceinline__ float2 elevation(const ModelConst& K, float q, float k, float yr2, float y2r)
{
    float dr = 0.f, di = 0.f;
    if (K.ng == 4) {
#pragma unroll
        for (int g = 0; g < 4; ++g)
            elevation_term<HASY>(K.g.a[g], K.g.a2[g], K.g.b[g], K.g.Ar[g], K.g.Ai[g], q, k, yr2, y2r, dr, di);
    } else {
        for (int g = 0; g < K.ng; ++g) {
            const float4 c = K.gset[g];
            elevation_term<HASY>(c.x, c.x * c.x, c.y, c.z, c.w, q, k, yr2, y2r, dr, di);
        }
    }
    return make_float2(dr, di);
}

// Cubic table of delta(0, r, k) as a function of w = q / (|q| + L):
// interval k of DELTA_NT holds (c0, c1, c2, c3) complex, delta = c0 + t (c1
// + t (c2 + t c3)), t in [0, 1).  Stored as two float4 per interval, in two
// arrays (dtab_a, dtab_b).  Argument qs = q inv_dw / L (see delta_fetch).
__device__ __forceinline__ float2 delta_table(const float4* tab, const DeltaParams& P, float qs)
{
    const float r = rcp_fast(fmaf(fabsf(qs), P.dw, 1.f));
    const float u = __builtin_amdgcn_fmed3f(fmaf(qs, r, P.u0), 0.f, P.umax);
    // u >= 0 after the clamp: the conversion truncates to the interval and
    // the hardware fraction gives the local coordinate
    const int k = (int)u;
    const float t = __builtin_amdgcn_fractf(u);
    const float4 a = tab[dtab_a(k)], b = tab[dtab_b(k)];
    float re = fmaf(t, b.z, b.x), im = fmaf(t, b.w, b.y);
    re = fmaf(t, re, a.z);
    im = fmaf(t, im, a.w);
    re = fmaf(t, re, a.x);
    im = fmaf(t, im, a.y);
    return make_float2(re, im);
}

// The table lookup in two steps, so that a lookup's LDS read can be in
// flight while earlier terms are evaluated.
struct DeltaFetch {
    float4 a, b;
    float t;
};

// Argument b = q inv_dw / L (a pair's kap pre-scaled by P.kscale): the table
// coordinate u0 + inv_dw q / (|q| + L) is u0 + b / (|b| dw + 1), one
// multiply fewer per term than from q.
__device__ __forceinline__ DeltaFetch delta_fetch(const float4* tab, const DeltaParams& P, float b)
{
    const float r = rcp_fast(fmaf(fabsf(b), P.dw, 1.f));
    const float u = __builtin_amdgcn_fmed3f(fmaf(b, r, P.u0), 0.f, P.umax);
    const int k = (int)u;                  // u >= 0: truncation is the floor
    DeltaFetch f;
    f.t = __builtin_amdgcn_fractf(u);
    f.a = tab[dtab_a(k)];
    f.b = tab[dtab_b(k)];
    return f;
}

__device__ __forceinline__ float2 delta_eval(const DeltaFetch& f)
{
    float re = fmaf(f.t, f.b.z, f.b.x), im = fmaf(f.t, f.b.w, f.b.y);
    re = fmaf(f.t, re, f.a.z);
    im = fmaf(f.t, im, f.a.w);
    re = fmaf(f.t, re, f.a.x);
    im = fmaf(f.t, im, f.a.y);
    return make_float2(re, im);
}

// delta with its partial derivatives in r and y, evaluated directly
// (y != 0 path of the adjoint, or without the table), one Gaussian at a
// time.  Per Gaussian, T = A sqrt(pi) alpha^{-1/2} exp(phi), phi =
// beta^2/(4 alpha) + gamma, and dT = T (-1/2 dalpha / alpha + dphi).
template <bool HASY>
__device__ __forceinline__ void elevation_grad_term(float a, float a2, float b, float Ar, float Ai,
                                                    float q, float ar_i, float k, float y, float inv_r,
                                                    float2& dl, float2& d_r, float2& d_y)
{
    const float bi = b + q;
    const float m2 = fmaf(bi, bi, a2);
    const float inv_mod = rsq_fast(m2);
    const float mod = m2 * inv_mod;
    const float x = 0.5f * (mod + a);
    const float rx = rsq_fast(x);
    const float zr = x * rx * inv_mod, zi = -0.5f * bi * rx * inv_mod;   // alpha^{-1/2}
    const float2 ia = make_float2(zr * zr - zi * zi, 2.f * zr * zi);     // 1/alpha
    float2 T = make_float2(Ar * zr - Ai * zi, Ar * zi + Ai * zr);
    // -1/2 (d alpha/dr) / alpha = -1/2 (i ar_i) ia
    float2 lr = make_float2(0.5f * ar_i * ia.y, -0.5f * ar_i * ia.x);
    float2 ly = make_float2(0.f, 0.f);
    if (HASY) {
        const float b2 = -k * k * y * y * inv_r * inv_r;               // beta^2 (real)
        const float gam = 0.5f * k * y * y * inv_r;                    // gamma = i gam
        const float2 phi = make_float2(0.25f * b2 * ia.x, 0.25f * b2 * ia.y + gam);
        // beta = -i k y / r, dbeta/dr = i k y / r^2, dbeta/dy = -i k / r
        // 2 beta dbeta/dr = 2 k^2 y^2 / r^3 (real); 2 beta dbeta/dy = -2 k^2 y / r^2
        const float bbr = 2.f * k * k * y * y * inv_r * inv_r * inv_r;
        const float bby = -2.f * k * k * y * inv_r * inv_r;
        // - beta^2 dalpha/dr / (4 alpha^2) = -(b2 / 4) (i ar_i) ia^2
        const float2 ia2 = cmul(ia, ia);
        const float2 t2 = make_float2(0.25f * b2 * ar_i * ia2.y, -0.25f * b2 * ar_i * ia2.x);
        lr.x += 0.25f * bbr * ia.x + t2.x;
        lr.y += 0.25f * bbr * ia.y + t2.y - 0.5f * k * y * y * inv_r * inv_r;
        ly = make_float2(0.25f * bby * ia.x, 0.25f * bby * ia.y + k * y * inv_r);
        float et = phi.y * 0.15915494309189535f;
        et -= rintf(et);
        const float mag = exp2_fast(phi.x * 1.4426950408889634f);
        T = cmul(T, make_float2(mag * cos_turns(et), mag * sin_turns(et)));
    }
    dl.x += T.x;
    dl.y += T.y;
    const float2 tr = cmul(T, lr), ty = cmul(T, ly);
    d_r.x += tr.x;
    d_r.y += tr.y;
    d_y.x += ty.x;
    d_y.y += ty.y;
}

template <bool HASY>
__device__ __forceinline__ void elevation_grad(const ModelConst& K, float k, float r, float y, float2& dl,
                                               float2& d_r, float2& d_y)
{
    const float inv_r = rcp_fast(r);
    const float q = 0.5f * k * (K.inv_rf - inv_r);
    const float ar_i = 0.5f * k * inv_r * inv_r;          // d alpha / dr = i ar_i
    dl = d_r = d_y = make_float2(0.f, 0.f);
    if (K.ng == 4) {
#pragma unroll
        for (int g = 0; g < 4; ++g)
            elevation_grad_term<HASY>(K.g.a[g], K.g.a2[g], K.g.b[g], K.g.Ar[g], K.g.Ai[g], q, ar_i, k, y,
                                      inv_r, dl, d_r, d_y);
    } else {
        for (int g = 0; g < K.ng; ++g) {
            const float4 c = K.gset[g];
            elevation_grad_term<HASY>(c.x, c.x * c.x, c.y, c.z, c.w, q, ar_i, k, y, inv_r, dl, d_r, d_y);
        }
    }
}

// Table lookup returning delta and d delta / dq.
__device__ __forceinline__ float2 delta_table_d(const float4* tab, const DeltaParams& P, float q,
                                                float2& dq)
{
    const float den = rcp_fast(fabsf(q) + P.L);
    const float w = q * den;
    const float u = __builtin_amdgcn_fmed3f(fmaf(w, P.inv_dw, P.u0), 0.f, P.umax);
    // u >= 0 after the clamp: the conversion truncates to the interval and
    // the hardware fraction gives the local coordinate
    const int k = (int)u;
    const float t = __builtin_amdgcn_fractf(u);
    const float4 a = tab[dtab_a(k)], b = tab[dtab_b(k)];
    float re = fmaf(t, b.z, b.x), im = fmaf(t, b.w, b.y);
    // derivative in t: c1 + t (2 c2 + 3 t c3)
    float gr = fmaf(3.f * t, b.z, 2.f * b.x), gi = fmaf(3.f * t, b.w, 2.f * b.y);
    gr = fmaf(t, gr, a.z);
    gi = fmaf(t, gi, a.w);
    re = fmaf(t, re, a.z);
    im = fmaf(t, im, a.w);
    re = fmaf(t, re, a.x);
    im = fmaf(t, im, a.y);
    const float dwdq = P.L * den * den * P.inv_dw;         // dt/dq
    dq = make_float2(gr * dwdq, gi * dwdq);
    return make_float2(re, im);
}

// Green's term and its gradient in the scatterer coordinates at bin j;
// advances the pair (and its cosine recurrence) to bin j + 1.
template <bool HASY, bool TABLE, int NX>
__device__ __forceinline__ float2 green_grad_next(const ModelConst& K, Geo& g, GeoD& D, float jf,
                                                  float inv_j, const float4* tab,
                                                  const DeltaParams& P, float2 (&dG)[NX])
{
    const float sn = g.s * inv_j;                          // sinc(u)
    const float k = jf * K.k_per_bin;
    const float ka = jf * K.ka_per_bin;
    const float2 A = make_float2(g.E.x * sn, g.E.y * sn);
    float2 dl, d_dq, d_r, d_y;
    if (TABLE) {
        dl = delta_table_d(tab, P, jf * g.kap, d_dq);
    } else {
        elevation_grad<HASY>(K, k, D.r, D.y, dl, d_r, d_y);
    }
    const float2 Gv = cmul(A, dl);
    const float2 Ed = cmul(g.E, dl);
    const float dsn = (D.c - sn) * inv_j * D.inv_theta;    // sinc'(u)
    // d delta / dr, through q = (k/2)(1/R_f - 1/r): dq/dr = k / (2 r^2)
    float2 ddr;
    if (TABLE) {
        const float s = k * D.hq;
        ddr = make_float2(d_dq.x * s, d_dq.y * s);
    } else {
        ddr = d_r;
    }
    // everything in dG/dr but the obliquity: (i k - k_a) G + A d delta/dr;
    // a coordinate's gradient is then G la + Rr dr/dxi + Ed sinc' k du/dxi
    float2 Rr = cmul(A, ddr);
    Rr.x = fmaf(-ka, Gv.x, fmaf(-k, Gv.y, Rr.x));
    Rr.y = fmaf(-ka, Gv.y, fmaf(k, Gv.x, Rr.y));
    const float su = dsn * k;
    const float2 Q = make_float2(Ed.x * su, Ed.y * su);
    constexpr int idx[3] = {0, 2, 1};                      // X, Z, Y
#pragma unroll
    for (int i = 0; i < NX; ++i) {
        const int a = idx[i];
        float2 v = make_float2(Gv.x * D.la[a], Gv.y * D.la[a]);
        v.x = fmaf(Rr.x, D.rd[a], v.x);
        v.y = fmaf(Rr.y, D.rd[a], v.y);
        v.x = fmaf(Q.x, D.ud[a], v.x);
        v.y = fmaf(Q.y, D.ud[a], v.y);
        if (!TABLE && a == 1) v = cfma(A, d_y, v);
        dG[i] = v;
    }
    g.E = cmul(g.E, g.dE);
    g.d = fmaf(g.lam, g.s, g.d);
    g.s += g.d;
    D.dc = fmaf(g.lam, D.c, D.dc);
    D.c += D.dc;
    return Gv;
}

// j G at bin j without an elevation term (2-D acoustics, Eqs. 36-38): the
// sinc's 1/j is left to the caller.  Advances the pair to bin j + 1.
__device__ __forceinline__ float2 green_next_2d(Geo& g)
{
    const float2 G = make_float2(g.E.x * g.s, g.E.y * g.s);
    g.E = cmul(g.E, g.dE);
    g.d = fmaf(g.lam, g.s, g.d);
    g.s += g.d;
    return G;
}

// j G at bin j from a fetched table interval (y = 0): the sinc's 1/j is left
// to the caller.  Advances the pair to bin j + 1.
__device__ __forceinline__ float2 green_next_fetched(Geo& g, const DeltaFetch& f)
{
    const float2 A = make_float2(g.E.x * g.s, g.E.y * g.s);
    const float2 d = delta_eval(f);
    g.E = cmul(g.E, g.dE);
    g.d = fmaf(g.lam, g.s, g.d);
    g.s += g.d;
    return cmul(A, d);
}

// Green's term at absolute bin j (jf = j, inv_j = 1/j); advances the pair to
// bin j + 1.  With TABLE the pair's kap must be pre-scaled by P.kscale.
template <bool HASY, bool TABLE>
__device__ __forceinline__ float2 green_next(const ModelConst& K, Geo& g, float jf, float inv_j,
                                             const float4* tab, const DeltaParams& P)
{
    const float sn = g.s * inv_j;                         // sinc(j theta)
    const float2 A = make_float2(g.E.x * sn, g.E.y * sn);
    const float q = jf * g.kap;
    float2 d;
    if (TABLE) d = delta_table(tab, P, q);
    else d = elevation<HASY>(K, q, jf * K.k_per_bin, g.yr2, g.y2r);
    g.E = cmul(g.E, g.dE);
    g.d = fmaf(g.lam, g.s, g.d);
    g.s += g.d;
    return cmul(A, d);
}

}  // namespace simus
