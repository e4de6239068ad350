// Device-side evaluation of the sub-element Green's term of SIMUS
// (Eqs. 10, 14-20, 39, 40 of Garcia, SIMUS Part I):
//
//   G(f_j) = exp(i k r) exp(-k_a r) / r * D(theta, k) * delta(y, r, k)
//
// Frequency-independent geometry is computed once per (sub-element,
// scatterer) pair (struct Geo); each bin then costs a handful of
// transcendentals.  The phase k r is carried as an unsigned 32-bit fixed
// point fraction of a turn: its start is reduced in FP64 from r * j df / c,
// and each next bin adds the FP64-rounded per-bin increment, so the only
// phase error is the rounding of the increment times the bins walked.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

#include "kernels.hpp"

namespace simus {

// sin(2 pi x), cos(2 pi x) with x in turns (hardware v_sin/v_cos, |x| <= 256).
__device__ __forceinline__ float sin_turns(float x) { return __builtin_amdgcn_sinf(x); }
__device__ __forceinline__ float cos_turns(float x) { return __builtin_amdgcn_cosf(x); }
__device__ __forceinline__ float exp2_fast(float x) { return __builtin_amdgcn_exp2f(x); }
__device__ __forceinline__ float rsq_fast(float x) { return __builtin_amdgcn_rsqf(x); }
__device__ __forceinline__ float rcp_fast(float x) { return __builtin_amdgcn_rcpf(x); }

// Fraction of a turn (x >= 0 or < 0) as a 2^-32 fixed point word.
__device__ __forceinline__ uint32_t turns_fixed(double x)
{
    const double fr = x - floor(x);                       // [0, 1)
    return (uint32_t)(unsigned long long)rint(fr * 4294967296.0);
}

// Fixed-point phase -> turns in [-0.5, 0.5).
__device__ __forceinline__ float fixed_turns(uint32_t p)
{
    return (float)(int32_t)p * 2.3283064365386963e-10f;
}

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

// Frequency-independent part of one (sub-element, scatterer) pair.
struct Geo {
    uint32_t ph;   // phase of exp(i k r) at the current bin, 2^-32 turns
    uint32_t dph;  // phase increment per bin
    float amp;     // obliquity / r, 0 behind the face
    float att;     // log2 attenuation per bin index
    float sig;     // sinc argument (turns) per bin index
    float kap;     // Im(alpha) shift per bin index
    float yr2;     // y^2 / r^2       (y != 0 path)
    float y2r;     // y^2 / (2 r)     (y != 0 path)
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

// Local geometry: distance r (FP64), azimuthal angle theta of the point
// seen from the sub-element face (Eq. 23), obliquity factor of Eq. (39).
template <bool HASY>
__device__ __forceinline__ Geo make_geo(const ModelConst& K, const SubFrame& f, float px, float py,
                                        float pz, int j_first)
{
    const double dx = (double)px - f.xc;
    const double dz = (double)pz - f.zc;
    const double yy = HASY ? (double)py : 0.0;
    const double r = sqrt(dx * dx + dz * dz + yy * yy);
    const float dxf = (float)dx, dzf = (float)dz;
    const float xl = dxf * f.tx + dzf * f.tz;
    const float zl = dxf * f.nx + dzf * f.nz;
    const bool ok = (zl > 0.f) && (r > 1e-9);
    const float rf = ok ? (float)r : 1.f;
    const float rho = HASY ? sqrtf(xl * xl + zl * zl) : rf;
    const float inv_rho = ok ? 1.f / rho : 0.f;
    const float st = xl * inv_rho;
    const float ct = ok ? zl * inv_rho : 1.f;
    float obl = ct;                                        // soft baffle
    if (K.baffle == 1) obl = 1.f;                          // rigid
    else if (K.baffle == 2) obl = ct / (ct + K.zeta);      // finite impedance
    Geo g;
    const float inv_r = 1.f / rf;
    g.amp = ok ? obl * inv_r : 0.f;
    const double tpb = r * K.turns_per_bin_m;
    g.ph = turns_fixed(tpb * (double)j_first);
    g.dph = turns_fixed(tpb);
    g.att = K.att_per_bin_m * rf;
    g.sig = K.sinc_per_bin * st;
    g.kap = K.q_per_bin * (K.inv_rf - inv_r);
    if (HASY) {
        const float yf = py;
        g.yr2 = yf * yf * inv_r * inv_r;
        g.y2r = 0.5f * yf * yf * inv_r;
    } else {
        g.yr2 = 0.f;
        g.y2r = 0.f;
    }
    return g;
}

// Elevation term delta (Eqs. 14-16) for the four Gaussians of Eq. (18),
// alpha_g = a_g + i (b_g + q).  alpha^{-1/2} is formed without trig:
// sqrt(alpha) = s + i b/(2 s), s = sqrt((|alpha| + a)/2), and
// alpha^{-1/2} = conj(sqrt(alpha)) / |alpha|.  For y != 0 each term is
// multiplied by exp(beta^2 / (4 alpha) + gamma), beta^2 = -k^2 y^2 / r^2,
// gamma = i k y^2 / (2 r).
template <bool HASY>
__device__ __forceinline__ float2 elevation(const Gauss4& G, float q, float k, float yr2, float y2r)
{
    float dr = 0.f, di = 0.f;
#pragma unroll
    for (int g = 0; g < 4; ++g) {
        const float bi = G.b[g] + q;
        const float m2 = fmaf(bi, bi, G.a2[g]);
        const float inv_mod = rsq_fast(m2);
        const float mod = m2 * inv_mod;
        const float x = 0.5f * (mod + G.a[g]);
        const float rx = rsq_fast(x);
        float zr = x * rx * inv_mod;              // Re alpha^{-1/2}
        float zi = -0.5f * bi * rx * inv_mod;     // Im alpha^{-1/2}
        if (HASY) {
            // 1/alpha = (alpha^{-1/2})^2
            const float ar = zr * zr - zi * zi, ai = 2.f * zr * zi;
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
        dr = fmaf(G.Ar[g], zr, dr);
        dr = fmaf(-G.Ai[g], zi, dr);
        di = fmaf(G.Ar[g], zi, di);
        di = fmaf(G.Ai[g], zr, di);
    }
    return make_float2(dr, di);
}

// Green's term at absolute bin j (jf = j as float); advances the phase.
template <bool HASY>
__device__ __forceinline__ float2 green_step(const ModelConst& K, Geo& g, float jf)
{
    const float pt = fixed_turns(g.ph);
    g.ph += g.dph;
    const float cs = cos_turns(pt), sn = sin_turns(pt);
    const float ea = exp2_fast(jf * g.att);
    const float v = jf * g.sig;
    const float snc = (v == 0.f) ? 1.f : sin_turns(v) * rcp_fast(6.283185307179586f * v);
    const float a = g.amp * ea * snc;
    const float q = jf * g.kap;
    const float2 d = elevation<HASY>(K.g, q, jf * K.k_per_bin, g.yr2, g.y2r);
    const float pr = a * cs, pi = a * sn;
    return make_float2(pr * d.x - pi * d.y, pr * d.y + pi * d.x);
}

}  // namespace simus
