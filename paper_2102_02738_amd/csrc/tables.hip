// Per-call tables of libsimus: the distance range of a call and the cubic
// table of the elevation term delta(0, r, k) (Eqs. 14-16 with y = 0) over
// the call's range of q = (k/2)(1/R_f - 1/r).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>

#include "green.hpp"
#include "kernels.hpp"

namespace simus {

__global__ void k_rr_init(uint32_t* rr)
{
    rr[0] = 0x7f800000u;   // +inf
    rr[1] = 0u;
}

// Min / max distance over the (sub-element, scatterer) pairs of the model's
// domain (pair_frame: in front of the sub-element's face, farther than
// 1e-9 m), which are the only pairs whose elevation term is read from the
// table; as float bits (positive floats order like their bit patterns).
// The table adds a margin.
__global__ __launch_bounds__(256) void k_rrange(uint32_t* rr, const float* __restrict__ x,
                                                const float* __restrict__ y,
                                                const float* __restrict__ z, int64_t n, SubGeo sub,
                                                int M)
{
    float lo = INFINITY, hi = 0.f;
    for (int64_t s = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; s < n;
         s += (int64_t)gridDim.x * blockDim.x) {
        const float px = x[s], pz = z[s], py = y ? y[s] : 0.f;
        for (int m = 0; m < M; ++m) {
            const PairFrame p = pair_frame<true>(load_frame(sub, m), px, py, pz);
            if (!p.ok) continue;
            const float r2 = (float)p.r2;
            lo = fminf(lo, r2);
            hi = fmaxf(hi, r2);
        }
    }
    for (int off = 32; off > 0; off >>= 1) {
        lo = fminf(lo, __shfl_xor(lo, off));
        hi = fmaxf(hi, __shfl_xor(hi, off));
    }
    if ((threadIdx.x & 63) == 0 && hi > 0.f) {
        atomicMin(&rr[0], __float_as_uint(sqrtf(lo)));
        atomicMax(&rr[1], __float_as_uint(sqrtf(hi)));
    }
}

hipError_t launch_rrange(uint32_t* rr, const float* x, const float* y, const float* z, int64_t n,
                         const SubGeo& sub, int M, hipStream_t st)
{
    hipLaunchKernelGGL(k_rr_init, dim3(1), dim3(1), 0, st, rr);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess || n == 0) return e;
    const int grid = (int)std::min<int64_t>((n + 255) / 256, 2048);
    hipLaunchKernelGGL(k_rrange, dim3(grid), dim3(256), 0, st, rr, x, y, z, n, sub, M);
    return hipGetLastError();
}

// delta(0, r, k) as a function of q and d delta / dq, FP64, over the
// Gaussians of the set (gs: [ng][4] = Re A, Im A, Re B, Im B).
__device__ void delta_q(double q, double h, const double* gs, int ng, double& dr, double& di, double& gr,
                        double& gi)
{
    dr = di = gr = gi = 0.0;
    const double sq_pi = 1.7724538509055160273;
    for (int g = 0; g < ng; ++g) {
        const double a = gs[4 * g + 2] / (h * h);
        const double b = gs[4 * g + 3] / (h * h) + q;
        const double mod = hypot(a, b);
        const double s = sqrt(0.5 * (mod + a));
        // alpha^{-1/2} = (s - i b/(2 s)) / |alpha|
        const double zr = s / mod, zi = -0.5 * b / (s * mod);
        // alpha^{-3/2} = (alpha^{-1/2})^3
        const double z2r = zr * zr - zi * zi, z2i = 2 * zr * zi;
        const double z3r = z2r * zr - z2i * zi, z3i = z2r * zi + z2i * zr;
        const double Ar = sq_pi * gs[4 * g], Ai = sq_pi * gs[4 * g + 1];
        dr += Ar * zr - Ai * zi;
        di += Ar * zi + Ai * zr;
        // d/dq alpha^{-1/2} = -1/2 alpha^{-3/2} i  ->  (0.5 z3i, -0.5 z3r)
        const double wr = 0.5 * z3i, wi = -0.5 * z3r;
        gr += Ar * wr - Ai * wi;
        gi += Ar * wi + Ai * wr;
    }
}

// One thread per interval: Hermite data at both knots in FP64, converted to
// the power basis of the local coordinate t in [0, 1).
__global__ __launch_bounds__(DELTA_NT) void k_dtable(float4* tab, DeltaParams* par,
                                                     const uint32_t* rr, const double* gs, int ng,
                                                     double q_per_bin, double inv_rf, double height,
                                                     int j_first, int j_last, int unit)
{
    double rmin = (double)__uint_as_float(rr[0]), rmax = (double)__uint_as_float(rr[1]);
    if (!(rmin <= rmax) || !(rmin > 0.0)) {   // no scatterers
        rmin = 1e-3;
        rmax = 1.0;
    }
    rmin *= 1.0 - 1e-4;
    rmax *= 1.0 + 1e-4;
    const double v_lo = inv_rf - 1.0 / rmin, v_hi = inv_rf - 1.0 / rmax;
    const double qa = q_per_bin * j_first, qb = q_per_bin * j_last;
    double q_lo = fmin(fmin(qa * v_lo, qb * v_lo), fmin(qa * v_hi, qb * v_hi));
    double q_hi = fmax(fmax(qa * v_lo, qb * v_lo), fmax(qa * v_hi, qb * v_hi));
    const double span = q_hi - q_lo;
    q_lo -= 1e-3 * span + 1.0;
    q_hi += 1e-3 * span + 1.0;
    const double L = 13.0 / (height * height);   // ~ |B_1| / (2 h^2)
    const double w_lo = q_lo / (fabs(q_lo) + L), w_hi = q_hi / (fabs(q_hi) + L);
    const double dw = (w_hi - w_lo) / DELTA_NT;
    const int k = threadIdx.x;
    double p[2][2], m[2][2];
    for (int e = 0; e < 2; ++e) {
        const double w = w_lo + (k + e) * dw;
        const double q = L * w / (1.0 - fabs(w));
        const double dqdw = L / ((1.0 - fabs(w)) * (1.0 - fabs(w)));
        double dr, di, gr, gi;
        delta_q(q, height, gs, ng, dr, di, gr, gi);
        p[e][0] = dr;
        p[e][1] = di;
        m[e][0] = gr * dqdw * dw;
        m[e][1] = gi * dqdw * dw;
    }
    float c[4][2];
    for (int i = 0; i < 2; ++i) {
        c[0][i] = (float)p[0][i];
        c[1][i] = (float)m[0][i];
        c[2][i] = (float)(3.0 * (p[1][i] - p[0][i]) - 2.0 * m[0][i] - m[1][i]);
        c[3][i] = (float)(2.0 * (p[0][i] - p[1][i]) + m[0][i] + m[1][i]);
        if (unit) c[0][i] = c[1][i] = c[2][i] = c[3][i] = 0.f;
    }
    if (unit) c[0][0] = 1.f;
    tab[dtab_a(k)] = make_float4(c[0][0], c[0][1], c[1][0], c[1][1]);
    tab[dtab_b(k)] = make_float4(c[2][0], c[2][1], c[3][0], c[3][1]);
    if (k == 0) {
        DeltaParams P;
        P.L = (float)L;
        P.u0 = (float)(-w_lo / dw);
        P.inv_dw = (float)(1.0 / dw);
        P.umax = (float)DELTA_NT - 1.0f / 256.0f;
        P.kscale = (float)(1.0 / (dw * L));
        P.dw = (float)dw;
        *par = P;
    }
}

hipError_t launch_dtable(float4* tab, DeltaParams* par, const uint32_t* rr, const ModelConst& K,
                         const double* gset64, double height, int j_first, int j_last, bool unit,
                         hipStream_t st)
{
    const double q_per_bin = M_PI * K.turns_per_bin_m;   // pi df / c
    hipLaunchKernelGGL(k_dtable, dim3(1), dim3(DELTA_NT), 0, st, tab, par, rr, gset64, K.ng, q_per_bin,
                       (double)K.inv_rf, height, j_first, j_last, unit ? 1 : 0);
    return hipGetLastError();
}

}  // namespace simus
