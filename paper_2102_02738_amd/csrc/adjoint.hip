// Adjoint of the RF synthesis: gradients of a misfit L with respect to the
// scatterer reflectivities and positions, given dL/drf.
//
// With Lam[t][e](w_j) = sum_q dL/drf[t][e][q] e^{-2 pi i j q / nfft} (the
// transpose of the inverse transform of Eq. 1) and, per scatterer s and bin j,
//   a_t  = sum_n W_{t,e(n)} G_{n,s},   b_t  = sum_n Lam_{t,e(n)} G_{n,s},
//   a'_t = sum_n W_{t,e(n)} dG_{n,s},  b'_t = sum_n Lam_{t,e(n)} dG_{n,s},
// the chain rule through Eqs. (29)-(34) gives
//   dL/dR_s  = Re sum_j P_j sum_t a_t b_t,
//   dL/dxi_s = R_s Re sum_j P_j sum_t (a'_t b_t + a_t b'_t),
// P_j = S_P S_T (Eqs. 28, 34).  The Green's terms and their gradients are
// recomputed here (nothing is kept from the forward pass).
//
// One thread owns one scatterer and loops over all sub-elements for a tile of
// JT bins: every sum over n stays in registers, the sub-element frames and the
// weights W, Lam are the same for the whole wave (scalar loads), and there is
// no reduction across lanes.  Blocks cover (phantom, 256 scatterers, bin
// range); a second kernel sums the bin ranges in a fixed order.
#include <hip/hip_runtime.h>

#include <algorithm>

#include "green.hpp"
#include "kernels.hpp"

namespace simus {

template <int JT, int TT, bool HASY, bool TABLE>
__global__ __launch_bounds__(256) void k_adjoint(AdjArgs A)
{
    constexpr int NX = HASY ? 3 : 2;          // coordinates: X, Z (, Y)
    __shared__ float4 s_tab[TABLE ? 2 * DELTA_NT : 1];
    DeltaParams P{};
    if (TABLE) {
        for (int i = threadIdx.x; i < 2 * DELTA_NT; i += 256) s_tab[i] = A.dtab[i];
        P = *A.dpar;
        __syncthreads();
    }
    const AdjItem it = A.items[blockIdx.x];
    const int s = it.s_begin + (int)threadIdx.x;
    const bool live = s < it.s_end;
    const float px = live ? A.x[s] : 0.f;
    const float py = (HASY && live) ? A.y[s] : 0.f;
    const float pz = live ? A.z[s] : 1.f;
    const int b_begin = it.range * A.range_bins;
    const int b_end = min(A.n_bins, b_begin + A.range_bins);
    const int p = it.phantom;

    float gR = 0.f, gX[NX];
#pragma unroll
    for (int i = 0; i < NX; ++i) gX[i] = 0.f;

    for (int tg = 0; tg * TT < A.n_tx; ++tg) {
        const int t0 = tg * TT;
        for (int jb0 = b_begin; jb0 < b_end; jb0 += JT) {
            // accumulators: [jj][t] of a, b and [jj][t][xi] of a', b'
            float2 a[JT][TT], b[JT][TT], da[JT][TT][NX], db[JT][TT][NX];
#pragma unroll
            for (int jj = 0; jj < JT; ++jj)
#pragma unroll
                for (int t = 0; t < TT; ++t) {
                    a[jj][t] = b[jj][t] = make_float2(0.f, 0.f);
#pragma unroll
                    for (int i = 0; i < NX; ++i) da[jj][t][i] = db[jj][t][i] = make_float2(0.f, 0.f);
                }
            // With the table (y = 0), a full tile (JT bins, TT transmits) runs
            // as one straight-line bin loop, with no branch per bin and
            // transmit: the compiler can then issue later bins' table reads
            // and weight loads early (one transmit, 5 plane waves' scatterers:
            // 54.3 -> 52.9 ms).  Without the table it would take 22 more
            // registers and a wave less per SIMD.  The loop below serves the
            // rest.  (A generic lambda: its body is compiled only where the
            // table branch calls it.)
            auto tile_full = [&](auto) {
                for (int n = 0; n < A.M; ++n) {
                    const SubFrame fr = load_frame(A.sub, n);
                    const int e = n / A.nu;
                    GeoD D;
                    Geo g = make_geo<HASY>(A.K, fr, px, py, pz, A.j_lo + jb0, &D);
                    if (!live) g.E = make_float2(0.f, 0.f);
#pragma unroll
                    for (int jj = 0; jj < JT; ++jj) {
                        const int jb = jb0 + jj;
                        const float jf = (float)(A.j_lo + jb);
                        float2 dG[NX];
                        const float2 G = green_grad_next<HASY, TABLE, NX>(A.K, g, D, jf, rcp_fast(jf),
                                                                          s_tab, P, dG);
#pragma unroll
                        for (int t = 0; t < TT; ++t) {
                            const float2 W = A.W[((int64_t)jb * A.n_tx + t0 + t) * A.N + e];
                            const float2 L =
                                A.lam[(((int64_t)p * A.n_bins + jb) * A.n_tx + t0 + t) * A.N + e];
                            a[jj][t] = cfma(W, G, a[jj][t]);
                            b[jj][t] = cfma(L, G, b[jj][t]);
#pragma unroll
                            for (int i = 0; i < NX; ++i) {
                                da[jj][t][i] = cfma(W, dG[i], da[jj][t][i]);
                                db[jj][t][i] = cfma(L, dG[i], db[jj][t][i]);
                            }
                        }
                    }
                }
            };
            const bool full = TABLE && !HASY && jb0 + JT <= b_end && t0 + TT <= A.n_tx;
            if constexpr (TABLE && !HASY) {
                if (full) tile_full(0);
            }
            for (int n = 0; !full && n < A.M; ++n) {
                const SubFrame fr = load_frame(A.sub, n);
                const int e = n / A.nu;
                GeoD D;
                Geo g = make_geo<HASY>(A.K, fr, px, py, pz, A.j_lo + jb0, &D);
                if (!live) g.E = make_float2(0.f, 0.f);
#pragma unroll
                for (int jj = 0; jj < JT; ++jj) {
                    const int jb = jb0 + jj;
                    if (jb < b_end) {
                        const float jf = (float)(A.j_lo + jb);
                        float2 dG[NX];
                        const float2 G = green_grad_next<HASY, TABLE, NX>(A.K, g, D, jf, rcp_fast(jf),
                                                                          s_tab, P, dG);
#pragma unroll
                        for (int t = 0; t < TT; ++t) {
                            if (t0 + t < A.n_tx) {
                                const float2 W = A.W[((int64_t)jb * A.n_tx + t0 + t) * A.N + e];
                                const float2 L =
                                    A.lam[(((int64_t)p * A.n_bins + jb) * A.n_tx + t0 + t) * A.N + e];
                                a[jj][t] = cfma(W, G, a[jj][t]);
                                b[jj][t] = cfma(L, G, b[jj][t]);
#pragma unroll
                                for (int i = 0; i < NX; ++i) {
                                    da[jj][t][i] = cfma(W, dG[i], da[jj][t][i]);
                                    db[jj][t][i] = cfma(L, dG[i], db[jj][t][i]);
                                }
                            }
                        }
                    }
                }
            }
#pragma unroll
            for (int jj = 0; jj < JT; ++jj) {
                if (jb0 + jj < b_end) {
                    const float2 pw = A.pw[jb0 + jj];
#pragma unroll
                    for (int t = 0; t < TT; ++t) {
                        gR += cmul(pw, cmul(a[jj][t], b[jj][t])).x;
#pragma unroll
                        for (int i = 0; i < NX; ++i) {
                            const float2 q = cfma(da[jj][t][i], b[jj][t], cmul(a[jj][t], db[jj][t][i]));
                            gX[i] += cmul(pw, q).x;
                        }
                    }
                }
            }
        }
    }
    if (live) {
        // layout [range][s] of (dR, dX, dY, dZ) before the R_s factor
        float4 v = make_float4(gR, gX[0], HASY ? gX[NX - 1] : 0.f, gX[1]);
        A.part[(int64_t)it.range * A.S_total + s] = v;
    }
}

// Sums the bin ranges of every scatterer in range order and applies R_s to
// the position gradients.  Outputs may be null.
__global__ void k_adjoint_reduce(const float4* __restrict__ part, int n_ranges, int64_t S,
                                 const float* __restrict__ refl, float* dR, float* dX, float* dY,
                                 float* dZ)
{
    for (int64_t s = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; s < S;
         s += (int64_t)gridDim.x * blockDim.x) {
        float4 acc = make_float4(0.f, 0.f, 0.f, 0.f);
        for (int r = 0; r < n_ranges; ++r) {
            const float4 v = part[(int64_t)r * S + s];
            acc.x += v.x;
            acc.y += v.y;
            acc.z += v.z;
            acc.w += v.w;
        }
        const float R = refl[s];
        if (dR) dR[s] = acc.x;
        if (dX) dX[s] = R * acc.y;
        if (dY) dY[s] = R * acc.z;
        if (dZ) dZ[s] = R * acc.w;
    }
}

// Lam in the layout [p][b][t][e] from dL/drf [p][t][e][q]: lam = sum_q rho[q]
// e^{-2 pi i j q / nfft}.  Thread = bin; the phase factor is stepped from
// sample to sample by e^{2 pi i j / nfft} and re-anchored every 32 samples
// from the exact integer angle index j q mod nfft.
__global__ __launch_bounds__(256) void k_dft_t(float2* __restrict__ lam, const float* __restrict__ rho,
                                               int64_t ch0, int n_bins, int j_lo, int nfft, int n_t,
                                               int n_tx, int N)
{
    constexpr int ANCHOR = 32;
    __shared__ float s_r[8192];
    const int64_t ch = ch0 + blockIdx.y;
    const float* R = rho + ch * n_t;
    const int b = blockIdx.x * blockDim.x + threadIdx.x;
    const bool live = b < n_bins;
    const int j = (j_lo + (live ? b : 0)) % nfft;
    const float inv_n = 1.f / (float)nfft;
    const int half = nfft / 2;
    auto turns = [&](int m) { return (float)(m >= half ? m - nfft : m) * inv_n; };
    const float dc = cos_turns(turns(j)), ds = sin_turns(turns(j));   // per-sample step
    int m = 0;                                     // j q mod nfft at the next sample
    float re = 0.f, im = 0.f;
    for (int c0 = 0; c0 < n_t; c0 += 8192) {
        const int cn = min(8192, n_t - c0);
        __syncthreads();
        for (int q = threadIdx.x; q < cn; q += blockDim.x) s_r[q] = R[c0 + q];
        __syncthreads();
        for (int q0 = 0; q0 < cn; q0 += ANCHOR) {
            const int nq = min(ANCHOR, cn - q0);
            float ec = cos_turns(turns(m)), es = sin_turns(turns(m));
            for (int q = 0; q < nq; ++q) {
                const float v = s_r[q0 + q];
                re = fmaf(v, ec, re);
                im = fmaf(-v, es, im);
                const float c1 = ec * dc - es * ds;
                es = fmaf(es, dc, ec * ds);
                ec = c1;
            }
            m = (int)(((int64_t)m + (int64_t)nq * j) % nfft);
        }
    }
    if (live) {
        const int e = (int)(ch % N);
        const int64_t pt = ch / N;
        const int t = (int)(pt % n_tx);
        const int64_t p = pt / n_tx;
        lam[((p * n_bins + b) * n_tx + t) * N + e] = make_float2(re, im);
    }
}

hipError_t launch_dft_t(float2* lam, const float* rho, int64_t n_chan, int n_bins, int j_lo, int nfft,
                        int n_t, int n_tx, int N, hipStream_t st)
{
    if (n_chan == 0 || n_bins == 0) return hipSuccess;
    for (int64_t c0 = 0; c0 < n_chan; c0 += 65535) {
        const unsigned nc = (unsigned)std::min<int64_t>(65535, n_chan - c0);
        hipLaunchKernelGGL(k_dft_t, dim3((n_bins + 255) / 256, nc), dim3(256), 0, st, lam, rho, c0,
                           n_bins, j_lo, nfft, n_t, n_tx, N);
        const hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}

// Bins per tile of the vector adjoint for tt transmits per group, measured
// (100k scatterers): one transmit 6 bins (158 VGPRs, three waves per SIMD;
// 53.9 ms against 55.1 with 5 and 60.4 with 4 at four waves per SIMD, and
// 70.5 with 8 at two on an earlier build), two transmits 4 (88.5 ms; 2 bins 96.7),
// four transmits 1 (64 elements: 65.2 ms; 2 bins 67.1); with y != 0 two
// transmits take 2 bins (4 would need 239 VGPRs).
constexpr int adj_jt(int tt, bool has_y) { return tt == 1 ? 6 : tt == 2 ? (has_y ? 2 : 4) : 1; }

AdjConfig adjoint_config(int n_tx, bool has_y)
{
    AdjConfig c{};
    c.tt = n_tx >= 8 ? 8 : n_tx >= 4 ? 4 : n_tx >= 2 ? 2 : 1;
    if (has_y && c.tt > 4) c.tt = 4;
    c.jt = adj_jt(c.tt, has_y);
    c.scatterers = 256;
    c.has_y = has_y;
    return c;
}

template <int JT, int TT>
static hipError_t launch_adj_jt(const AdjConfig& c, const AdjArgs& a, int n_items, hipStream_t st)
{
    if (c.has_y)
        hipLaunchKernelGGL((k_adjoint<JT, TT, true, false>), dim3(n_items), dim3(256), 0, st, a);
    else if (c.table)
        hipLaunchKernelGGL((k_adjoint<JT, TT, false, true>), dim3(n_items), dim3(256), 0, st, a);
    else
        hipLaunchKernelGGL((k_adjoint<JT, TT, false, false>), dim3(n_items), dim3(256), 0, st, a);
    return hipGetLastError();
}


hipError_t launch_adjoint(const AdjConfig& c, const AdjArgs& a, int n_items, hipStream_t st)
{
    if (n_items <= 0) return hipSuccess;
    // the kernel's tile must be the one the item ranges were cut for
    if (c.jt != adj_jt(c.tt, c.has_y)) return hipErrorInvalidValue;
    switch (c.tt) {
    case 1: return launch_adj_jt<6, 1>(c, a, n_items, st);
    case 2: return c.has_y ? launch_adj_jt<2, 2>(c, a, n_items, st) : launch_adj_jt<4, 2>(c, a, n_items, st);
    case 4: return launch_adj_jt<1, 4>(c, a, n_items, st);
    case 8: return c.has_y ? hipErrorInvalidValue : launch_adj_jt<1, 8>(c, a, n_items, st);
    default: return hipErrorInvalidValue;
    }
}

hipError_t launch_adjoint_reduce(const float4* part, int n_ranges, int64_t S, const float* refl,
                                 float* dR, float* dX, float* dY, float* dZ, hipStream_t st)
{
    if (S == 0) return hipSuccess;
    const int grid = (int)std::min<int64_t>((S + 255) / 256, 4096);
    hipLaunchKernelGGL(k_adjoint_reduce, dim3(grid), dim3(256), 0, st, part, n_ranges, S, refl, dR, dX,
                       dY, dZ);
    return hipGetLastError();
}

}  // namespace simus
