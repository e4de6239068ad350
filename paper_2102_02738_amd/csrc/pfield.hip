// RMS pressure field (Section VII of SIMUS Part I):
//   P(X, w_j) = P_Tx(w_j) sum_n W_n exp(i w_j tau_n) G_n(X, w_j)   (Eq. 22)
//   P_RMS(X)  = sqrt(dw sum_{j=0}^{N_f} |P(X, w_j)|^2)             (Eq. 42)
// with w_j = 2 w_c j / N_f, dw = 2 w_c / N_f and P_Tx = S_P sqrt(S_T) (Eq. 28).
// The j = 0 node contributes nothing (S_P(0) = 0).
//
// One thread owns one field point and loops over all sub-elements for a tile
// of up to JT frequencies, so that each (point, sub-element) set-up, with its
// FP64 distance, serves up to JT terms; blocks cover (256 points, frequency
// range), the ranges and their tiles of nearly equal size (no short tail
// tile pays a whole set-up), and a second kernel sums the ranges in a fixed
// order.  The tile accumulates j P
// (terms j G, as in the synthesis), and 1/j^2 is applied to |j P|^2 once per
// point and frequency.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <type_traits>

#include "green.hpp"
#include "kernels.hpp"

namespace simus {

template <int JT, bool HASY, bool TABLE>
__global__ __launch_bounds__(256) void k_pfield(FieldArgs A)
{
    __shared__ float4 s_tab[TABLE ? 2 * DELTA_NT : 1];
    DeltaParams P{};
    if (TABLE) {
        for (int i = threadIdx.x; i < 2 * DELTA_NT; i += 256) s_tab[i] = A.dtab[i];
        P = *A.dpar;
        __syncthreads();
    }
    const int pblk = blockIdx.x, range = blockIdx.y;
    const int64_t pt = (int64_t)pblk * 256 + threadIdx.x;
    const bool live = pt < A.n_pts;
    const float px = live ? A.X[pt] : 0.f;
    const float py = (HASY && live) ? A.Y[pt] : 0.f;
    const float pz = live ? A.Z[pt] : 1.f;
    // the range's bins, then tiles of at most JT bins of nearly equal size
    const int b_begin = (int)((int64_t)range * A.n_bins / A.n_ranges);
    const int b_len = (int)((int64_t)(range + 1) * A.n_bins / A.n_ranges) - b_begin;
    const int n_tiles = (b_len + JT - 1) / JT;
    float sum = 0.f;
    for (int t = 0; t < n_tiles; ++t) {
        const int jb0 = b_begin + t * b_len / n_tiles;
        const int b_end = b_begin + (t + 1) * b_len / n_tiles;
        float2 acc[JT];
#pragma unroll
        for (int jj = 0; jj < JT; ++jj) acc[jj] = make_float2(0.f, 0.f);
        // A tile of exactly NT bins with the table (y = 0): one straight-line
        // bin loop that reads each next bin's table interval while the bin
        // before it is evaluated, the same operations in the same order as
        // the loop below.  Behind per-bin branches every read was waited for
        // at once, and the scalar loads of the weights, which share the LDS
        // reads' counter, made each wait a full one: Fig. 9 shape 1.336 ->
        // 1.209 ms, Fig. 10 shape 8.70 -> 8.08 ms.  Without the table, or
        // with y, the unrolled tile takes twice the registers.
        auto tile_table = [&](auto nt) {
            constexpr int NT = decltype(nt)::value;
            for (int n = 0; n < A.M; ++n) {
                const SubFrame fr = load_frame(A.sub, n);
                const int e = n / A.nu;
                Geo g = make_geo<false>(A.K, fr, px, py, pz, A.j_lo + jb0);
                if (!live) g.E = make_float2(0.f, 0.f);
                g.kap *= P.kscale;
                DeltaFetch fn = delta_fetch(s_tab, P, (float)(A.j_lo + jb0) * g.kap);
#pragma unroll
                for (int jj = 0; jj < NT; ++jj) {
                    const int jb = jb0 + jj;
                    const DeltaFetch f = fn;
                    if (jj + 1 < NT) fn = delta_fetch(s_tab, P, (float)(A.j_lo + jb + 1) * g.kap);
                    const float2 G = green_next_fetched(g, f);                           // j G
                    acc[jj] = cfma(A.W[(int64_t)jb * A.N + e], G, acc[jj]);
                }
            }
        };
        bool done = false;
        if constexpr (TABLE && !HASY) {
            // the tiles hold JT or JT - 1 bins unless the range is shorter
            const int nbt = b_end - jb0;
            if (nbt == JT) {
                tile_table(std::integral_constant<int, JT>{});
                done = true;
            } else if (nbt == JT - 1) {
                tile_table(std::integral_constant<int, JT - 1>{});
                done = true;
            }
        }
        // any other tile: each bin under its own (uniform) branch
        if (!done) {
            for (int n = 0; n < A.M; ++n) {
                const SubFrame fr = load_frame(A.sub, n);
                const int e = n / A.nu;
                Geo g = make_geo<HASY>(A.K, fr, px, py, pz, A.j_lo + jb0);
                if (!live) g.E = make_float2(0.f, 0.f);
                if (TABLE) g.kap *= P.kscale;          // the table lookup's argument
#pragma unroll
                for (int jj = 0; jj < JT; ++jj) {
                    const int jb = jb0 + jj;
                    if (jb < b_end) {
                        const float jf = (float)(A.j_lo + jb);
                        const float2 G = green_next<HASY, TABLE>(A.K, g, jf, 1.f, s_tab, P);   // j G
                        acc[jj] = cfma(A.W[(int64_t)jb * A.N + e], G, acc[jj]);
                    }
                }
            }
        }
#pragma unroll
        for (int jj = 0; jj < JT; ++jj) {
            if (jb0 + jj < b_end) {
                const float inv_j = 1.f / (float)(A.j_lo + jb0 + jj);
                const float2 v = cmul(A.ptx[jb0 + jj], acc[jj]);
                sum = fmaf(fmaf(v.x, v.x, v.y * v.y), inv_j * inv_j, sum);
            }
        }
    }
    if (live) A.part[(int64_t)range * A.n_pts + pt] = sum;
}

__global__ void k_pfield_reduce(const float* __restrict__ part, int n_ranges, int64_t n_pts,
                                float dw, float* __restrict__ out)
{
    for (int64_t p = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; p < n_pts;
         p += (int64_t)gridDim.x * blockDim.x) {
        float s = 0.f;
        for (int r = 0; r < n_ranges; ++r) s += part[(int64_t)r * n_pts + p];
        out[p] = sqrtf(dw * s);
    }
}

template <int JT>
static hipError_t launch_pf(const FieldArgs& a, bool has_y, bool table, dim3 grid, hipStream_t st)
{
    if (has_y) hipLaunchKernelGGL((k_pfield<JT, true, false>), grid, dim3(256), 0, st, a);
    else if (table) hipLaunchKernelGGL((k_pfield<JT, false, true>), grid, dim3(256), 0, st, a);
    else hipLaunchKernelGGL((k_pfield<JT, false, false>), grid, dim3(256), 0, st, a);
    return hipGetLastError();
}

hipError_t launch_pfield(const FieldArgs& a, bool has_y, bool table, int n_ranges, hipStream_t st)
{
    if (a.n_pts == 0 || n_ranges == 0) return hipSuccess;
    const dim3 grid((unsigned)((a.n_pts + 255) / 256), (unsigned)n_ranges);
    return launch_pf<PFIELD_JT>(a, has_y, table, grid, st);
}

hipError_t launch_pfield_reduce(const float* part, int n_ranges, int64_t n_pts, float dw, float* out,
                                hipStream_t st)
{
    if (n_pts == 0) return hipSuccess;
    const int grid = (int)std::min<int64_t>((n_pts + 255) / 256, 4096);
    hipLaunchKernelGGL(k_pfield_reduce, dim3(grid), dim3(256), 0, st, part, n_ranges, n_pts, dw, out);
    return hipGetLastError();
}

}  // namespace simus
