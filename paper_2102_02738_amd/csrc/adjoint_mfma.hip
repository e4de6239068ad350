// Adjoint on the matrix cores (up to 16 transmits, N <= 128, nu in {1, 2}):
// k_adjoint_mq for up to 8 transmits (four bins per step, below), k_adjoint_mt
// for 9 to 16.
//
// The gradients of the misfit need, per scatterer s, bin j and transmit t,
// four sums over the sub-elements n (see adjoint.hip):
//   a_t = sum_n W_t G,  b_t = sum_n Lam_t G,  a'_t = sum_n W_t dG,  b'_t = sum_n Lam_t dG,
// and since W and Lam depend only on the element, all of them are sums over
// elements of the element sums B = sum_{mu in e} G and dB = sum_{mu in e} dG.
// Stacking the rows (scatterer, {B, dB/dx, dB/dz, dB/dy}) and the columns
// [W_0 .. W_{TG-1} | Lam_0 .. Lam_{TG-1}] makes them one complex GEMM per
// chunk and bin:
//   V[(s, L)][col] = sum_e Brow[(s, L)][e] WL[e][col]    (32 x N x 16 NTC),
// run with FP32 MFMA (16x16x4), three real products per complex product.
// Then dL/dR_s += Re P_j sum_t a_t b_t and dL/dxi_s += Re P_j sum_t (a'_t b_t
// + a_t b'_t) (the R_s factor of the positions is applied by the reduction
// kernel), accumulated across the item's bins in registers.  Nothing is
// accumulated per bin, so each (sub-element, scatterer) pair is set up once
// per 32 bins and stepped across them (green.hpp).
//
// k_adjoint_mt.  Block: 512 threads (8 waves), chunks of 8 scatterers (32
// rows, two row tiles); work item = (phantom, scatterer slice, bin range).  With y = 0 the
// rows dB/dy are zero, and for nu = 2 a chunk takes 10 scatterers of three
// rows instead (30 of the 32 rows), so that one GEMM serves 25 % more
// scatterers.
//   Synthesis: thread = (sub-element n, group of PPT scatterers): G and its
//     gradient, element sums by one DPP exchange (nu = 2).
//   GEMM: wave = (row tile, share of the elements); three product tiles per
//     column tile go to LDS and are summed over the shares in a fixed order.
//   Gradient: lane = (scatterer, transmit); lanes of a scatterer are summed
//     once per chunk.
// The steps are software-pipelined over a chunk's bins with two barriers per
// bin: [reduction of the previous bin, synthesis] and [GEMM, gradient terms
// of the previous bin].
#include <hip/hip_runtime.h>

#include <algorithm>

#include "green.hpp"
#include "kernels.hpp"

namespace simus {


__device__ __forceinline__ floatx4 mfma_a(float a, float b, floatx4 c)
{
    return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
}

__device__ __forceinline__ float dpp_xor1(float v)
{
    return __int_as_float(__builtin_amdgcn_mov_dpp(__float_as_int(v), 0xB1, 0xF, 0xF, true));
}

// Scatterers per chunk: 10 of three rows for nu = 2 and y = 0, else 8 of four.
constexpr int adj_mt_chunk(int nuv, bool hasy) { return nuv == 2 && !hasy ? 10 : 8; }

template <int NTC, int NUV, bool HASY, bool TABLE>
__global__ __launch_bounds__(512) void k_adjoint_mt(AdjArgs A)
{
    constexpr int NB = 512;
    constexpr int NE = 128;                 // element slots
    constexpr int MS = NE * NUV;            // sub-element slots
    constexpr int SCH = adj_mt_chunk(NUV, HASY);   // scatterers per chunk
    constexpr int NL = SCH == 10 ? 3 : 4;   // rows per scatterer: B, dB/dx, dB/dz(, dB/dy)
    constexpr int ROWS = 32;                // SCH NL rows, the rest zero
    constexpr int RT = ROWS / 16;           // row tiles
    constexpr int KP = 8 / RT;              // element shares per row tile
    constexpr int KW = NE / KP;             // elements per wave
    constexpr int KS = KW / 4;              // k-steps per wave
    constexpr int TG = 8 * NTC;             // transmits
    constexpr int NC = 2 * TG;              // columns: W, then Lam
    constexpr int PPT = SCH * MS / NB;      // pairs per synthesis thread
    // LDS strides free of bank conflicts for the GEMM's reads (lanes: 16 rows,
    // 2 columns, rows NE + 2 apart) and for the product tiles (per lane, the
    // accumulator registers v rows PV apart, column tiles PC apart)
    constexpr int LST = NE + 2;             // row stride of the element sums
    constexpr int WS = NE + 2;              // row stride of the staged columns
    constexpr int PV = 80;
    constexpr int PC = 4 * PV + 32;         // per column tile
    constexpr int PP = NTC * PC;            // per product
    constexpr int JS = 32;                  // bins per set-up
    constexpr int NX = HASY ? 3 : 2;        // coordinates: X, Z (, Y)
    static_assert(NUV == 1 || NUV == 2, "nu must be 1 or 2");
    static_assert(PPT * (NB / MS) == SCH, "synthesis threads must cover the chunk");
    static_assert(SCH * NL <= ROWS, "rows of a chunk");
    static_assert(NC * NE % NB == 0, "column staging must divide evenly");

    __shared__ float4 s_sc[SCH];
    __shared__ float2 s_L[ROWS * LST];
    __shared__ float2 s_WL[NC * WS];
    __shared__ float s_part[8][3 * PP];
    __shared__ float2 s_V[ROWS][NC];
    __shared__ float4 s_tab[TABLE ? 2 * DELTA_NT : 1];

    const int tid = threadIdx.x;
    const int wave = tid >> 6, lane = tid & 63;
    const int gi = lane & 15, gk = lane >> 4;
    // synthesis role
    const int n = tid % MS, sp = tid / MS;
    const bool active = n < A.M;
    const SubFrame fr = load_frame(A.sub, active ? n : 0);
    // GEMM role
    const int rt = wave / KP, kp = wave % KP;
    // gradient role
    const bool glane = tid < SCH * TG;
    const int gs = tid / TG, gt = tid % TG;

    DeltaParams P{};
    if (TABLE) {
        for (int i = tid; i < 2 * DELTA_NT; i += NB) s_tab[i] = A.dtab[i];
        P = *A.dpar;
    }
    // rows that no scatterer fills (dB/dy for y = 0 with 8-scatterer chunks,
    // rows 30 and 31 with 10) stay zero
    for (int i = tid; i < ROWS * LST; i += NB) s_L[i] = make_float2(0.f, 0.f);

    const AdjItem it = A.items[blockIdx.x];
    const int b_begin = it.range * A.range_bins;
    const int b_end = min(A.n_bins, b_begin + A.range_bins);
    const int p = it.phantom;

    for (int s0 = it.s_begin; s0 < it.s_end; s0 += SCH) {
        if (tid < SCH) {
            const int s = s0 + tid;
            float4 v = make_float4(0.f, 0.f, 1.f, 0.f);     // padding
            if (s < it.s_end) v = make_float4(A.x[s], HASY ? A.y[s] : 0.f, A.z[s], 0.f);
            s_sc[tid] = v;
        }
        __syncthreads();
        float gR = 0.f, gX[NX];
#pragma unroll
        for (int i = 0; i < NX; ++i) gX[i] = 0.f;

        // 3. the partial products of a bin -> s_V (sum over the element
        //    shares in a fixed order, the three products combined)
        auto reduce = [&]() {
            for (int idx = tid; idx < ROWS * NC; idx += NB) {
                const int r = idx / NC, col = idx % NC;
                const int d = (col >> 4) * PC + (r & 3) * PV + ((r >> 2) & 3) * 16 + (col & 15);
                const int w0 = (r >> 4) * KP;
                float q1 = 0.f, q2 = 0.f, q3 = 0.f;
#pragma unroll
                for (int k = 0; k < KP; ++k) {
                    q1 += s_part[w0 + k][d];
                    q2 += s_part[w0 + k][PP + d];
                    q3 += s_part[w0 + k][2 * PP + d];
                }
                s_V[r][col] = make_float2(q1 - q2, q3 - q1 - q2);
            }
        };
        // 4. gradient terms of bin jb for lane (scatterer gs, transmit gt)
        auto gradient = [&](int jb) {
            if (!glane) return;
            const float2 pw = A.pw[jb];
            const float2 a = s_V[gs * NL][gt], b = s_V[gs * NL][TG + gt];
            gR += cmul(pw, cmul(a, b)).x;
#pragma unroll
            for (int i = 0; i < NX; ++i) {
                const float2 da = s_V[gs * NL + 1 + i][gt], db = s_V[gs * NL + 1 + i][TG + gt];
                gX[i] += cmul(pw, cfma(da, b, cmul(a, db))).x;
            }
        };
        // Software pipeline over the chunk's bins, two barriers per bin:
        //   A: reduce the previous bin (3); this bin's synthesis (1) and columns;
        //   B: this bin's GEMM (2); the previous bin's gradient terms (4).
        // The chunk's last bin is finished after the loop.
        bool pend = false;                     // uniform: a bin awaits steps 3-4
        int pend_jb = 0;
        for (int jb0 = b_begin; jb0 < b_end; jb0 += JS) {
            Geo g[PPT];
            GeoD D[PPT];
#pragma unroll
            for (int k = 0; k < PPT; ++k) {
                const float4 v = s_sc[sp * PPT + k];
                g[k] = make_geo<HASY, true>(A.K, fr, v.x, v.y, v.z, A.j_lo + jb0, &D[k]);
                if (!active) g[k].E = make_float2(0.f, 0.f);
            }
            const int nb = min(JS, b_end - jb0);
            for (int jj = 0; jj < nb; ++jj) {
                const int jb = jb0 + jj;
                const float jf = (float)(A.j_lo + jb);
                const float inv_j = rcp_fast(jf);
                // ---- segment A
                // 0. columns of this bin: W of the transmits, then Lam; zero
                //    outside N x n_tx.  Loaded here, stored to LDS after the
                //    synthesis so that the loads' latency is hidden behind it.
                constexpr int NW = NC * NE / NB;
                float2 wl[NW];
#pragma unroll
                for (int q = 0; q < NW; ++q) {
                    const int idx = tid + q * NB;
                    const int col = idx / NE, e = idx % NE;
                    const int t = col < TG ? col : col - TG;
                    const int tt = min(t, A.n_tx - 1), ee = min(e, A.N - 1);
                    const float2 w = col < TG ? A.W[((int64_t)jb * A.n_tx + tt) * A.N + ee]
                                              : A.lam[(((int64_t)p * A.n_bins + jb) * A.n_tx + tt) * A.N + ee];
                    const bool use = e < A.N && t < A.n_tx;
                    wl[q] = make_float2(use ? w.x : 0.f, use ? w.y : 0.f);
                }
                if (pend) reduce();
                // 1. G and its gradient -> element sums, rows (s, L)
#pragma unroll
                for (int k = 0; k < PPT; ++k) {
                    const int s = sp * PPT + k;
                    float2 dG[NX];
                    float2 v[NX + 1];
                    v[0] = green_grad_next<HASY, TABLE, NX>(A.K, g[k], D[k], jf, inv_j, s_tab, P, dG);
#pragma unroll
                    for (int i = 0; i < NX; ++i) v[1 + i] = dG[i];
#pragma unroll
                    for (int L = 0; L <= NX; ++L) {
                        float2 b = v[L];
                        if (NUV == 2) {
                            b.x += dpp_xor1(b.x);
                            b.y += dpp_xor1(b.y);
                        }
                        s_L[(s * NL + L) * LST + (NUV == 2 ? (n >> 1) : n)] = b;
                    }
                }
#pragma unroll
                for (int q = 0; q < NW; ++q) {
                    const int idx = tid + q * NB;
                    s_WL[(idx / NE) * WS + idx % NE] = wl[q];
                }
                __syncthreads();
                // ---- segment B
                // 2. GEMM share: rows rt 16 + gi, columns ct 16 + gi, elements
                //    kp KW + 4 k + gk
                {
                    const float2* lp = s_L + (rt * 16 + gi) * LST + kp * KW + gk;
                    float2 la[KS];
#pragma unroll
                    for (int k = 0; k < KS; ++k) la[k] = lp[4 * k];
#pragma unroll
                    for (int ct = 0; ct < NTC; ++ct) {
                        const float2* wp = s_WL + (ct * 16 + gi) * WS + kp * KW + gk;
                        float2 wa[KS];
#pragma unroll
                        for (int k = 0; k < KS; ++k) wa[k] = wp[4 * k];
                        floatx4 p1 = {0.f, 0.f, 0.f, 0.f}, p2 = p1, p3 = p1;
#pragma unroll
                        for (int k = 0; k < KS; ++k) {
                            p1 = mfma_a(la[k].x, wa[k].x, p1);
                            p2 = mfma_a(la[k].y, wa[k].y, p2);
                            p3 = mfma_a(la[k].x + la[k].y, wa[k].x + wa[k].y, p3);
                        }
                        // D[row][col]: col = lane % 16, row = 4 (lane / 16) + v
#pragma unroll
                        for (int v = 0; v < 4; ++v) {
                            float* q = &s_part[wave][ct * PC + v * PV + lane];
                            q[0] = p1[v];
                            q[PP] = p2[v];
                            q[2 * PP] = p3[v];
                        }
                    }
                }
                if (pend) gradient(pend_jb);
                __syncthreads();
                pend = true;
                pend_jb = jb;
            }
        }
        if (pend) {     // steps 3-4 of the chunk's last bin
            reduce();
            __syncthreads();
            gradient(pend_jb);
        }
        // sum the transmit lanes of each scatterer; layout [range][s] of
        // (dR, dX, dY, dZ) before the R_s factor
        if (glane) {
#pragma unroll
            for (int m = 1; m < TG; m <<= 1) {
                gR += __shfl_xor(gR, m);
#pragma unroll
                for (int i = 0; i < NX; ++i) gX[i] += __shfl_xor(gX[i], m);
            }
            const int s = s0 + gs;
            if (gt == 0 && s < it.s_end)
                A.part[(int64_t)it.range * A.S_total + s] = make_float4(gR, gX[0], HASY ? gX[NX - 1] : 0.f, gX[1]);
        }
        __syncthreads();
    }
}

// Up to 8 transmits: four bins per step, two barriers per step.  The
// columns [W_0 .. W_7 | Lam_0 .. Lam_7] come from a padded table WL in global
// memory (zero outside N x n_tx), read by each wave ahead of its GEMM, so
// nothing is staged or reduced in LDS:
//   P1  every thread: the gradient terms of the previous step's four bins
//       (lane = (scatterer, transmit, bin)), then G and its gradient for its
//       pairs and four bins -> element sums, rows (s, L), one LDS tile per bin;
//   P2  BF: waves 0-3, the GEMM of bin w, both row tiles, over all 128
//       element slots -> V of that bin in LDS; a bin's columns are read once
//       per block and step, the zero ones past the transmit count as one
//       cache line.  With each wave on one row tile (both waves of a bin
//       reading its 16 KiB of columns), 5 plane waves, 100k scatterers took
//       77.9 ms instead of 72.5 (results bit-identical); summing two halves
//       of the elements in LDS with float atomics took 160.8 ms.  FP32
//       products: wave w, bin w / 2, row tile w % 2.
// BF: the GEMM's products as three products of bf16 high and low parts
// (v_mfma_f32_16x16x32_bf16, FP32 accumulation, about 2^-16 of each
// product, as in k_synth_mb): the element sums go to LDS in FP32 and the
// GEMM wave splits each once as it reads it (splitting in the synthesis,
// where both lanes of a sub-element pair split the same sum, took 72.8 ms
// instead of 69.6 on 5 plane waves, 100k scatterers, results
// bit-identical); the table holds WL[p][bin][col][e] as (h, l) words.
// Otherwise FP32 16x16x4 MFMAs with three products per complex product and
// WL[p][bin][e][col] as float2.
// Lanes of a scatterer are summed once per chunk (transmits and bins, in a
// fixed order).
template <int NUV, bool HASY, bool TABLE, bool BF>
__global__ __launch_bounds__(512) void k_adjoint_mq(AdjArgs A)
{
    constexpr int NB = 512;
    constexpr int NE = 128;                 // element slots
    constexpr int MS = NE * NUV;            // sub-element slots
    constexpr int SCH = adj_mt_chunk(NUV, HASY);   // scatterers per chunk
    constexpr int NL = SCH == 10 ? 3 : 4;   // rows per scatterer: B, dB/dx, dB/dz(, dB/dy)
    constexpr int ROWS = 32;                // SCH NL rows, the rest zero
    constexpr int LST = BF ? NE + 4 : NE + 2;   // row stride (float2) of the element sums
    constexpr int TG = 8;                   // transmits
    constexpr int NC = 2 * TG;              // columns: W, then Lam
    constexpr int VST = NC + 2;             // row stride of V
    constexpr int JB = 4;                   // bins per step: wave = (bin, row tile)
    constexpr int JS = 32;                  // bins per set-up, a multiple of JB
    constexpr int KS = NE / 4;              // FP32 k-steps (4 elements)
    constexpr int KB = 8;                   // FP32 k-steps of columns loaded ahead
    constexpr int KSB = NE / 16;            // bf16 k-steps (16 elements)
    constexpr int PPT = SCH * MS / NB;      // pairs per synthesis thread
    constexpr int NX = HASY ? 3 : 2;        // coordinates: X, Z (, Y)
    constexpr int GL = SCH * TG * JB;       // gradient lanes
    constexpr int NPL = BF ? 2 : 1;         // LDS planes of the element sums
    static_assert(NUV == 1 || NUV == 2, "nu must be 1 or 2");
    static_assert(PPT * (NB / MS) == SCH, "synthesis threads must cover the chunk");
    static_assert(SCH * NL <= ROWS && GL <= NB && JS % JB == 0 && KS % KB == 0, "shape");
    static_assert(TG * JB == 32, "a scatterer's gradient lanes are 32 consecutive lanes");

    __shared__ float4 s_sc[SCH];
    // the element sums: one plane of float2 [row][LST] (BF: over both halves of
    // the array, LST = 132; else LST = 130)
    __shared__ __align__(16) uint32_t s_L[JB][NPL][ROWS * LST * (BF ? 1 : 2)];
    __shared__ float2 s_V[JB][ROWS * VST];
    __shared__ float4 s_tab[TABLE ? 2 * DELTA_NT : 1];

    const int tid = threadIdx.x;
    const int wave = tid >> 6, lane = tid & 63;
    const int gi = lane & 15, gk = lane >> 4;
    // synthesis role
    const int n = tid % MS, sp = tid / MS;
    const bool active = n < A.M;
    const SubFrame fr = load_frame(A.sub, active ? n : 0);
    // GEMM role (FP32 products): bin wj of the step, row tile rt
    const int wj = wave >> 1, rt = wave & 1;
    // gradient role: lane = (scatterer gs, transmit gt, bin gj)
    const bool glane = tid < GL;
    const int gs = tid >> 5, gt = (tid >> 2) & 7, gj = tid & 3;

    DeltaParams P{};
    if (TABLE) {
        for (int i = tid; i < 2 * DELTA_NT; i += NB) s_tab[i] = A.dtab[i];
        P = *A.dpar;
    }
    // rows that no scatterer fills stay zero
    for (int i = tid; i < (int)(sizeof(s_L) / 4); i += NB) (&s_L[0][0][0])[i] = 0u;

    const AdjItem it = A.items[blockIdx.x];
    const int b_begin = it.range * A.range_bins;
    const int b_end = min(A.n_bins, b_begin + A.range_bins);
    const int p = it.phantom;
    const float2* wl_p = A.WL + (int64_t)p * A.n_bins * NE * NC;

    for (int s0 = it.s_begin; s0 < it.s_end; s0 += SCH) {
        if (tid < SCH) {
            const int s = s0 + tid;
            float4 v = make_float4(0.f, 0.f, 1.f, 0.f);     // padding
            if (s < it.s_end) v = make_float4(A.x[s], HASY ? A.y[s] : 0.f, A.z[s], 0.f);
            s_sc[tid] = v;
        }
        __syncthreads();
        float gR = 0.f, gX[NX];
#pragma unroll
        for (int i = 0; i < NX; ++i) gX[i] = 0.f;

        // gradient terms of the step's bin j0 + gj for lane (gs, gt)
        auto gradient = [&](int j0) {
            const int jb = j0 + gj;
            if (!glane || jb >= b_end) return;
            const float2 pw = A.pw[jb];
            const float2* V = s_V[gj];
            const float2 a = V[gs * NL * VST + gt], b = V[gs * NL * VST + TG + gt];
            gR += cmul(pw, cmul(a, b)).x;
#pragma unroll
            for (int i = 0; i < NX; ++i) {
                const float2 da = V[(gs * NL + 1 + i) * VST + gt], db = V[(gs * NL + 1 + i) * VST + TG + gt];
                gX[i] += cmul(pw, cfma(da, b, cmul(a, db))).x;
            }
        };
        bool pend = false;                     // uniform: a step awaits its gradient terms
        int pend_j0 = 0;
        for (int jb0 = b_begin; jb0 < b_end; jb0 += JS) {
            Geo g[PPT];
            GeoD D[PPT];
#pragma unroll
            for (int k = 0; k < PPT; ++k) {
                const float4 v = s_sc[sp * PPT + k];
                g[k] = make_geo<HASY, true>(A.K, fr, v.x, v.y, v.z, A.j_lo + jb0, &D[k]);
                if (!active) g[k].E = make_float2(0.f, 0.f);
            }
            const int nb = min(JS, b_end - jb0);
            for (int jq = 0; jq < nb; jq += JB) {
                // ---- P1: the previous step's gradient terms; G and its
                //      gradient for the step's four bins (past the range's
                //      end they are stepped but not used)
                if (pend) gradient(pend_j0);
                // the four bins unrolled, so that their table reads can be
                // issued ahead (5 plane waves, 100k scatterers: 82.0 -> 78.3 ms)
#pragma unroll
                for (int jj = 0; jj < JB; ++jj) {
                    prio_by_progress(jj, JB);
                    const float jf = (float)(A.j_lo + jb0 + jq + jj);
                    const float inv_j = rcp_fast(jf);
#pragma unroll
                    for (int k = 0; k < PPT; ++k) {
                        const int s = sp * PPT + k;
                        float2 dG[NX];
                        float2 v[NX + 1];
                        v[0] = green_grad_next<HASY, TABLE, NX>(A.K, g[k], D[k], jf, inv_j, s_tab, P, dG);
#pragma unroll
                        for (int i = 0; i < NX; ++i) v[1 + i] = dG[i];
#pragma unroll
                        for (int L = 0; L <= NX; ++L) {
                            float2 b = v[L];
                            if (NUV == 2) {
                                b.x += dpp_xor1(b.x);
                                b.y += dpp_xor1(b.y);
                            }
                            const int e = NUV == 2 ? (n >> 1) : n;
                            const int at = (s * NL + L) * LST + e;
                            if constexpr (BF) {
                                // FP32 element sums, float2 [row][LST]; the GEMM
                                // wave splits them.  nu = 2: the pair's even
                                // lane stores Re, the odd one Im
                                if (NUV == 2)
                                    reinterpret_cast<float*>(s_L[jj][0])[2 * at + (n & 1)] = (n & 1) ? b.y : b.x;
                                else
                                    reinterpret_cast<float2*>(s_L[jj][0])[at] = b;
                            } else {
                                reinterpret_cast<float2*>(s_L[jj][0])[at] = b;
                            }
                        }
                    }
                }
                const int jbw = min(jb0 + jq + wj, b_end - 1);
                if constexpr (BF) {
                    // waves 0..3: bin w of the step, both row tiles; the split
                    // columns WL[p][bin][col = gi][e = 16 k + 4 gk .. + 3]
                    const int bj = wave & (JB - 1);
                    const int jbr = min(jb0 + jq + bj, b_end - 1);
                    // (columns past the transmit count are zero in the table:
                    // their lanes all read the first of them)
                    const int wc = (gi & TG) | min(gi & (TG - 1), A.n_tx);
                    const uint2* wg = reinterpret_cast<const uint2*>(wl_p) + ((int64_t)jbr * NC + wc) * NE + 4 * gk;
                    uint4 wr[KSB][2];
                    if (wave < JB) {
#pragma unroll
                        for (int k = 0; k < KSB; ++k) {
                            const uint4* q = reinterpret_cast<const uint4*>(wg + 16 * k);
                            wr[k][0] = q[0];
                            wr[k][1] = q[1];
                        }
                    }
                    __syncthreads();
                    if (wave < JB) {
                        floatx4 re[2], im[2];
#pragma unroll
                        for (int r = 0; r < 2; ++r) re[r] = im[r] = floatx4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
                        for (int k = 0; k < KSB; ++k) {
                            const uint32_t wh[4] = {wr[k][0].x, wr[k][0].z, wr[k][1].x, wr[k][1].z};
                            const uint32_t wlo[4] = {wr[k][0].y, wr[k][0].w, wr[k][1].y, wr[k][1].w};
                            const u32x4 rh = {bf_conj(wh[0]), bf_conj(wh[1]), bf_conj(wh[2]), bf_conj(wh[3])};
                            const u32x4 rl = {bf_conj(wlo[0]), bf_conj(wlo[1]), bf_conj(wlo[2]), bf_conj(wlo[3])};
                            const u32x4 ih = {bf_swap(wh[0]), bf_swap(wh[1]), bf_swap(wh[2]), bf_swap(wh[3])};
                            const u32x4 il = {bf_swap(wlo[0]), bf_swap(wlo[1]), bf_swap(wlo[2]), bf_swap(wlo[3])};
#pragma unroll
                            for (int r = 0; r < 2; ++r) {
                                // elements 16 k + 4 gk .. + 3 of row 16 r + gi, split
                                const float2* pf = reinterpret_cast<const float2*>(s_L[bj][0]) + (r * 16 + gi) * LST + 16 * k + 4 * gk;
                                const float4 f01 = *reinterpret_cast<const float4*>(pf);
                                const float4 f23 = *reinterpret_cast<const float4*>(pf + 2);
                                const float fx[4] = {f01.x, f01.z, f23.x, f23.z}, fy[4] = {f01.y, f01.w, f23.y, f23.w};
                                u32x4 ah, al;
#pragma unroll
                                for (int q = 0; q < 4; ++q) {
                                    const uint32_t h = pack_bf16(fx[q], fy[q]);
                                    ah[q] = h;
                                    al[q] = pack_bf16(fx[q] - bf16_lo(h), fy[q] - bf16_hi(h));
                                }
                                re[r] = mfma_bf(ah, rh, re[r]);
                                re[r] = mfma_bf(ah, rl, re[r]);
                                re[r] = mfma_bf(al, rh, re[r]);
                                im[r] = mfma_bf(ah, ih, im[r]);
                                im[r] = mfma_bf(ah, il, im[r]);
                                im[r] = mfma_bf(al, ih, im[r]);
                            }
                        }
                        float2* V = s_V[bj];
#pragma unroll
                        for (int r = 0; r < 2; ++r)
#pragma unroll
                            for (int v = 0; v < 4; ++v) V[(r * 16 + 4 * gk + v) * VST + gi] = make_float2(re[r][v], im[r][v]);
                    }
                } else {
                    // this wave's columns: WL[p][bin][e = 4 k + gk][col = gi],
                    // k-step stride 64; the first batch in flight across the barrier
                    const float2* wg = wl_p + ((int64_t)jbw * NE + gk) * NC + gi;
                    float2 wa[2][KB];
#pragma unroll
                    for (int k = 0; k < KB; ++k) wa[0][k] = wg[64 * k];
                    __syncthreads();
                    // ---- P2: GEMM of bin wj, row tile rt: rows rt 16 + gi,
                    //      k = element 4 k + gk, columns gi
                    const float2* lp = reinterpret_cast<const float2*>(s_L[wj][0]) + (rt * 16 + gi) * LST + gk;
                    floatx4 p1 = {0.f, 0.f, 0.f, 0.f}, p2 = p1, p3 = p1;
#pragma unroll
                    for (int k0 = 0; k0 < KS; k0 += KB) {
                        const int cur = (k0 / KB) & 1;
                        if (k0 + KB < KS) {
#pragma unroll
                            for (int k = 0; k < KB; ++k) wa[cur ^ 1][k] = wg[64 * (k0 + KB + k)];
                        }
                        float2 la[KB];
#pragma unroll
                        for (int k = 0; k < KB; ++k) la[k] = lp[4 * (k0 + k)];
#pragma unroll
                        for (int k = 0; k < KB; ++k) {
                            p1 = mfma_a(la[k].x, wa[cur][k].x, p1);
                            p2 = mfma_a(la[k].y, wa[cur][k].y, p2);
                            p3 = mfma_a(la[k].x + la[k].y, wa[cur][k].x + wa[cur][k].y, p3);
                        }
                    }
                    // D[row][col]: row rt 16 + 4 gk + v, col gi
                    float2* V = s_V[wj];
#pragma unroll
                    for (int v = 0; v < 4; ++v)
                        V[(rt * 16 + 4 * gk + v) * VST + gi] = make_float2(p1[v] - p2[v], p3[v] - p1[v] - p2[v]);
                }
                __syncthreads();
                pend = true;
                pend_j0 = jb0 + jq;
            }
        }
        if (pend) gradient(pend_j0);
        // sum a scatterer's 32 lanes (transmits, bins); layout [range][s] of
        // (dR, dX, dY, dZ) before the R_s factor
        if (glane) {
#pragma unroll
            for (int m = 1; m < 32; m <<= 1) {
                gR += __shfl_xor(gR, m);
#pragma unroll
                for (int i = 0; i < NX; ++i) gX[i] += __shfl_xor(gX[i], m);
            }
            const int s = s0 + gs;
            if ((tid & 31) == 0 && s < it.s_end)
                A.part[(int64_t)it.range * A.S_total + s] = make_float4(gR, gX[0], HASY ? gX[NX - 1] : 0.f, gX[1]);
        }
        __syncthreads();
    }
}

template <int NUV, bool BF>
static hipError_t launch_adj_mq_nuv(const AdjConfig& c, const AdjArgs& a, int n_items, hipStream_t st)
{
    if (c.has_y)
        hipLaunchKernelGGL((k_adjoint_mq<NUV, true, false, BF>), dim3(n_items), dim3(512), 0, st, a);
    else if (c.table)
        hipLaunchKernelGGL((k_adjoint_mq<NUV, false, true, BF>), dim3(n_items), dim3(512), 0, st, a);
    else
        hipLaunchKernelGGL((k_adjoint_mq<NUV, false, false, BF>), dim3(n_items), dim3(512), 0, st, a);
    return hipGetLastError();
}

// WL for k_adjoint_mq: column c is W of transmit c (c < 8), then Lam of
// transmit c - 8, zero outside N x n_tx.  bf16 == false: float2
// WL[p][bin][e][16]; bf16 == true: WL[p][bin][16][e] as packed split words
// (x = (re_h, im_h), y = (re_l, im_l)).
__global__ void k_wltable(float2* __restrict__ WL, const float2* __restrict__ W,
                          const float2* __restrict__ lam, int n_ph, int n_bins, int n_tx, int N, bool bf16)
{
    const int64_t total = (int64_t)n_ph * n_bins * 128 * 16;
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < total;
         i += (int64_t)gridDim.x * blockDim.x) {
        const int c = bf16 ? (int)((i >> 7) & 15) : (int)(i & 15);
        const int e = bf16 ? (int)(i & 127) : (int)((i >> 4) & 127);
        const int64_t pb = i >> 11;                 // p n_bins + bin
        const int b = (int)(pb % n_bins);
        const int t = c & 7;
        float2 w = make_float2(0.f, 0.f);
        if (e < N && t < n_tx)
            w = c < 8 ? W[((int64_t)b * n_tx + t) * N + e] : lam[(pb * n_tx + t) * N + e];
        if (bf16) {
            const uint32_t h = pack_bf16(w.x, w.y);
            const uint32_t l = pack_bf16(w.x - bf16_lo(h), w.y - bf16_hi(h));
            w = make_float2(__uint_as_float(h), __uint_as_float(l));
        }
        WL[i] = w;
    }
}

hipError_t launch_wltable(float2* WL, const float2* W, const float2* lam, int n_ph, int n_bins, int n_tx,
                          int N, bool bf16, hipStream_t st)
{
    const int64_t total = (int64_t)n_ph * n_bins * 128 * 16;
    if (total == 0) return hipSuccess;
    const int grid = (int)std::min<int64_t>((total + 255) / 256, 8192);
    hipLaunchKernelGGL(k_wltable, dim3(grid), dim3(256), 0, st, WL, W, lam, n_ph, n_bins, n_tx, N, bf16);
    return hipGetLastError();
}

template <int NTC, int NUV>
static hipError_t launch_adj_mt_nuv(const AdjConfig& c, const AdjArgs& a, int n_items, hipStream_t st)
{
    if (c.has_y)
        hipLaunchKernelGGL((k_adjoint_mt<NTC, NUV, true, false>), dim3(n_items), dim3(512), 0, st, a);
    else if (c.table)
        hipLaunchKernelGGL((k_adjoint_mt<NTC, NUV, false, true>), dim3(n_items), dim3(512), 0, st, a);
    else
        hipLaunchKernelGGL((k_adjoint_mt<NTC, NUV, false, false>), dim3(n_items), dim3(512), 0, st, a);
    return hipGetLastError();
}

bool adjoint_mt_supported(int M, int N, int n_tx)
{
    const int nu = N > 0 ? M / N : 0;
    return n_tx >= 1 && n_tx <= 16 && N >= 1 && N <= 128 && (nu == 1 || nu == 2) && M == nu * N;
}

AdjConfig adjoint_mt_config(int M, int N, int n_tx, bool has_y)
{
    AdjConfig c{};
    c.mfma = true;
    c.tt = n_tx <= 8 ? 8 : 16;
    c.wl = n_tx <= 8;         // k_adjoint_mq, columns from the padded table WL
    c.jt = 32;                // bins per set-up (JS), the bin-range granule
    c.pair = M == 2 * N;
    // scatterers per item, a multiple of the chunk
    c.scatterers = adj_mt_chunk(c.pair ? 2 : 1, has_y) == 10 ? 60 : 64;
    c.has_y = has_y;
    return c;
}

hipError_t launch_adjoint_mt(const AdjConfig& c, const AdjArgs& a, int n_items, hipStream_t st)
{
    if (n_items <= 0) return hipSuccess;
    if (c.tt == 8 && c.wl) {
        if (!a.WL) return hipErrorInvalidValue;
        if (c.bf) return c.pair ? launch_adj_mq_nuv<2, true>(c, a, n_items, st) : launch_adj_mq_nuv<1, true>(c, a, n_items, st);
        return c.pair ? launch_adj_mq_nuv<2, false>(c, a, n_items, st) : launch_adj_mq_nuv<1, false>(c, a, n_items, st);
    }
    if (c.tt == 16) return c.pair ? launch_adj_mt_nuv<2, 2>(c, a, n_items, st) : launch_adj_mt_nuv<2, 1>(c, a, n_items, st);
    return hipErrorInvalidValue;
}

}  // namespace simus
