// Synthesis for many transmits: the transmit contraction of Eq. (29),
//   a[s][t] = sum_n G[n][s] W[n][t],
// is a complex GEMM (16 scatterers x nu N sub-elements x up to 32 transmits
// per group), and so is the receive contraction of Eqs. (32)-(33),
//   X[e][t] += sum_s (sum_{mu in e} G[mu][s]) R_s a[s][t]
// (elements x 16 scatterers x transmits).  Both run on the matrix cores with
// FP32 MFMA (16x16x4); the Green's terms are synthesised on the VALU
// (green.hpp).  X accumulates in MFMA registers across all scatterers of the
// item.
//
// Block: 512 threads (8 waves).  Synthesis: thread = (sub-element n, half of
// the 16-scatterer chunk), 8 pairs stepped across the item's bin tile.
// Transmit GEMM: a complex product is four real MFMA products; the 2 * NTP
// output tiles (re/im of each 16-transmit tile) are spread over the 8 waves,
// each wave covering a share of the sub-elements, and the shares are summed
// in LDS in a fixed order.  Receive GEMM: wave w owns elements 16 w .. 16 w + 15
// and all output tiles of the group.
#include <hip/hip_runtime.h>

#include <algorithm>

#include "green.hpp"
#include "kernels.hpp"

namespace simus {

typedef float floatx4 __attribute__((ext_vector_type(4)));

template <int NTP, int NQ, int JT, bool HASY, bool TABLE, bool PERSIST>
__global__ __launch_bounds__(512) void k_synth_mt(SynthArgs A)
{
    constexpr int NB = 512;
    constexpr int MS = 256;                 // sub-element slots
    constexpr int SCH = 16;                 // scatterers per chunk (MFMA rows)
    constexpr int GS = MS + 4;              // LDS row stride of the G tile (float2)
    constexpr int TPG = 16 * NTP;           // transmit columns of the group
    constexpr int NOUT = 2 * NTP;           // output tiles (re, im per column tile)
    constexpr int KSPLIT = 8 / NOUT;        // waves per output tile
    constexpr int KW = MS / KSPLIT;         // sub-elements per wave
    constexpr int EP = NB / NQ;             // element slots

    __shared__ float4 s_sc[SCH];
    __shared__ float2 s_G[SCH * GS];
    __shared__ float s_part[8][256];
    __shared__ float2 s_c[SCH][TPG];
    __shared__ float4 s_tab[TABLE ? 2 * DELTA_NT : 1];
    constexpr int WS = EP + 1;              // LDS row stride of the staged weights
    __shared__ float2 s_W[TPG * WS];

    const int tid = threadIdx.x;
    const int wave = tid >> 6, lane = tid & 63;
    // synthesis role
    const int n = tid & (MS - 1), sh = tid / MS;
    const bool active = n < A.M;
    const SubFrame fr = load_frame(A.sub, active ? n : 0);
    // receive role: element tile of this wave
    const int mt_e = wave * 16;
    const bool re_live = mt_e < A.N;
    // GEMM role
    const int otile = wave % NOUT, kpart = wave / NOUT;
    const int ct = otile >> 1;              // column tile
    const bool out_im = otile & 1;

    DeltaParams P{};
    if (TABLE) {
        for (int i = tid; i < 2 * DELTA_NT; i += NB) s_tab[i] = A.dtab[i];
        P = *A.dpar;
    }

    // Static launch: one item per block.  Persistent launch: blocks draw
    // items from a work counter until it passes n_items (every block exits).
    __shared__ int s_item;
    int item = blockIdx.x;
    if (PERSIST) {
        if (tid == 0) s_item = atomicAdd(A.ticket, 1);
        __syncthreads();
        item = s_item;
    }
    while (item < A.n_items) {
        const Item it = A.items[item];
        const int bt = it.tile & 0xffff, tg = it.tile >> 16;
        const int jb0 = bt * JT;
        const int nb = min(JT, A.n_bins - jb0);
        const int t0 = tg * TPG;

        // receive accumulators: [bin][column tile][re, im]
        floatx4 X[JT][NTP][2];
#pragma unroll
        for (int jj = 0; jj < JT; ++jj)
#pragma unroll
            for (int c = 0; c < NTP; ++c) X[jj][c][0] = X[jj][c][1] = floatx4{0.f, 0.f, 0.f, 0.f};

        for (int s0 = it.s_begin; s0 < it.s_end; s0 += SCH) {
            __syncthreads();
            if (tid < SCH) {
                const int s = s0 + tid;
                float4 v = make_float4(0.f, 0.f, 1.f, 0.f);     // padding: R = 0
                if (s < it.s_end) v = make_float4(A.x[s], HASY ? A.y[s] : 0.f, A.z[s], A.refl[s]);
                s_sc[tid] = v;
            }
            __syncthreads();
            Geo g[8];
#pragma unroll
            for (int k = 0; k < 8; ++k) {
                const float4 v = s_sc[sh * 8 + k];
                g[k] = make_geo<HASY>(A.K, fr, v.x, v.y, v.z, A.j_lo + jb0);
                if (!active) g[k].E = make_float2(0.f, 0.f);
            }
            // GEMM operand lanes: rows s = lane % 16, columns t = ct * 16 + lane % 16
            const int gi = lane & 15, gk = lane >> 4;
            const int nbase = kpart * KW;
            // The bin loop is unrolled so that the receive accumulators X[jj] stay
            // in registers; nb is uniform, so the barriers inside are too.
#pragma unroll
            for (int jj = 0; jj < JT; ++jj) {
                if (jj >= nb) break;
                const int jb = jb0 + jj;
                const float jf = (float)(A.j_lo + jb);
                const float inv_j = rcp_fast(jf);
                // 0. stage the transmit weights of this bin, W[t][e], in LDS
                {
                    const int e2 = tid % EP;
#pragma unroll
                    for (int t = tid / EP; t < TPG; t += NQ) {
                        const int tt = t0 + t;
                        if (e2 < A.N)
                            s_W[t * WS + e2] = tt < A.n_tx ? A.W[((int64_t)jb * A.n_tx + tt) * A.N + e2]
                                                           : make_float2(0.f, 0.f);
                    }
                }
                // 1. Green's terms of the chunk -> LDS tile [s][n]
#pragma unroll
                for (int k = 0; k < 8; ++k)
                    s_G[(sh * 8 + k) * GS + n] = green_next<HASY, TABLE>(A.K, g[k], jf, inv_j, s_tab, P);
                __syncthreads();
                // 2. transmit GEMM share; two accumulators keep the MFMA chain short
                {
                    floatx4 acc0 = {0.f, 0.f, 0.f, 0.f}, acc1 = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
                    for (int k = 0; k < KW / 4; ++k) {
                        const int nn = nbase + 4 * k + gk;
                        const float2 gv = s_G[gi * GS + nn];
                        const float2 wk = (nn < A.M) ? s_W[(ct * 16 + gi) * WS + nn / A.nu]
                                                     : make_float2(0.f, 0.f);
                        // re: Gr Wr - Gi Wi ; im: Gr Wi + Gi Wr
                        const float b0 = out_im ? wk.y : wk.x;
                        const float b1 = out_im ? wk.x : -wk.y;
                        if (k & 1) {
                            acc1 = __builtin_amdgcn_mfma_f32_16x16x4f32(gv.x, b0, acc1, 0, 0, 0);
                            acc1 = __builtin_amdgcn_mfma_f32_16x16x4f32(gv.y, b1, acc1, 0, 0, 0);
                        } else {
                            acc0 = __builtin_amdgcn_mfma_f32_16x16x4f32(gv.x, b0, acc0, 0, 0, 0);
                            acc0 = __builtin_amdgcn_mfma_f32_16x16x4f32(gv.y, b1, acc0, 0, 0, 0);
                        }
                    }
                    // D[row][col]: col = lane % 16, row = 4 (lane / 16) + v
#pragma unroll
                    for (int v = 0; v < 4; ++v)
                        s_part[wave][(4 * (lane >> 4) + v) * 16 + (lane & 15)] = acc0[v] + acc1[v];
                }
                __syncthreads();
                // 3. sum the shares (fixed order), scale by R_s
                for (int idx = tid; idx < SCH * TPG; idx += NB) {
                    const int s = idx / TPG, t = idx % TPG;
                    const int c_tile = t >> 4, col = t & 15;
                    float re = 0.f, im = 0.f;
#pragma unroll
                    for (int kp = 0; kp < KSPLIT; ++kp) {
                        re += s_part[kp * NOUT + 2 * c_tile][s * 16 + col];
                        im += s_part[kp * NOUT + 2 * c_tile + 1][s * 16 + col];
                    }
                    const float R = s_sc[s].w;
                    s_c[s][t] = make_float2(R * re, R * im);
                }
                __syncthreads();
                // 4. receive GEMM: X[e][t] += sum_s Ge[e][s] c[s][t], rows e = mt_e + lane % 16
                if (re_live) {
                    const int e = mt_e + gi;
#pragma unroll
                    for (int k = 0; k < SCH / 4; ++k) {
                        const int s = 4 * k + gk;
                        float2 ge = make_float2(0.f, 0.f);
                        if (e < A.N)
                            for (int mu = 0; mu < A.nu; ++mu) {
                                const float2 v = s_G[s * GS + e * A.nu + mu];
                                ge.x += v.x;
                                ge.y += v.y;
                            }
#pragma unroll
                        for (int c = 0; c < NTP; ++c) {
                            const float2 cv = s_c[s][c * 16 + gi];
                            // re: Ger cr - Gei ci ; im: Ger ci + Gei cr
                            X[jj][c][0] = __builtin_amdgcn_mfma_f32_16x16x4f32(ge.x, cv.x, X[jj][c][0], 0, 0, 0);
                            X[jj][c][0] = __builtin_amdgcn_mfma_f32_16x16x4f32(ge.y, -cv.y, X[jj][c][0], 0, 0, 0);
                            X[jj][c][1] = __builtin_amdgcn_mfma_f32_16x16x4f32(ge.x, cv.y, X[jj][c][1], 0, 0, 0);
                            X[jj][c][1] = __builtin_amdgcn_mfma_f32_16x16x4f32(ge.y, cv.x, X[jj][c][1], 0, 0, 0);
                        }
                    }
                }
                __syncthreads();
            }
        }
        // per-element partials [item][JT][TPG][N]; D[row][col]: row = element
        // mt_e + 4 (lane / 16) + v, col = transmit c * 16 + lane % 16
        if (re_live) {
            float2* out = A.part + (int64_t)item * JT * TPG * A.N;
#pragma unroll
            for (int jj = 0; jj < JT; ++jj)
#pragma unroll
                for (int c = 0; c < NTP; ++c)
#pragma unroll
                    for (int v = 0; v < 4; ++v) {
                        const int e = mt_e + 4 * (lane >> 4) + v;
                        const int t = c * 16 + (lane & 15);
                        if (e < A.N)
                            out[((int64_t)jj * TPG + t) * A.N + e] = make_float2(X[jj][c][0][v], X[jj][c][1][v]);
                    }
        }

        if (!PERSIST) break;
        __syncthreads();
        if (tid == 0) s_item = atomicAdd(A.ticket, 1);
        __syncthreads();
        item = s_item;
    }
}

template <int NTP, int NQ, bool PERSIST>
static SynthKernel mt_kernel_p(const SynthConfig& c)
{
    constexpr int JT = NTP == 1 ? 4 : 2;   // receive accumulators: 16 JT NTP floats
    if (c.jt != JT) return nullptr;
    if (c.has_y) return k_synth_mt<NTP, NQ, JT, true, false, PERSIST>;
    if (c.table) return k_synth_mt<NTP, NQ, JT, false, true, PERSIST>;
    return k_synth_mt<NTP, NQ, JT, false, false, PERSIST>;
}

template <int NTP, int NQ>
static SynthKernel mt_kernel_nq(const SynthConfig& c)
{
    return c.persistent ? mt_kernel_p<NTP, NQ, true>(c) : mt_kernel_p<NTP, NQ, false>(c);
}

// The matrix-core path serves n_tx >= 4 with nu N <= 256 and N <= 128.
bool mt_supported(int M, int N, int n_tx) { return n_tx >= 4 && M <= 256 && N <= 128; }

SynthConfig mt_config(int M, int N, int n_tx, bool has_y)
{
    SynthConfig c{};
    c.bs = 512;
    c.tt = n_tx > 16 ? 32 : 16;               // transmits per group
    int np = 64;
    while (np < N) np *= 2;                   // element slots
    const int nq = 512 / np;
    c.jt = c.tt == 16 ? 4 : 2;
    c.sc = 16;
    c.has_y = has_y;
    c.mfma = true;
    c.nq = nq;
    (void)M;
    return c;
}

SynthKernel synth_mt_kernel(const SynthConfig& c)
{
    const int ntp = c.tt / 16;
    if (ntp == 1) {
        switch (c.nq) {
        case 4: return mt_kernel_nq<1, 4>(c);
        case 8: return mt_kernel_nq<1, 8>(c);
        default: return nullptr;
        }
    }
    if (ntp == 2) {
        switch (c.nq) {
        case 4: return mt_kernel_nq<2, 4>(c);
        case 8: return mt_kernel_nq<2, 8>(c);
        default: return nullptr;
        }
    }
    return nullptr;
}

hipError_t launch_synth_mt(const SynthConfig& c, const SynthArgs& a, hipStream_t st)
{
    if (c.grid <= 0) return hipSuccess;
    if (c.persistent != (a.ticket != nullptr)) return hipErrorInvalidValue;
    const SynthKernel k = synth_mt_kernel(c);
    if (!k) return hipErrorInvalidValue;
    SynthArgs arg = a;
    void* args[] = {&arg};
    return hipLaunchKernel(reinterpret_cast<const void*>(k), dim3(c.grid), dim3(512), args, 0, st);
}

}  // namespace simus
