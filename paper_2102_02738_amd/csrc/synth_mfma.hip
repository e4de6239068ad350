// Synthesis for many transmits on the matrix cores.  The weight of Eq. (29)
// is the same for the nu sub-elements of an element, so with the element
// sums B[e][s] = sum_{mu in e} G[s][mu] both contractions run over elements:
// per chunk of 16 scatterers and per bin, the transmit contraction
//   a[s][t] = sum_e B[e][s] W[e][t]      (16 x N x 16-32 transmits)
// and the receive contraction of Eqs. (32)-(33)
//   X[e][t] += sum_s B[e][s] R_s a[s][t]  (elements x 16 x transmits)
// are complex GEMMs run with FP32 MFMA (16x16x4).  Each complex product
// takes three real products (Karatsuba): with P1 = Re Re, P2 = Im Im and
// P3 = (Re + Im)(Re + Im) summed over k, the product is (P1 - P2, P3 - P1 - P2).
// The Green's terms are synthesised on the VALU (green.hpp) and stepped
// across the item's bins; X accumulates in registers across the item's
// scatterers, as the three sums, and is combined once at the end.
//
// Block: 512 threads (8 waves), nu in {1, 2} at compile time.
//   Synthesis: thread = (sub-element n, group of PPT scatterers).  Writes the
//     element sums B (for nu = 2 one DPP exchange between the two
//     sub-elements of an element, which are neighbouring lanes).
//   Transmit GEMM: wave = (column tile ct of 16 transmits, share kp of the
//     elements); its three product tiles go to LDS and are summed over the
//     shares in a fixed order, scaled by R_s, into c[s][t].
//   Receive GEMM: wave w owns elements 16 w .. 16 w + 15 and all column tiles.
// The steps are software-pipelined over the item's (chunk, bin) sequence with
// two barriers per bin: [reduction of the previous bin, synthesis] and
// [receive GEMM of the previous bin, transmit GEMM]; the element sums are
// double-buffered by bin.  Partial spectra of every item, per element, go to `part`
// ([item][JT][TPG][N]); like the vector path the terms are j G, and the
// finaliser divides by j^2.
#include <hip/hip_runtime.h>

#include <algorithm>

#include "green.hpp"
#include "kernels.hpp"

namespace simus {


// Receive sums of the eight-bin kernel with 128 element slots: (Re, Im)
// pairs.  The three-product form needs 24 more registers per lane and then
// spills (29 dwords): 16 transmits x 11 items of 4 uneven phantoms, quarter
// size, 329 vs 312 ms.  With 64 slots the three products fit (155 VGPRs):
// 64-element phased array, 16 transmits, 40k scatterers 5.20 vs 5.66 ms.
#ifndef MQ_NX
#define MQ_NX 2
#endif
constexpr int MQ_NX64 = 3;

__device__ __forceinline__ floatx4 mfma4(float a, float b, floatx4 c)
{
    return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
}

template <int NE, int NTP, int JT, int NUV, int NX, bool HASY, bool TABLE>
__global__ __launch_bounds__(512) void k_synth_mt(SynthArgs A)
{
    constexpr int NB = 512;
    constexpr int MS = NE * NUV;            // sub-element slots (NE: element slots)
    constexpr int SCH = 16;                 // scatterers per chunk (MFMA rows)
    constexpr int PPT = SCH * MS / NB;      // pairs per synthesis thread
    constexpr int NSG = NB / MS;            // scatterer groups
    constexpr int BST = NE + 2;             // row stride of the element sums
    constexpr int TPG = 16 * NTP;           // transmit columns of the group
    constexpr int KP = 8 / NTP;             // element shares per column tile
    constexpr int KW = NE / KP;             // elements per wave
    constexpr int KS = KW / 4;              // transmit-GEMM k-steps per wave
    constexpr int WS = NE + 2;              // row stride of the staged weights
    constexpr int RXE = NE / 16;            // receive element tiles
    constexpr int CS = 8 / RXE;             // waves per element tile (column split)
    constexpr int CPW = NTP / CS;           // receive column tiles per wave
    static_assert(NE == 64 || NE == 128, "64 or 128 element slots");
    static_assert(CPW * CS == NTP && KP * NTP == 8, "waves must cover the GEMMs");
    static_assert(NUV == 1 || NUV == 2, "nu must be 1 or 2");
    static_assert(NX == 2 || NX == 3, "receive sums: (Re, Im) or three products");
    static_assert(PPT * NSG == SCH, "synthesis threads must cover the chunk");
    static_assert(JT % 2 == 0, "the element sums alternate between two buffers by bin");
    constexpr int NRED = (SCH * TPG + NB - 1) / NB;     // reduction outputs per thread
    // LDS layouts free of bank conflicts (64 banks of 4 bytes; a wave's 8-byte
    // accesses are served 32 lanes at a time, its 4-byte ones 64):
    //  - element sums and weights with rows NE + 2 apart, for the transmit
    //    GEMM (lanes: 16 rows, 2 columns; the receive GEMM's reads of the sums,
    //    16 columns by 2 rows, meet 2-way conflicts: a swizzle that also
    //    serves them costs registers for per-step addresses);
    //  - product tiles per lane with register v rows PV apart and waves PB
    //    apart, so that the share sums read 64 distinct banks;
    //  - scaled sums c with rows CST = 16 (mod 32) apart (lanes: 16 columns,
    //    2 rows).
    constexpr int PV = 80;
    constexpr int PS = 4 * PV;              // stride of a product
    constexpr int PB = 3 * PS + (NTP == 2 ? 32 : NTP == 4 ? 16 : 0);
    constexpr int CST = TPG % 32 == 16 ? TPG : TPG + 16;

    __shared__ float4 s_sc[SCH];
    __shared__ float2 s_B[2 * SCH * BST];   // element sums, two buffers
    __shared__ float2 s_W[TPG * WS];
    __shared__ float s_part[8 * PB];
    __shared__ float2 s_c[SCH * CST];
    __shared__ float4 s_tab[TABLE ? 2 * DELTA_NT : 1];

    const int tid = threadIdx.x;
    const int wave = tid >> 6, lane = tid & 63;
    const int gi = lane & 15, gk = lane >> 4;      // MFMA operand lane roles
    // synthesis role
    const int n = tid % MS, sh = tid / MS;
    const bool active = n < A.M;
    const SubFrame fr = load_frame(A.sub, active ? n : 0);
    // transmit-GEMM role
    const int ct = wave % NTP, kp = wave / NTP;
    // receive-GEMM role: element tile, and the first of its CPW column tiles
    const int mt_e = (wave % RXE) * 16;
    const int rc0 = (wave / RXE) * CPW;
    const bool re_live = mt_e < A.N;

    DeltaParams P{};
    if (TABLE) {
        for (int i = tid; i < 2 * DELTA_NT; i += NB) s_tab[i] = A.dtab[i];
        P = *A.dpar;
    }

    // Persistent launch: blocks draw items from a work counter until it passes
    // n_items (every block exits).
    __shared__ int s_item;
    if (tid == 0) s_item = atomicAdd(A.ticket, 1);
    __syncthreads();
    int item = s_item;
    while (item < A.n_items) {
        const int id = A.order[item];          // costliest first
        const Item it = A.items[id];
        const int bt = it.tile & 0xffff, tg = it.tile >> 16;
        const int jb0 = bt * JT;
        const int nb = min(JT, A.n_bins - jb0);
        const int t0 = tg * TPG;

        // receive sums [bin][column tile of the wave]: (Re, Im), or the three
        // products
        floatx4 X[JT][CPW][NX];
#pragma unroll
        for (int jj = 0; jj < JT; ++jj)
#pragma unroll
            for (int c = 0; c < CPW; ++c)
#pragma unroll
                for (int q = 0; q < NX; ++q) X[jj][c][q] = floatx4{0.f, 0.f, 0.f, 0.f};

        // 3. the partial products of a bin -> c[s][t] = R_s (sum over the
        //    element shares, in a fixed order, of the three products combined)
        auto reduce = [&](const float (&R)[NRED]) {
#pragma unroll
            for (int q = 0; q < NRED; ++q) {
                const int idx = tid + q * NB;
                if (idx < SCH * TPG) {
                    const int s = idx / TPG, t = idx % TPG;
                    // row s of a tile = 4 (lane / 16) + v of the wave that wrote it
                    const int c = t >> 4, d = (s & 3) * PV + (s >> 2) * 16 + (t & 15);
                    float q1 = 0.f, q2 = 0.f, q3 = 0.f;
#pragma unroll
                    for (int k = 0; k < KP; ++k) {
                        const float* sp = s_part + (k * NTP + c) * PB + d;
                        q1 += sp[0];
                        q2 += sp[PS];
                        q3 += sp[2 * PS];
                    }
                    s_c[s * CST + t] = make_float2(R[q] * (q1 - q2), R[q] * (q3 - q1 - q2));
                }
            }
        };
        // 4. receive GEMM of a bin: Xj[e][t] += sum_s B[e][s] c[s][t], rows
        //    e = mt_e + gi, columns of tiles rc0 ..., k = scatterer 4 k + gk
        auto rgemm = [&](floatx4 (&Xj)[CPW][NX], const float2* sBp) {
            if (!re_live) return;
            float2 ba[SCH / 4], ca[SCH / 4][CPW];
#pragma unroll
            for (int k = 0; k < SCH / 4; ++k) {
                const int s = 4 * k + gk;
                ba[k] = sBp[s * BST + mt_e + gi];
#pragma unroll
                for (int c = 0; c < CPW; ++c) ca[k][c] = s_c[s * CST + (rc0 + c) * 16 + gi];
            }
#pragma unroll
            for (int k = 0; k < SCH / 4; ++k)
#pragma unroll
                for (int c = 0; c < CPW; ++c) {
                    if (NX == 3) {
                        Xj[c][0] = mfma4(ba[k].x, ca[k][c].x, Xj[c][0]);
                        Xj[c][1] = mfma4(ba[k].y, ca[k][c].y, Xj[c][1]);
                        Xj[c][NX - 1] = mfma4(ba[k].x + ba[k].y, ca[k][c].x + ca[k][c].y, Xj[c][NX - 1]);
                    } else {
                        // Re += Br cr - Bi ci, Im += Br ci + Bi cr
                        Xj[c][0] = mfma4(ba[k].x, ca[k][c].x, Xj[c][0]);
                        Xj[c][0] = mfma4(-ba[k].y, ca[k][c].y, Xj[c][0]);
                        Xj[c][1] = mfma4(ba[k].x, ca[k][c].y, Xj[c][1]);
                        Xj[c][1] = mfma4(ba[k].y, ca[k][c].x, Xj[c][1]);
                    }
                }
        };

        // Software pipeline over the item's (chunk, bin) sequence, two barriers
        // per bin:
        //   A: reduce the previous bin (3); synthesise this bin's element
        //      sums (1) and stage its weights;
        //   B: the previous bin's receive GEMM (4); this bin's transmit GEMM (2).
        // The element sums alternate between two buffers by bin (JT is even, so
        // a chunk's first bin follows the previous chunk's last in the other
        // one).  Every chunk runs all JT bins; bins past n_bins are computed
        // (weights of the last bin) but not written.
        bool prev = false;                     // uniform: a bin awaits steps 3-4
        float Rc[NRED], Rp[NRED];              // R_s of the reduction rows: this chunk, previous
#pragma unroll
        for (int q = 0; q < NRED; ++q) Rc[q] = Rp[q] = 0.f;
        for (int s0 = it.s_begin; s0 < it.s_end; s0 += SCH) {
            if (tid < SCH) {
                const int s = s0 + tid;
                float4 v = make_float4(0.f, 0.f, 1.f, 0.f);     // padding: R = 0
                if (s < it.s_end) v = make_float4(A.x[s], HASY ? A.y[s] : 0.f, A.z[s], A.refl[s]);
                s_sc[tid] = v;
            }
            __syncthreads();
#pragma unroll
            for (int q = 0; q < NRED; ++q) {
                const int idx = tid + q * NB;
                Rp[q] = Rc[q];
                Rc[q] = idx < SCH * TPG ? s_sc[idx / TPG].w : 0.f;
            }
            Geo g[PPT];
#pragma unroll
            for (int k = 0; k < PPT; ++k) {
                const float4 v = s_sc[sh * PPT + k];
                g[k] = make_geo<HASY, true>(A.K, fr, v.x, v.y, v.z, A.j_lo + jb0);
                if (!active) g[k].E = make_float2(0.f, 0.f);
                if (TABLE) g[k].kap *= P.kscale;          // delta_fetch's argument
            }
            // The bin loop is unrolled so that the receive sums X[jj] stay in
            // registers.
#pragma unroll
            for (int jj = 0; jj < JT; ++jj) {
                const int jb = min(jb0 + jj, A.n_bins - 1);
                const float jf = (float)(A.j_lo + jb0 + jj);
                float2* sB = s_B + (jj & 1) * (SCH * BST);
                // ---- segment A
                // 0. transmit weights of this bin, W[t][e], zero outside N x n_tx.
                //    With 16 columns they are loaded here and stored to LDS after
                //    the synthesis, which hides the loads' latency; with 32 the
                //    registers are short and they are stored at once.
                constexpr int NW = TPG * NE / NB;
                constexpr bool HOIST = NW <= 4;
                auto w_at = [&](int idx) {
                    const int t = idx / NE, e = idx % NE;
                    const int tt = min(t0 + t, A.n_tx - 1), ee = min(e, A.N - 1);
                    const float2 w = A.W[((int64_t)jb * A.n_tx + tt) * A.N + ee];
                    const bool use = e < A.N && t0 + t < A.n_tx;
                    return make_float2(use ? w.x : 0.f, use ? w.y : 0.f);
                };
                float2 wv[HOIST ? NW : 1];
                if (HOIST) {
#pragma unroll
                    for (int q = 0; q < NW; ++q) wv[q] = w_at(tid + q * NB);
                } else {
                    // batches of four loads, so that a bin pays the load
                    // latency twice rather than once per weight
                    static_assert(NW % 4 == 0, "weights staged in batches of four");
#pragma unroll 1
                    for (int q0 = 0; q0 < NW; q0 += 4) {
                        float2 wq[4];
#pragma unroll
                        for (int q = 0; q < 4; ++q) wq[q] = w_at(tid + (q0 + q) * NB);
#pragma unroll
                        for (int q = 0; q < 4; ++q) {
                            const int idx = tid + (q0 + q) * NB;
                            s_W[(idx / NE) * WS + idx % NE] = wq[q];
                        }
                    }
                }
                if (prev) reduce(jj == 0 ? Rp : Rc);
                // 1. j G of the chunk -> element sums B[s][e]
                float2 G[PPT];
                if constexpr (TABLE) {
                    // each term's table read is issued while the previous term
                    // is evaluated
                    DeltaFetch fch[2];
                    fch[0] = delta_fetch(s_tab, P, jf * g[0].kap);
#pragma unroll
                    for (int k = 0; k < PPT; ++k) {
                        if (k + 1 < PPT) fch[(k + 1) & 1] = delta_fetch(s_tab, P, jf * g[k + 1].kap);
                        __builtin_amdgcn_sched_barrier(0);
                        G[k] = green_next_fetched(g[k], fch[k & 1]);
                    }
                } else {
#pragma unroll
                    for (int k = 0; k < PPT; ++k) G[k] = green_next<HASY, TABLE>(A.K, g[k], jf, 1.f, s_tab, P);
                }
#pragma unroll
                for (int k = 0; k < PPT; ++k) {
                    const int s = sh * PPT + k;
                    if (NUV == 2) {
                        // both lanes of the pair store the same sum (no extra LDS cost)
                        const float bx = G[k].x + __int_as_float(__builtin_amdgcn_mov_dpp(
                                                      __float_as_int(G[k].x), 0xB1, 0xF, 0xF, true));
                        const float by = G[k].y + __int_as_float(__builtin_amdgcn_mov_dpp(
                                                      __float_as_int(G[k].y), 0xB1, 0xF, 0xF, true));
                        sB[s * BST + (n >> 1)] = make_float2(bx, by);
                    } else {
                        sB[s * BST + n] = G[k];
                    }
                }
                if (HOIST) {
#pragma unroll
                    for (int q = 0; q < NW; ++q) {
                        const int idx = tid + q * NB;
                        s_W[(idx / NE) * WS + idx % NE] = wv[q];
                    }
                }
                __syncthreads();
                // ---- segment B
                if (prev) rgemm(X[(jj + JT - 1) % JT], s_B + ((jj + 1) & 1) * (SCH * BST));
                // 2. transmit GEMM share: rows s = gi, columns t = ct 16 + gi,
                //    elements kp KW + 4 k + gk
                {
                    const float2* gp = sB + gi * BST + kp * KW + gk;
                    const float2* wp = s_W + (ct * 16 + gi) * WS + kp * KW + gk;
                    // operands loaded in batches of KB k-steps ahead of their MFMAs
                    constexpr int KB = KS > 8 ? 8 : KS;
                    floatx4 p1 = {0.f, 0.f, 0.f, 0.f}, p2 = p1, p3 = p1;
#pragma unroll
                    for (int k0 = 0; k0 < KS; k0 += KB) {
                        float2 ga[KB], wa[KB];
#pragma unroll
                        for (int k = 0; k < KB; ++k) {
                            ga[k] = gp[4 * (k0 + k)];
                            wa[k] = wp[4 * (k0 + k)];
                        }
#pragma unroll
                        for (int k = 0; k < KB; ++k) {
                            p1 = mfma4(ga[k].x, wa[k].x, p1);
                            p2 = mfma4(ga[k].y, wa[k].y, p2);
                            p3 = mfma4(ga[k].x + ga[k].y, wa[k].x + wa[k].y, p3);
                        }
                        __builtin_amdgcn_sched_barrier(0);
                    }
                    // D[row][col]: col = lane % 16, row = 4 (lane / 16) + v
#pragma unroll
                    for (int v = 0; v < 4; ++v) {
                        float* sp = s_part + wave * PB + v * PV + lane;
                        sp[0] = p1[v];
                        sp[PS] = p2[v];
                        sp[2 * PS] = p3[v];
                    }
                }
                __syncthreads();
                prev = true;
            }
        }
        if (prev) {     // steps 3-4 of the item's last bin
            reduce(Rc);
            __syncthreads();
            rgemm(X[JT - 1], s_B + ((JT - 1) & 1) * (SCH * BST));
        }
        // per-element partials [item][JT][TPG][N]; D[row][col]: row = element
        // mt_e + 4 (lane / 16) + v, col = transmit (rc0 + c) 16 + lane % 16
        if (re_live) {
            float2* out = A.part + (int64_t)id * JT * TPG * A.N;
#pragma unroll
            for (int jj = 0; jj < JT; ++jj)
#pragma unroll
                for (int c = 0; c < CPW; ++c)
#pragma unroll
                    for (int v = 0; v < 4; ++v) {
                        const int e = mt_e + 4 * gk + v;
                        const int t = (rc0 + c) * 16 + gi;
                        const float x1 = X[jj][c][0][v], x2 = X[jj][c][1][v], x3 = X[jj][c][NX - 1][v];
                        const float2 xv = NX == 3 ? make_float2(x1 - x2, x3 - x1 - x2) : make_float2(x1, x2);
                        if (e < A.N && jj < nb) out[((int64_t)jj * TPG + t) * A.N + e] = xv;
                    }
        }

        __syncthreads();
        if (tid == 0) s_item = atomicAdd(A.ticket, 1);
        __syncthreads();
        item = s_item;
    }
}


// One group of 16 transmit columns and 128 or 64 element slots, eight bins
// per item, two per SIMD: wave w (waves w and w ^ 4 share SIMD w % 4) runs
// the transmit GEMM of bin w and the receive GEMM of bin w ^ 4.  Per chunk
// of 16 scatterers:
//   P1  every thread sets up its pairs once and synthesises the element sums
//       of all eight bins into LDS;
//   P2  every wave: transmit GEMM of its bin over all elements (three real
//       products per complex product, no reduction over waves), the weights
//       read from the padded table WT in global memory a batch of k-steps
//       ahead; c = R_s a to LDS;
//   P3  every wave: receive GEMM of its other bin, X[e][t] += sum_s B[e][s]
//       c[s][t] over all elements, in its registers; wave 0 loads the next
//       chunk's scatterers meanwhile.
// Three barriers per chunk of eight bins, and each pair is set up once per
// eight bins.
template <int NE, int NUV, int NX, bool HASY, bool TABLE>
__global__ __launch_bounds__(512) void k_synth_mq(SynthArgs A)
{
    constexpr int NB = 512;
    constexpr int MS = NE * NUV;            // sub-element slots
    constexpr int SCH = 16;                 // scatterers per chunk (MFMA rows)
    constexpr int PPT = SCH * MS / NB;      // pairs per synthesis thread
    constexpr int NSG = NB / MS;            // scatterer groups
    constexpr int JT = 8;                   // bins per item: two per SIMD
    constexpr int TPG = 16;                 // transmit columns
    constexpr int BST = NE + 2;             // row stride of the element sums
    constexpr int CST = 16;                 // row stride of c[s][t]
    constexpr int KS = NE / 4;              // transmit-GEMM k-steps (all elements)
    constexpr int KB = 8;                   // k-steps of weights loaded ahead
    constexpr int RXE = NE / 16;            // receive element tiles
    static_assert(NE == 64 || NE == 128, "64 or 128 element slots");
    static_assert(NUV == 1 || NUV == 2, "nu must be 1 or 2");
    static_assert(NX == 2 || NX == 3, "receive sums: (Re, Im) or three products");
    static_assert(PPT * NSG == SCH && KS % KB == 0, "threads must cover the chunk");

    __shared__ float4 s_sc[SCH];
    __shared__ float2 s_B[JT][SCH * BST];
    __shared__ float2 s_c[JT][SCH * CST];
    __shared__ float4 s_tab[TABLE ? 2 * DELTA_NT : 1];
    __shared__ int s_item;

    const int tid = threadIdx.x;
    const int wave = tid >> 6, lane = tid & 63;
    const int gi = lane & 15, gk = lane >> 4;      // MFMA operand lane roles
    const int btx = wave, brx = wave ^ 4;          // the wave's transmit and receive bins
    // synthesis role
    const int n = tid % MS, sh = tid / MS;
    const bool active = n < A.M;
    const SubFrame fr = load_frame(A.sub, active ? n : 0);
    const int n_tg = (A.n_tx + TPG - 1) / TPG;

    DeltaParams P{};
    if (TABLE) {
        for (int i = tid; i < 2 * DELTA_NT; i += NB) s_tab[i] = A.dtab[i];
        P = *A.dpar;
    }

    auto load_chunk = [&](int s0, int s_end) {
        if (tid < SCH) {
            const int s = s0 + tid;
            float4 v = make_float4(0.f, 0.f, 1.f, 0.f);     // padding: R = 0
            if (s < s_end) v = make_float4(A.x[s], HASY ? A.y[s] : 0.f, A.z[s], A.refl[s]);
            s_sc[tid] = v;
        }
    };

    if (tid == 0) s_item = atomicAdd(A.ticket, 1);
    __syncthreads();
    int item = s_item;
    while (item < A.n_items) {
        const int id = A.order[item];          // costliest first
        const Item it = A.items[id];
        const int bt = it.tile & 0xffff, tg = it.tile >> 16;
        const int jb0 = bt * JT;
        const int nb = min(JT, A.n_bins - jb0);
        // this wave's weights: WT[bin][tg][e = 4 k + gk][t = gi], k-step stride 64
        const int jbw = min(jb0 + btx, A.n_bins - 1);
        const float2* wg = A.WT + (((int64_t)jbw * n_tg + tg) * NE + gk) * TPG + gi;

        // receive sums of the wave's receive bin: element tiles x ((Re, Im)
        // or the three products)
        floatx4 X[RXE][NX];
#pragma unroll
        for (int m = 0; m < RXE; ++m)
#pragma unroll
            for (int q = 0; q < NX; ++q) X[m][q] = floatx4{0.f, 0.f, 0.f, 0.f};

        load_chunk(it.s_begin, it.s_end);
        __syncthreads();
        for (int s0 = it.s_begin; s0 < it.s_end; s0 += SCH) {
            // ---- P1: set-up, the element sums of the eight bins
            {
                Geo g[PPT];
#pragma unroll
                for (int k = 0; k < PPT; ++k) {
                    const float4 v = s_sc[sh * PPT + k];
                    g[k] = make_geo<HASY, true>(A.K, fr, v.x, v.y, v.z, A.j_lo + jb0);
                    if (!active) g[k].E = make_float2(0.f, 0.f);
                    if (TABLE) g[k].kap *= P.kscale;          // delta_fetch's argument
                }
#pragma unroll 1
                for (int jj = 0; jj < JT; ++jj) {
                    prio_by_progress(jj, JT);
                    const float jf = (float)(A.j_lo + jb0 + jj);
                    float2 G[PPT];
                    if constexpr (TABLE) {
                        DeltaFetch fch[2];
                        fch[0] = delta_fetch(s_tab, P, jf * g[0].kap);
#pragma unroll
                        for (int k = 0; k < PPT; ++k) {
                            if (k + 1 < PPT) fch[(k + 1) & 1] = delta_fetch(s_tab, P, jf * g[k + 1].kap);
                            __builtin_amdgcn_sched_barrier(0);
                            G[k] = green_next_fetched(g[k], fch[k & 1]);
                        }
                    } else {
#pragma unroll
                        for (int k = 0; k < PPT; ++k) G[k] = green_next<HASY, TABLE>(A.K, g[k], jf, 1.f, s_tab, P);
                    }
                    float2* sB = s_B[jj];
#pragma unroll
                    for (int k = 0; k < PPT; ++k) {
                        const int s = sh * PPT + k;
                        if (NUV == 2) {
                            // both lanes of the pair store the same sum
                            const float bx = G[k].x + __int_as_float(__builtin_amdgcn_mov_dpp(
                                                          __float_as_int(G[k].x), 0xB1, 0xF, 0xF, true));
                            const float by = G[k].y + __int_as_float(__builtin_amdgcn_mov_dpp(
                                                          __float_as_int(G[k].y), 0xB1, 0xF, 0xF, true));
                            sB[s * BST + (n >> 1)] = make_float2(bx, by);
                        } else {
                            sB[s * BST + n] = G[k];
                        }
                    }
                }
            }
            __builtin_amdgcn_s_setprio(0);
            // the first batch of weights, in flight across the barrier
            float2 wa[2][KB];
#pragma unroll
            for (int k = 0; k < KB; ++k) wa[0][k] = wg[64 * k];
            __syncthreads();
            // ---- P2: transmit GEMM of bin btx: rows s = gi, columns t = gi,
            //      k = element 4 k + gk
            {
                const float2* gp = s_B[btx] + gi * BST + gk;
                floatx4 p1 = {0.f, 0.f, 0.f, 0.f}, p2 = p1, p3 = p1;
#pragma unroll
                for (int k0 = 0; k0 < KS; k0 += KB) {
                    const int cur = (k0 / KB) & 1;
                    if (k0 + KB < KS) {
#pragma unroll
                        for (int k = 0; k < KB; ++k) wa[cur ^ 1][k] = wg[64 * (k0 + KB + k)];
                    }
                    float2 ga[KB];
#pragma unroll
                    for (int k = 0; k < KB; ++k) ga[k] = gp[4 * (k0 + k)];
#pragma unroll
                    for (int k = 0; k < KB; ++k) {
                        p1 = mfma4(ga[k].x, wa[cur][k].x, p1);
                        p2 = mfma4(ga[k].y, wa[cur][k].y, p2);
                        p3 = mfma4(ga[k].x + ga[k].y, wa[cur][k].x + wa[cur][k].y, p3);
                    }
                }
                // D[row][col]: row s = 4 gk + v, col t = gi; c = R_s a
                float2* sc = s_c[btx];
#pragma unroll
                for (int v = 0; v < 4; ++v) {
                    const int s = 4 * gk + v;
                    const float R = s_sc[s].w;
                    sc[s * CST + gi] = make_float2(R * (p1[v] - p2[v]), R * (p3[v] - p1[v] - p2[v]));
                }
            }
            __syncthreads();
            // ---- P3: receive GEMM of bin brx; the next chunk's scatterers
            {
                const float2* cb = s_c[brx];
                const float2* bb = s_B[brx];
                float2 ca[SCH / 4];
#pragma unroll
                for (int k = 0; k < SCH / 4; ++k) ca[k] = cb[(4 * k + gk) * CST + gi];
#pragma unroll
                for (int m = 0; m < RXE; ++m) {
                    float2 ba[SCH / 4];
#pragma unroll
                    for (int k = 0; k < SCH / 4; ++k) ba[k] = bb[(4 * k + gk) * BST + 16 * m + gi];
#pragma unroll
                    for (int k = 0; k < SCH / 4; ++k) {
                        if (NX == 3) {
                            X[m][0] = mfma4(ba[k].x, ca[k].x, X[m][0]);
                            X[m][1] = mfma4(ba[k].y, ca[k].y, X[m][1]);
                            X[m][2] = mfma4(ba[k].x + ba[k].y, ca[k].x + ca[k].y, X[m][2]);
                        } else {
                            X[m][0] = mfma4(ba[k].x, ca[k].x, X[m][0]);
                            X[m][0] = mfma4(-ba[k].y, ca[k].y, X[m][0]);
                            X[m][1] = mfma4(ba[k].x, ca[k].y, X[m][1]);
                            X[m][1] = mfma4(ba[k].y, ca[k].x, X[m][1]);
                        }
                    }
                }
            }
            if (s0 + SCH < it.s_end) load_chunk(s0 + SCH, it.s_end);
            __syncthreads();
        }
        // per-element partials [item][JT][TPG][N] of the wave's receive bin;
        // D[row][col]: row = element 16 m + 4 gk + v, col = transmit gi
        if (brx < nb) {
            float2* out = A.part + ((int64_t)id * JT + brx) * TPG * A.N;
#pragma unroll
            for (int m = 0; m < RXE; ++m)
#pragma unroll
                for (int v = 0; v < 4; ++v) {
                    const int e = 16 * m + 4 * gk + v;
                    const float x1 = X[m][0][v], x2 = X[m][1][v], x3 = X[m][NX - 1][v];
                    const float2 xv = NX == 3 ? make_float2(x1 - x2, x3 - x1 - x2) : make_float2(x1, x2);
                    if (e < A.N) out[(int64_t)gi * A.N + e] = xv;
                }
        }
        if (tid == 0) s_item = atomicAdd(A.ticket, 1);
        __syncthreads();
        item = s_item;
    }
}

// Shape of a group: element slots NE (64 or 128) and 16-transmit column
// tiles NTP; bins per item JT and receive sums NX are chosen so that the
// receive sums (4 NX JT NTP / CS floats per lane) fit the register file.
struct MtShape {
    int ne, ntp, jt, nx;
};

static MtShape mt_shape(int N, int n_tx, bool alt, bool fp32)
{
    // Default: the eight-bin kernel over groups of 16 transmit columns, 64 or
    // 128 element slots (products in split bf16, k_synth_mb; in FP32 with
    // SIMUS_FLAG_FP32_PRODUCTS, k_synth_mq).  Measured against the four- and
    // six-bin kernels (k_synth_mt), the alternative shape: curved array, 11
    // transmits, a quarter of the uneven 16-phantom batch 255 ms (bf16) / 312
    // (FP32) vs 398 with 4 bins; 5 plane waves, 100k scatterers 38.7 / 47.4
    // vs 62.0; 21 plane waves, 200k scatterers 161 / 197 vs 188 (32 columns,
    // 4 bins; 258 with 16 columns); 128 focused transmits on a 64-element
    // array, 40k scatterers 30.7 / 38.6 vs 40.7 (64 columns, 6 bins);
    // 64-element arrays with up to 16 transmits about half the time of 32
    // columns and 6 bins.
    // More than 16 transmits (split bf16): groups of 32 columns, four bins per
    // set-up (k_synth_mw), which synthesises G once per 32 transmits: 21
    // plane waves, 200k scatterers 112 vs 158 ms over two groups of 16; 128
    // focused transmits on 64 elements 19.8 vs 26.1 ms; 40 plane waves, 100k
    // scatterers 119 vs 122 ms.
    // More than 32 transmits on 64 element slots: groups of 64 columns, two
    // column tiles per wave (128 focused transmits on 64 elements 17.2 vs
    // 14.1 ms with groups of 32).
    if (!alt && n_tx > 32 && !fp32 && N <= 64) return {64, 4, 4, 2};
    if (!alt && n_tx > 16 && !fp32) return {N <= 64 ? 64 : 128, 2, 4, 2};
    if (!alt) return {N <= 64 ? 64 : 128, 1, 8, N <= 64 ? MQ_NX64 : MQ_NX};
    // the alternative, k_synth_mt: 64 element slots, 6 bins per item, groups
    // of 64 transmit columns where they pad no more than groups of 32 (40k
    // scatterers: 128 transmits 42.5 vs 44.7 ms with 32; 40 and 64 equal; 96
    // transmits 41.9 vs 32.5 ms, so 32 there); 128 slots, 4 bins per item (5
    // spill): 16 columns up to 16 transmits, else 32
    if (N <= 64) {
        const bool wide = (n_tx + 63) / 64 * 64 == (n_tx + 31) / 32 * 32;
        if (n_tx > 32 && wide) return {64, 4, 6, 2};
        return {64, 2, 6, 3};
    }
    if (n_tx <= 16) return {128, 1, 4, 3};
    return {128, 2, 4, 2};
}

template <int NE, int NTP, int JT, int NX, int NUV>
static SynthKernel mt_kernel_nuv(const SynthConfig& c)
{
    if (c.has_y) return k_synth_mt<NE, NTP, JT, NUV, NX, true, false>;
    if (c.table) return k_synth_mt<NE, NTP, JT, NUV, NX, false, true>;
    return k_synth_mt<NE, NTP, JT, NUV, NX, false, false>;
}

template <int NE, int NTP, int JT, int NX>
static SynthKernel mt_kernel_shape(const SynthConfig& c)
{
    if (c.jt != JT || c.nx != NX) return nullptr;
    return c.pair ? mt_kernel_nuv<NE, NTP, JT, NX, 2>(c) : mt_kernel_nuv<NE, NTP, JT, NX, 1>(c);
}

// The matrix-core path serves n_tx >= 4 with N <= 128 elements and nu in {1, 2}.
bool mt_supported(int M, int N, int n_tx)
{
    const int nu = N > 0 ? M / N : 0;
    return n_tx >= 4 && N >= 1 && N <= 128 && (nu == 1 || nu == 2) && M == nu * N;
}

SynthConfig mt_config(int M, int N, int n_tx, bool has_y, bool alt, bool fp32)
{
    const MtShape sh = mt_shape(N, n_tx, alt, fp32);
    SynthConfig c{};
    c.bs = 512;
    c.groups = 1;
    c.ne = sh.ne;
    c.tt = 16 * sh.ntp;                       // transmits per group
    c.jt = sh.jt;
    c.nx = sh.nx;
    // the kernels that read the padded weight table: eight bins over 16
    // columns (split bf16 or FP32 products), four bins over 32 (split bf16)
    c.wt = !alt;
    c.bf = c.wt && !fp32;
    c.sc = 16;
    c.pair = M == 2 * N;
    c.has_y = has_y;
    c.mfma = true;
    c.persistent = true;
    return c;
}

// The eight-bin kernel with its two GEMMs on bf16 matrix cores
// (v_mfma_f32_16x16x32_bf16, FP32 accumulation).  Every operand x is split
// into bf16 parts x = x_h + x_l (x_h = x rounded, x_l = x - x_h rounded), and
// a product takes three bf16 products, x_h y_h + x_h y_l + x_l y_h: the
// dropped x_l y_l and the rounding of x_l leave about 2^-16 of |x y|.  A
// complex value (re, im) is stored as two packed words, (re_h, im_h) and
// (re_l, im_l); a complex product's real part pairs (re, im) with (W_re,
// -W_im) and its imaginary part with (W_im, W_re) along k, so each MFMA
// contracts 16 complex values (K = 32):
//   P1  pair by pair (its set-up, then its eight bins with their table
//       fetches in flight together: 6 % faster than bin by bin over all
//       pairs), element sums, split, into two LDS planes per bin (h and l);
//       for nu = 2 a thread takes both sub-elements of an element;
//   P2  wave w, bin w: a[s][t] = sum_e B[s][e] W[e][t], 8 (NE = 128) or 4
//       k-steps of 16 elements, 6 MFMAs each; weights from the split table
//       WT[bin][group][t][e] (uint2: h, l); c = R_s a, split;
//   P3  wave w, bin w: X[e][t] += sum_s B[e][s] c[s][t], one k-step per
//       element tile (16 scatterers), 6 MFMAs.
// The transmit GEMM leaves c[s = 4 (lane / 16) + v][t = lane % 16] in the
// lane that takes it as the receive GEMM's B operand (k = scatterers 4
// (lane / 16) .. + 3, column lane % 16): with both GEMMs of a wave on one
// bin, c never leaves the registers, the two GEMMs need no barrier between
// them, and the next chunk's positions go to the other of two buffers: two
// barriers per chunk.  16 phantoms at a quarter of their scatterers: 235.9
// ms with c through LDS and three barriers, 232.4 with two, 230.0 with c in
// registers (results bit-identical).
// FP32 16x16x4 MFMAs contract 4 real values in 32 cycles, bf16 16x16x32 ones
// 32 in about 16-20; per complex product this takes 6 x 2 bf16 products
// instead of 3 (or 4) FP32 ones.

template <int NE, int NUV, bool HASY, bool TABLE>
__global__ __launch_bounds__(512) void k_synth_mb(SynthArgs A)
{
    constexpr int NB = 512;
    constexpr int MS = NE * NUV;            // sub-element slots
    constexpr int SCH = 16;                 // scatterers per chunk (MFMA rows)
    constexpr int PPT = SCH * MS / NB;      // pairs per synthesis thread
    constexpr int NSG = NB / MS;            // scatterer groups
    constexpr int JT = 8;                   // bins per item: two per SIMD
    constexpr int TPG = 16;                 // transmit columns
    constexpr int BPS = NE + 4;             // row stride (words) of the element-sum planes
    constexpr int KS = NE / 16;             // transmit-GEMM k-steps (16 elements each)
    constexpr int RXE = NE / 16;            // receive element tiles
    static_assert(NE == 64 || NE == 128, "64 or 128 element slots");
    static_assert(NUV == 1 || NUV == 2, "nu must be 1 or 2");
    static_assert(PPT * NSG == SCH, "threads must cover the chunk");

    __shared__ float4 s_sc[2][SCH];          // by chunk parity
    __shared__ __align__(16) uint32_t s_Bh[JT][SCH * BPS];
    __shared__ __align__(16) uint32_t s_Bl[JT][SCH * BPS];
    __shared__ float4 s_tab[TABLE ? 2 * DELTA_NT : 1];
    __shared__ int s_item;

    const int tid = threadIdx.x;
    const int wave = tid >> 6, lane = tid & 63;
    const int gi = lane & 15, gk = lane >> 4;      // MFMA lane roles: row/column, k block
    const int bw = wave;                           // the wave's bin in both GEMMs
    // synthesis role: nu = 1, thread = (sub-element n, scatterer group sh);
    // nu = 2, thread = (element ne, scatterer group sge), both sub-elements
    const int n = tid % MS, sh = tid / MS;
    const int ne = tid % NE, sge = tid / NE;
    const bool active = NUV == 2 ? 2 * ne < A.M : n < A.M;
    const SubFrame fr = load_frame(A.sub, NUV == 2 ? (active ? 2 * ne : 0) : (active ? n : 0));
    const SubFrame fr1 = load_frame(A.sub, NUV == 2 && active ? 2 * ne + 1 : 0);
    const int n_tg = (A.n_tx + TPG - 1) / TPG;
    const uint2* WTb = reinterpret_cast<const uint2*>(A.WT);

    DeltaParams P{};
    if (TABLE) {
        for (int i = tid; i < 2 * DELTA_NT; i += NB) s_tab[i] = A.dtab[i];
        P = *A.dpar;
    }

    auto load_chunk = [&](int s0, int s_end, int par) {
        if (tid < SCH) {
            const int s = s0 + tid;
            float4 v = make_float4(0.f, 0.f, 1.f, 0.f);     // padding: R = 0
            if (s < s_end) v = make_float4(A.x[s], HASY ? A.y[s] : 0.f, A.z[s], A.refl[s]);
            s_sc[par][tid] = v;
        }
    };

    if (tid == 0) s_item = atomicAdd(A.ticket, 1);
    __syncthreads();
    int item = s_item;
    while (item < A.n_items) {
        const int id = A.order[item];          // costliest first
        const Item it = A.items[id];
        const int bt = it.tile & 0xffff, tg = it.tile >> 16;
        const int jb0 = bt * JT;
        const int nb = min(JT, A.n_bins - jb0);
        // this wave's weights: WT[bin][tg][t = gi][e = 16 k + 4 gk .. + 3]
        const int jbw = min(jb0 + bw, A.n_bins - 1);
        // columns past the transmit count are zero in the table: their lanes
        // all read the first of them (one cache line per load)
        const int wc = min(gi, A.n_tx - tg * TPG);
        const uint2* wg = WTb + (((int64_t)jbw * n_tg + tg) * TPG + wc) * NE + 4 * gk;

        // the wave's split weights are the same for every chunk of the item:
        // those of the first KH k-steps stay in registers (all of them for 64
        // element slots; the first half for 128, where all would spill 72
        // dwords, three of eight for nu = 2, whose synthesis holds both
        // sub-elements' sums; none with y, which then spills 19): 128 focused
        // transmits on a 64-element array 30.7 -> 26.3 ms, a quarter of the
        // uneven 16-phantom batch 255.7 -> 251.2 ms
        constexpr int KH = NE == 64 ? KS : HASY ? 0 : NUV == 2 ? 3 : KS / 2;
        uint4 wr[KS][2];
#pragma unroll
        for (int k = 0; k < KH; ++k) {
            const uint4* q = reinterpret_cast<const uint4*>(wg + 16 * k);
            wr[k][0] = q[0];
            wr[k][1] = q[1];
        }
        // receive sums of the wave's receive bin: element tiles x (Re, Im)
        floatx4 X[RXE][2];
#pragma unroll
        for (int m = 0; m < RXE; ++m) X[m][0] = X[m][1] = floatx4{0.f, 0.f, 0.f, 0.f};

        load_chunk(it.s_begin, it.s_end, 0);
        __syncthreads();
        for (int s0 = it.s_begin, par = 0; s0 < it.s_end; s0 += SCH, par ^= 1) {
            // ---- P1: the element sums of the eight bins, split; pair by pair
            //      (set-up, then its eight bins), so that one pair's state is
            //      live at a time and its eight table fetches are in flight
            //      together
            if constexpr (NUV == 2) {
                // both sub-elements of element ne in one thread: their sum
                // is split once (a lane per sub-element, summed by a DPP
                // exchange and split by both lanes: a quarter of the uneven
                // 16-phantom batch 227.5 -> 202.7 ms, results bit-identical)
                constexpr int PPS = SCH * NE / NB;   // scatterers per thread
#pragma unroll 1
                for (int k = 0; k < PPS; ++k) {
                    prio_by_progress(k, PPS);
                    const int s = sge * PPS + k;
                    const float4 v = s_sc[par][s];
                    float2 B[JT];
#pragma unroll
                    for (int u = 0; u < 2; ++u) {
                        Geo g = make_geo<HASY, true>(A.K, u ? fr1 : fr, v.x, v.y, v.z, A.j_lo + jb0);
                        if (!active) g.E = make_float2(0.f, 0.f);
                        if (TABLE) g.kap *= P.kscale;             // delta_fetch's argument
                        float2 G[JT];
                        if constexpr (TABLE) {
                            DeltaFetch fch[JT];
#pragma unroll
                            for (int jj = 0; jj < JT; ++jj) fch[jj] = delta_fetch(s_tab, P, (float)(A.j_lo + jb0 + jj) * g.kap);
#pragma unroll
                            for (int jj = 0; jj < JT; ++jj) G[jj] = green_next_fetched(g, fch[jj]);
                        } else {
#pragma unroll
                            for (int jj = 0; jj < JT; ++jj)
                                G[jj] = green_next<HASY, TABLE>(A.K, g, (float)(A.j_lo + jb0 + jj), 1.f, s_tab, P);
                        }
#pragma unroll
                        for (int jj = 0; jj < JT; ++jj)
                            B[jj] = u ? make_float2(B[jj].x + G[jj].x, B[jj].y + G[jj].y) : G[jj];
                    }
#pragma unroll
                    for (int jj = 0; jj < JT; ++jj) {
                        const uint32_t h = pack_bf16(B[jj].x, B[jj].y);
                        s_Bh[jj][s * BPS + ne] = h;
                        s_Bl[jj][s * BPS + ne] = pack_bf16(B[jj].x - bf16_lo(h), B[jj].y - bf16_hi(h));
                    }
                }
            } else {
#pragma unroll 1
                for (int k = 0; k < PPT; ++k) {
                    prio_by_progress(k, PPT);
                    const int s = sh * PPT + k;
                    const float4 v = s_sc[par][s];
                    Geo g = make_geo<HASY, true>(A.K, fr, v.x, v.y, v.z, A.j_lo + jb0);
                    if (!active) g.E = make_float2(0.f, 0.f);
                    if (TABLE) g.kap *= P.kscale;                 // delta_fetch's argument
                    float2 G[JT];
                    if constexpr (TABLE) {
                        DeltaFetch fch[JT];
#pragma unroll
                        for (int jj = 0; jj < JT; ++jj) fch[jj] = delta_fetch(s_tab, P, (float)(A.j_lo + jb0 + jj) * g.kap);
#pragma unroll
                        for (int jj = 0; jj < JT; ++jj) G[jj] = green_next_fetched(g, fch[jj]);
                    } else {
#pragma unroll
                        for (int jj = 0; jj < JT; ++jj)
                            G[jj] = green_next<HASY, TABLE>(A.K, g, (float)(A.j_lo + jb0 + jj), 1.f, s_tab, P);
                    }
                    const int e = n;
#pragma unroll
                    for (int jj = 0; jj < JT; ++jj) {
                        const float bx = G[jj].x, by = G[jj].y;
                        const uint32_t h = pack_bf16(bx, by);
                        s_Bh[jj][s * BPS + e] = h;
                        s_Bl[jj][s * BPS + e] = pack_bf16(bx - bf16_lo(h), by - bf16_hi(h));
                    }
                }
            }
            // the GEMM phase: a wave in the transmit GEMM issues before one
            // already in the receive GEMM
            __builtin_amdgcn_s_setprio(3);
            // the rest of the wave's split weights, per chunk
#pragma unroll
            for (int k = KH; k < KS; ++k) {
                const uint4* q = reinterpret_cast<const uint4*>(wg + 16 * k);
                wr[k][0] = q[0];
                wr[k][1] = q[1];
            }
            __syncthreads();
            // ---- P2: transmit GEMM of bin bw: rows s = gi, columns t = gi,
            //      k = (element 16 k + 4 gk + q, Re/Im)
            uint32_t ch[4], cl[4];
            {
                const uint32_t* bh = s_Bh[bw] + gi * BPS + 4 * gk;
                const uint32_t* bl = s_Bl[bw] + gi * BPS + 4 * gk;
                floatx4 re = {0.f, 0.f, 0.f, 0.f}, im = re;
#pragma unroll
                for (int k = 0; k < KS; ++k) {
                    const uint4 ah4 = *reinterpret_cast<const uint4*>(bh + 16 * k);
                    const uint4 al4 = *reinterpret_cast<const uint4*>(bl + 16 * k);
                    const u32x4 ah = {ah4.x, ah4.y, ah4.z, ah4.w}, al = {al4.x, al4.y, al4.z, al4.w};
                    // weights of elements q = 0..3: (h, l) words
                    const uint32_t wh[4] = {wr[k][0].x, wr[k][0].z, wr[k][1].x, wr[k][1].z};
                    const uint32_t wl[4] = {wr[k][0].y, wr[k][0].w, wr[k][1].y, wr[k][1].w};
                    const u32x4 rh = {bf_conj(wh[0]), bf_conj(wh[1]), bf_conj(wh[2]), bf_conj(wh[3])};
                    const u32x4 rl = {bf_conj(wl[0]), bf_conj(wl[1]), bf_conj(wl[2]), bf_conj(wl[3])};
                    const u32x4 ih = {bf_swap(wh[0]), bf_swap(wh[1]), bf_swap(wh[2]), bf_swap(wh[3])};
                    const u32x4 il = {bf_swap(wl[0]), bf_swap(wl[1]), bf_swap(wl[2]), bf_swap(wl[3])};
                    re = mfma_bf(ah, rh, re);
                    re = mfma_bf(ah, rl, re);
                    re = mfma_bf(al, rh, re);
                    im = mfma_bf(ah, ih, im);
                    im = mfma_bf(ah, il, im);
                    im = mfma_bf(al, ih, im);
                }
                // D[row][col]: row s = 4 gk + v, col t = gi; c = R_s a, split.
                // The receive GEMM's B operand takes k = (scatterer 4 gk + q,
                // Re/Im) and column gi in the same lane: c stays in registers
#pragma unroll
                for (int v = 0; v < 4; ++v) {
                    const float R = s_sc[par][4 * gk + v].w;
                    const float cx = R * re[v], cy = R * im[v];
                    ch[v] = pack_bf16(cx, cy);
                    cl[v] = pack_bf16(cx - bf16_lo(ch[v]), cy - bf16_hi(ch[v]));
                }
            }
            __builtin_amdgcn_s_setprio(2);
            // ---- P3: receive GEMM of bin bw: rows e, columns t = gi,
            //      k = (scatterer 4 gk + q, Re/Im); the next chunk's scatterers
            {
                const u32x4 rh = {bf_conj(ch[0]), bf_conj(ch[1]), bf_conj(ch[2]), bf_conj(ch[3])};
                const u32x4 rl = {bf_conj(cl[0]), bf_conj(cl[1]), bf_conj(cl[2]), bf_conj(cl[3])};
                const u32x4 ih = {bf_swap(ch[0]), bf_swap(ch[1]), bf_swap(ch[2]), bf_swap(ch[3])};
                const u32x4 il = {bf_swap(cl[0]), bf_swap(cl[1]), bf_swap(cl[2]), bf_swap(cl[3])};
                const uint32_t* bh = s_Bh[bw] + 4 * gk * BPS + gi;
                const uint32_t* bl = s_Bl[bw] + 4 * gk * BPS + gi;
#pragma unroll
                for (int m = 0; m < RXE; ++m) {
                    const u32x4 ah = {bh[16 * m], bh[BPS + 16 * m], bh[2 * BPS + 16 * m], bh[3 * BPS + 16 * m]};
                    const u32x4 al = {bl[16 * m], bl[BPS + 16 * m], bl[2 * BPS + 16 * m], bl[3 * BPS + 16 * m]};
                    X[m][0] = mfma_bf(ah, rh, X[m][0]);
                    X[m][0] = mfma_bf(ah, rl, X[m][0]);
                    X[m][0] = mfma_bf(al, rh, X[m][0]);
                    X[m][1] = mfma_bf(ah, ih, X[m][1]);
                    X[m][1] = mfma_bf(ah, il, X[m][1]);
                    X[m][1] = mfma_bf(al, ih, X[m][1]);
                }
            }
            if (s0 + SCH < it.s_end) load_chunk(s0 + SCH, it.s_end, par ^ 1);
            __syncthreads();
        }
        // per-element partials [item][JT][TPG][N] of the wave's receive bin;
        // D[row][col]: row = element 16 m + 4 gk + v, col = transmit gi
        if (bw < nb) {
            float2* out = A.part + ((int64_t)id * JT + bw) * TPG * A.N;
#pragma unroll
            for (int m = 0; m < RXE; ++m)
#pragma unroll
                for (int v = 0; v < 4; ++v) {
                    const int e = 16 * m + 4 * gk + v;
                    if (e < A.N) out[(int64_t)gi * A.N + e] = make_float2(X[m][0][v], X[m][1][v]);
                }
        }
        if (tid == 0) s_item = atomicAdd(A.ticket, 1);
        __syncthreads();
        item = s_item;
    }
}

// More than 16 transmits: groups of 32 transmit columns (64 with CPW = 2,
// for 64 element slots and more than 32 transmits), four bins per item,
// split-bf16 products as in k_synth_mb.  The Green's terms of a pair are
// synthesised once per group (twice over two groups of 16 in k_synth_mb),
// at the price of a set-up every four bins.  Wave w = (bin w / 2, CPW
// column tiles from CPW (w % 2)):
//   P1  every thread: set-up and the element sums of the four bins, split;
//   P2  the transmit GEMM of its bin and column tiles (16 CPW transmits);
//   P3  the receive GEMM of its bin and column tiles over all elements, into
//       its registers, from the c of P2 kept in registers as in k_synth_mb
//       (two barriers per chunk).  With the receive GEMM over element halves
//       and both column tiles, c went through LDS with a barrier between the
//       GEMMs: 128 focused transmits on 64 elements 18.8 -> 17.3 ms, 21
//       plane waves 101.0 -> 100.2 ms (results bit-identical).
template <int NE, int NUV, bool HASY, bool TABLE, int CPW>
__global__ __launch_bounds__(512) void k_synth_mw(SynthArgs A)
{
    constexpr int NB = 512;
    constexpr int MS = NE * NUV;            // sub-element slots
    constexpr int SCH = 16;                 // scatterers per chunk (MFMA rows)
    constexpr int PPT = SCH * MS / NB;      // pairs per synthesis thread
    constexpr int NSG = NB / MS;            // scatterer groups
    constexpr int JT = 4;                   // bins per item: two waves per bin
    constexpr int TPG = 32 * CPW;           // transmit columns: two halves of CPW tiles of 16
    constexpr int BPS = NE + 4;             // row stride (words) of the element-sum planes
    constexpr int KS = NE / 16;             // transmit-GEMM k-steps (16 elements each)
    constexpr int RXE = NE / 16;            // receive element tiles
    static_assert(NE == 64 || NE == 128, "64 or 128 element slots");
    static_assert(NUV == 1 || NUV == 2, "nu must be 1 or 2");
    static_assert(PPT * NSG == SCH, "threads must cover the chunk");
    static_assert(CPW == 1 || (CPW == 2 && NE == 64), "two column tiles per wave for 64 slots only");

    __shared__ float4 s_sc[2][SCH];          // by chunk parity
    __shared__ __align__(16) uint32_t s_Bh[JT][SCH * BPS];
    __shared__ __align__(16) uint32_t s_Bl[JT][SCH * BPS];
    __shared__ float4 s_tab[TABLE ? 2 * DELTA_NT : 1];
    __shared__ int s_item;

    const int tid = threadIdx.x;
    const int wave = tid >> 6, lane = tid & 63;
    const int gi = lane & 15, gk = lane >> 4;      // MFMA lane roles: row/column, k block
    const int wj = wave >> 1, wh = wave & 1;       // the wave's bin and half
    // synthesis role: nu = 1, thread = (sub-element n, scatterer group sh);
    // nu = 2, thread = (element ne, scatterer group sge), both sub-elements
    const int n = tid % MS, sh = tid / MS;
    const int ne = tid % NE, sge = tid / NE;
    const bool active = NUV == 2 ? 2 * ne < A.M : n < A.M;
    const SubFrame fr = load_frame(A.sub, NUV == 2 ? (active ? 2 * ne : 0) : (active ? n : 0));
    const SubFrame fr1 = load_frame(A.sub, NUV == 2 && active ? 2 * ne + 1 : 0);
    const int n_tg = (A.n_tx + TPG - 1) / TPG;
    const uint2* WTb = reinterpret_cast<const uint2*>(A.WT);

    DeltaParams P{};
    if (TABLE) {
        for (int i = tid; i < 2 * DELTA_NT; i += NB) s_tab[i] = A.dtab[i];
        P = *A.dpar;
    }

    auto load_chunk = [&](int s0, int s_end, int par) {
        if (tid < SCH) {
            const int s = s0 + tid;
            float4 v = make_float4(0.f, 0.f, 1.f, 0.f);     // padding: R = 0
            if (s < s_end) v = make_float4(A.x[s], HASY ? A.y[s] : 0.f, A.z[s], A.refl[s]);
            s_sc[par][tid] = v;
        }
    };

    if (tid == 0) s_item = atomicAdd(A.ticket, 1);
    __syncthreads();
    int item = s_item;
    while (item < A.n_items) {
        const int id = A.order[item];          // costliest first
        const Item it = A.items[id];
        const int bt = it.tile & 0xffff, tg = it.tile >> 16;
        const int jb0 = bt * JT;
        const int nb = min(JT, A.n_bins - jb0);
        // this wave's weights: WT[bin][tg][t = 16 (CPW wh + ct) + gi][e = 16 k + 4 gk .. + 3]
        const int jbw = min(jb0 + wj, A.n_bins - 1);
        // columns past the transmit count are zero in the table: their lanes
        // all read the first of them (one cache line per load)
        const uint2* wg[CPW];
#pragma unroll
        for (int ct = 0; ct < CPW; ++ct) {
            const int wc = min(16 * (CPW * wh + ct) + gi, A.n_tx - tg * TPG);
            wg[ct] = WTb + (((int64_t)jbw * n_tg + tg) * TPG + wc) * NE + 4 * gk;
        }
        // the weights of the first KH k-steps stay in registers for the item
        // (all of them for 64 element slots, half for 128 without y: 21 plane
        // waves, 200k scatterers 112.6 -> 101.1 ms; half with two column tiles
        // per wave, where all spill 26 dwords: 128 focused transmits on 64
        // elements 14.1 ms, 15.6 with three of four k-steps, 19.7 with none;
        // one for nu = 2, whose synthesis holds both sub-elements' sums)
        constexpr int KH = CPW == 2 ? (HASY ? 0 : NUV == 2 ? 1 : KS / 2) : NE == 64 ? KS : HASY ? 0 : KS / 2;
        uint4 wr[CPW][KS][2];
#pragma unroll
        for (int ct = 0; ct < CPW; ++ct)
#pragma unroll
            for (int k = 0; k < KH; ++k) {
                const uint4* q = reinterpret_cast<const uint4*>(wg[ct] + 16 * k);
                wr[ct][k][0] = q[0];
                wr[ct][k][1] = q[1];
            }
        // receive sums of the wave's bin and column tiles: element tiles x
        // column tiles x (Re, Im)
        floatx4 X[RXE][CPW][2];
#pragma unroll
        for (int m = 0; m < RXE; ++m)
#pragma unroll
            for (int ct = 0; ct < CPW; ++ct) X[m][ct][0] = X[m][ct][1] = floatx4{0.f, 0.f, 0.f, 0.f};

        load_chunk(it.s_begin, it.s_end, 0);
        __syncthreads();
        for (int s0 = it.s_begin, par = 0; s0 < it.s_end; s0 += SCH, par ^= 1) {
            // ---- P1: the element sums of the four bins, split; pair by pair
            //      (set-up, then its four bins)
            if constexpr (NUV == 2) {
                // both sub-elements of element ne in one thread: their sum
                // is split once (21 plane waves, 200k scatterers 99.5 -> 88.9
                // ms, results bit-identical)
                constexpr int PPS = SCH * NE / NB;   // scatterers per thread
#pragma unroll 1
                for (int k = 0; k < PPS; ++k) {
                    prio_by_progress(k, PPS);
                    const int s = sge * PPS + k;
                    const float4 v = s_sc[par][s];
                    float2 B[JT];
#pragma unroll
                    for (int u = 0; u < 2; ++u) {
                        Geo g = make_geo<HASY, true>(A.K, u ? fr1 : fr, v.x, v.y, v.z, A.j_lo + jb0);
                        if (!active) g.E = make_float2(0.f, 0.f);
                        if (TABLE) g.kap *= P.kscale;             // delta_fetch's argument
                        float2 G[JT];
                        if constexpr (TABLE) {
                            DeltaFetch fch[JT];
#pragma unroll
                            for (int jj = 0; jj < JT; ++jj) fch[jj] = delta_fetch(s_tab, P, (float)(A.j_lo + jb0 + jj) * g.kap);
#pragma unroll
                            for (int jj = 0; jj < JT; ++jj) G[jj] = green_next_fetched(g, fch[jj]);
                        } else {
#pragma unroll
                            for (int jj = 0; jj < JT; ++jj)
                                G[jj] = green_next<HASY, TABLE>(A.K, g, (float)(A.j_lo + jb0 + jj), 1.f, s_tab, P);
                        }
#pragma unroll
                        for (int jj = 0; jj < JT; ++jj)
                            B[jj] = u ? make_float2(B[jj].x + G[jj].x, B[jj].y + G[jj].y) : G[jj];
                    }
#pragma unroll
                    for (int jj = 0; jj < JT; ++jj) {
                        const uint32_t h = pack_bf16(B[jj].x, B[jj].y);
                        s_Bh[jj][s * BPS + ne] = h;
                        s_Bl[jj][s * BPS + ne] = pack_bf16(B[jj].x - bf16_lo(h), B[jj].y - bf16_hi(h));
                    }
                }
            } else {
#pragma unroll 1
                for (int k = 0; k < PPT; ++k) {
                    prio_by_progress(k, PPT);
                    const int s = sh * PPT + k;
                    const float4 v = s_sc[par][s];
                    Geo g = make_geo<HASY, true>(A.K, fr, v.x, v.y, v.z, A.j_lo + jb0);
                    if (!active) g.E = make_float2(0.f, 0.f);
                    if (TABLE) g.kap *= P.kscale;                 // delta_fetch's argument
                    float2 G[JT];
                    if constexpr (TABLE) {
                        DeltaFetch fch[JT];
#pragma unroll
                        for (int jj = 0; jj < JT; ++jj) fch[jj] = delta_fetch(s_tab, P, (float)(A.j_lo + jb0 + jj) * g.kap);
#pragma unroll
                        for (int jj = 0; jj < JT; ++jj) G[jj] = green_next_fetched(g, fch[jj]);
                    } else {
#pragma unroll
                        for (int jj = 0; jj < JT; ++jj)
                            G[jj] = green_next<HASY, TABLE>(A.K, g, (float)(A.j_lo + jb0 + jj), 1.f, s_tab, P);
                    }
                    const int e = n;
#pragma unroll
                    for (int jj = 0; jj < JT; ++jj) {
                        const float bx = G[jj].x, by = G[jj].y;
                        const uint32_t h = pack_bf16(bx, by);
                        s_Bh[jj][s * BPS + e] = h;
                        s_Bl[jj][s * BPS + e] = pack_bf16(bx - bf16_lo(h), by - bf16_hi(h));
                    }
                }
            }
            // the GEMM phase: a wave in the transmit GEMM issues before one
            // already in the receive GEMM
            __builtin_amdgcn_s_setprio(3);
            // the rest of the wave's split weights, per chunk
#pragma unroll
            for (int ct = 0; ct < CPW; ++ct)
#pragma unroll
                for (int k = KH; k < KS; ++k) {
                    const uint4* q = reinterpret_cast<const uint4*>(wg[ct] + 16 * k);
                    wr[ct][k][0] = q[0];
                    wr[ct][k][1] = q[1];
                }
            __syncthreads();
            uint32_t ch[CPW][4], cl[CPW][4];
            // ---- P2: transmit GEMM of bin wj, column tiles CPW wh .. + CPW - 1:
            //      rows s = gi, columns t = 16 (CPW wh + ct) + gi, k = (element
            //      16 k + 4 gk + q, Re/Im)
#pragma unroll
            for (int ct = 0; ct < CPW; ++ct) {
                const uint32_t* bh = s_Bh[wj] + gi * BPS + 4 * gk;
                const uint32_t* bl = s_Bl[wj] + gi * BPS + 4 * gk;
                floatx4 re = {0.f, 0.f, 0.f, 0.f}, im = re;
#pragma unroll
                for (int k = 0; k < KS; ++k) {
                    const uint4 ah4 = *reinterpret_cast<const uint4*>(bh + 16 * k);
                    const uint4 al4 = *reinterpret_cast<const uint4*>(bl + 16 * k);
                    const u32x4 ah = {ah4.x, ah4.y, ah4.z, ah4.w}, al = {al4.x, al4.y, al4.z, al4.w};
                    const uint32_t wh4[4] = {wr[ct][k][0].x, wr[ct][k][0].z, wr[ct][k][1].x, wr[ct][k][1].z};
                    const uint32_t wl4[4] = {wr[ct][k][0].y, wr[ct][k][0].w, wr[ct][k][1].y, wr[ct][k][1].w};
                    const u32x4 rh = {bf_conj(wh4[0]), bf_conj(wh4[1]), bf_conj(wh4[2]), bf_conj(wh4[3])};
                    const u32x4 rl = {bf_conj(wl4[0]), bf_conj(wl4[1]), bf_conj(wl4[2]), bf_conj(wl4[3])};
                    const u32x4 ih = {bf_swap(wh4[0]), bf_swap(wh4[1]), bf_swap(wh4[2]), bf_swap(wh4[3])};
                    const u32x4 il = {bf_swap(wl4[0]), bf_swap(wl4[1]), bf_swap(wl4[2]), bf_swap(wl4[3])};
                    re = mfma_bf(ah, rh, re);
                    re = mfma_bf(ah, rl, re);
                    re = mfma_bf(al, rh, re);
                    im = mfma_bf(ah, ih, im);
                    im = mfma_bf(ah, il, im);
                    im = mfma_bf(al, ih, im);
                }
                // D[row][col]: row s = 4 gk + v, col t = 16 (CPW wh + ct) + gi;
                // c = R_s a, split.  The receive GEMM's B operand takes k =
                // (scatterer 4 gk + q, Re/Im) and column gi in the same lane: c
                // stays in registers
#pragma unroll
                for (int v = 0; v < 4; ++v) {
                    const float R = s_sc[par][4 * gk + v].w;
                    const float cx = R * re[v], cy = R * im[v];
                    ch[ct][v] = pack_bf16(cx, cy);
                    cl[ct][v] = pack_bf16(cx - bf16_lo(ch[ct][v]), cy - bf16_hi(ch[ct][v]));
                }
            }
            __builtin_amdgcn_s_setprio(2);
            // ---- P3: receive GEMM of bin wj, the wave's column tiles, all
            //      element tiles, k = (scatterer 4 gk + q, Re/Im); the next
            //      chunk's scatterers
            {
                u32x4 rh[CPW], rl[CPW], ih[CPW], il[CPW];
#pragma unroll
                for (int ct = 0; ct < CPW; ++ct) {
                    rh[ct] = u32x4{bf_conj(ch[ct][0]), bf_conj(ch[ct][1]), bf_conj(ch[ct][2]), bf_conj(ch[ct][3])};
                    rl[ct] = u32x4{bf_conj(cl[ct][0]), bf_conj(cl[ct][1]), bf_conj(cl[ct][2]), bf_conj(cl[ct][3])};
                    ih[ct] = u32x4{bf_swap(ch[ct][0]), bf_swap(ch[ct][1]), bf_swap(ch[ct][2]), bf_swap(ch[ct][3])};
                    il[ct] = u32x4{bf_swap(cl[ct][0]), bf_swap(cl[ct][1]), bf_swap(cl[ct][2]), bf_swap(cl[ct][3])};
                }
                const uint32_t* bh = s_Bh[wj] + 4 * gk * BPS + gi;
                const uint32_t* bl = s_Bl[wj] + 4 * gk * BPS + gi;
#pragma unroll
                for (int m = 0; m < RXE; ++m) {
                    const u32x4 ah = {bh[16 * m], bh[BPS + 16 * m], bh[2 * BPS + 16 * m], bh[3 * BPS + 16 * m]};
                    const u32x4 al = {bl[16 * m], bl[BPS + 16 * m], bl[2 * BPS + 16 * m], bl[3 * BPS + 16 * m]};
#pragma unroll
                    for (int ct = 0; ct < CPW; ++ct) {
                        X[m][ct][0] = mfma_bf(ah, rh[ct], X[m][ct][0]);
                        X[m][ct][0] = mfma_bf(ah, rl[ct], X[m][ct][0]);
                        X[m][ct][0] = mfma_bf(al, rh[ct], X[m][ct][0]);
                        X[m][ct][1] = mfma_bf(ah, ih[ct], X[m][ct][1]);
                        X[m][ct][1] = mfma_bf(ah, il[ct], X[m][ct][1]);
                        X[m][ct][1] = mfma_bf(al, ih[ct], X[m][ct][1]);
                    }
                }
            }
            if (s0 + SCH < it.s_end) load_chunk(s0 + SCH, it.s_end, par ^ 1);
            __syncthreads();
        }
        // per-element partials [item][JT][TPG][N] of the wave's bin and column
        // tiles; D[row][col]: row = element 16 m + 4 gk + v, col = transmit
        // 16 (CPW wh + ct) + gi
        if (wj < nb) {
            float2* out = A.part + ((int64_t)id * JT + wj) * TPG * A.N;
#pragma unroll
            for (int m = 0; m < RXE; ++m)
#pragma unroll
                for (int ct = 0; ct < CPW; ++ct)
#pragma unroll
                    for (int v = 0; v < 4; ++v) {
                        const int e = 16 * m + 4 * gk + v;
                        if (e < A.N)
                            out[(int64_t)(16 * (CPW * wh + ct) + gi) * A.N + e] = make_float2(X[m][ct][0][v], X[m][ct][1][v]);
                    }
        }
        if (tid == 0) s_item = atomicAdd(A.ticket, 1);
        __syncthreads();
        item = s_item;
    }
}

template <int NE, int NUV, int CPW = 1>
static SynthKernel mw_kernel_nuv(const SynthConfig& c)
{
    if (c.has_y) return k_synth_mw<NE, NUV, true, false, CPW>;
    if (c.table) return k_synth_mw<NE, NUV, false, true, CPW>;
    return k_synth_mw<NE, NUV, false, false, CPW>;
}

template <int NE, int NUV>
static SynthKernel mb_kernel_nuv(const SynthConfig& c)
{
    if (c.has_y) return k_synth_mb<NE, NUV, true, false>;
    if (c.table) return k_synth_mb<NE, NUV, false, true>;
    return k_synth_mb<NE, NUV, false, false>;
}

template <int NE, int NX, int NUV>
static SynthKernel mq_kernel_nuv(const SynthConfig& c)
{
    if (c.has_y) return k_synth_mq<NE, NUV, NX, true, false>;
    if (c.table) return k_synth_mq<NE, NUV, NX, false, true>;
    return k_synth_mq<NE, NUV, NX, false, false>;
}

SynthKernel synth_mt_kernel(const SynthConfig& c)
{
    if (c.bf && c.wt && c.tt == 64 && c.jt == 4 && c.ne == 64)
        return c.pair ? mw_kernel_nuv<64, 2, 2>(c) : mw_kernel_nuv<64, 1, 2>(c);
    if (c.bf && c.wt && c.tt == 32 && c.jt == 4) {
        if (c.ne == 128) return c.pair ? mw_kernel_nuv<128, 2>(c) : mw_kernel_nuv<128, 1>(c);
        if (c.ne == 64) return c.pair ? mw_kernel_nuv<64, 2>(c) : mw_kernel_nuv<64, 1>(c);
    }
    if (c.bf && c.wt && c.tt == 16 && c.jt == 8) {
        if (c.ne == 128) return c.pair ? mb_kernel_nuv<128, 2>(c) : mb_kernel_nuv<128, 1>(c);
        if (c.ne == 64) return c.pair ? mb_kernel_nuv<64, 2>(c) : mb_kernel_nuv<64, 1>(c);
    }
    if (c.wt && c.ne == 128 && c.tt == 16 && c.jt == 8 && c.nx == MQ_NX)
        return c.pair ? mq_kernel_nuv<128, MQ_NX, 2>(c) : mq_kernel_nuv<128, MQ_NX, 1>(c);
    if (c.wt && c.ne == 64 && c.tt == 16 && c.jt == 8 && c.nx == MQ_NX64)
        return c.pair ? mq_kernel_nuv<64, MQ_NX64, 2>(c) : mq_kernel_nuv<64, MQ_NX64, 1>(c);
    if (c.wt) return nullptr;
    if (c.ne == 128 && c.tt == 16) return mt_kernel_shape<128, 1, 4, 3>(c);
    if (c.ne == 128 && c.tt == 32) return mt_kernel_shape<128, 2, 4, 2>(c);
    if (c.ne == 64 && c.tt == 32) return mt_kernel_shape<64, 2, 6, 3>(c);
    if (c.ne == 64 && c.tt == 64) return mt_kernel_shape<64, 4, 6, 2>(c);
    return nullptr;
}

hipError_t launch_synth_mt(const SynthConfig& c, const SynthArgs& a, hipStream_t st)
{
    if (c.grid <= 0) return hipSuccess;
    if (!c.persistent || !a.ticket) return hipErrorInvalidValue;
    const SynthKernel k = synth_mt_kernel(c);
    if (!k) return hipErrorInvalidValue;
    SynthArgs arg = a;
    void* args[] = {&arg};
    return hipLaunchKernel(reinterpret_cast<const void*>(k), dim3(c.grid), dim3(512), args, 0, st);
}

}  // namespace simus
