// libsimus HIP kernels for gfx950: transmit weights, Green's-tile synthesis
// with both contractions (Eqs. 22, 29-33), finalisation (Eq. 34) and the
// inverse transform of Eq. (1).
#include <hip/hip_runtime.h>

#include <algorithm>

#include "green.hpp"
#include "kernels.hpp"

namespace simus {

// ---------------------------------------------------------------------------
// Transmit weights W[b][t][e] = apod[t][e] exp(i w_j tau[t][e]) (Eqs. 20, 22),
// phase reduced in FP64.
// ---------------------------------------------------------------------------
__global__ void k_wtable(float2* __restrict__ W, const double* __restrict__ delays,
                         const float* __restrict__ apod, int n_bins, int n_tx, int N, int j_lo,
                         double df)
{
    const int64_t total = (int64_t)n_bins * n_tx * N;
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < total;
         i += (int64_t)gridDim.x * blockDim.x) {
        const int te = (int)(i % ((int64_t)n_tx * N));
        const int b = (int)(i / ((int64_t)n_tx * N));
        const double turns = (double)(j_lo + b) * df * delays[te];
        const float t = (float)(turns - rint(turns));
        const float a = apod ? apod[te] : 1.f;
        W[i] = make_float2(a * cos_turns(t), a * sin_turns(t));
    }
}

hipError_t launch_wtable(float2* W, const double* delays, const float* apod, int n_bins, int n_tx,
                         int N, int j_lo, double df, hipStream_t st)
{
    const int64_t total = (int64_t)n_bins * n_tx * N;
    if (total == 0) return hipSuccess;
    const int grid = (int)std::min<int64_t>((total + 255) / 256, 4096);
    hipLaunchKernelGGL(k_wtable, dim3(grid), dim3(256), 0, st, W, delays, apod, n_bins, n_tx, N,
                       j_lo, df);
    return hipGetLastError();
}

// bf16 == false: float2 WT[bin][group][e][16 columns];
// bf16 == true:  uint2  WT[bin][group][16 columns][e], the weight split into
//   bf16 high and low parts, packed (Re, Im): x = (Re_h | Im_h << 16),
//   y = (Re_l | Im_l << 16), with Re = Re_h + Re_l to 16 significant bits.
__global__ void k_wtable_mt(float2* __restrict__ WT, const double* __restrict__ delays,
                            const float* __restrict__ apod, int n_bins, int n_tx, int N, int ne,
                            int tpg, int n_tg, int j_lo, double df, bool bf16)
{
    const int64_t total = (int64_t)n_bins * n_tg * ne * tpg;
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < total;
         i += (int64_t)gridDim.x * blockDim.x) {
        int c, e;
        int64_t r;
        if (bf16) {
            e = (int)(i % ne);
            r = i / ne;
            c = (int)(r % tpg);
            r /= tpg;
        } else {
            c = (int)(i % 16);
            r = i / 16;
            e = (int)(r % ne);
            r /= ne;
        }
        const int g = (int)(r % n_tg);
        const int b = (int)(r / n_tg);
        const int t = tpg * g + c;
        float2 w = make_float2(0.f, 0.f);
        if (e < N && t < n_tx) {
            const int te = t * N + e;
            const double turns = (double)(j_lo + b) * df * delays[te];
            const float ph = (float)(turns - rint(turns));
            const float a = apod ? apod[te] : 1.f;
            w = make_float2(a * cos_turns(ph), a * sin_turns(ph));
        }
        if (bf16) {
            const uint32_t h = pack_bf16(w.x, w.y);
            const uint32_t l = pack_bf16(w.x - bf16_lo(h), w.y - bf16_hi(h));
            WT[i] = make_float2(__uint_as_float(h), __uint_as_float(l));
        } else {
            WT[i] = w;
        }
    }
}

hipError_t launch_wtable_mt(float2* WT, const double* delays, const float* apod, int n_bins, int n_tx,
                            int N, int ne, int tpg, int n_tg, int j_lo, double df, bool bf16, hipStream_t st)
{
    if (!bf16 && tpg != 16) return hipErrorInvalidValue;
    const int64_t total = (int64_t)n_bins * n_tg * ne * tpg;
    if (total == 0) return hipSuccess;
    const int grid = (int)std::min<int64_t>((total + 255) / 256, 8192);
    hipLaunchKernelGGL(k_wtable_mt, dim3(grid), dim3(256), 0, st, WT, delays, apod, n_bins, n_tx, N, ne,
                       tpg, n_tg, j_lo, df, bf16);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Synthesis.  One block owns all sub-elements (thread n = sub-element n) and
// walks the scatterers of one work item in chunks of SC.  For each bin of
// its tile it
//   1. builds G[n][s] for the chunk in registers (Green's term, green.hpp),
//   2. Tx contraction a[s][t] = sum_n W[t][e(n)] G[n][s]: neighbouring lanes
//      are summed with DPP, the pair sums go to LDS and groups of lanes
//      reduce them (no atomics, fixed order),
//   3. scales by the reflectivity, c[s][t] = R_s a[s][t],
//   4. Rx contraction X[n][t] += sum_s G[n][s] c[s][t], accumulated in an
//      LDS slot private to the thread.
// Steps 2-3 of bin j and step 4 of bin j-1 share one barrier: the reduction
// rows and the reduced values are double-buffered, and G of bin j-1 stays in
// registers (two register sets, bins taken in pairs).
//
// PAIR (nu = 2): lanes 2e and 2e+1 hold the two sub-elements of element e,
// whose transmit weight is the same, so both contractions only need the
// element sum B[e][s] = G[2e][s] + G[2e+1][s] (Eqs. 29, 33), formed by one
// DPP exchange.  The receive sum of element e is then split over its lanes:
// the even lane accumulates Re X[e], the odd lane Im X[e], one float each.
// Otherwise every lane accumulates its own sub-element's complex X, and the
// finaliser sums the nu sub-elements of each element.
// ---------------------------------------------------------------------------

// Tunables of the synthesis launch (compile-time): scatterers per chunk for
// single-transmit groups and a waves-per-SIMD floor.
#ifndef SIMUS_SC1
#define SIMUS_SC1 8
#endif
#ifndef SIMUS_WAVES_PER_EU
#define SIMUS_WAVES_PER_EU 0
#endif
#if SIMUS_WAVES_PER_EU > 0
#define SIMUS_OCCUPANCY __attribute__((amdgpu_waves_per_eu(SIMUS_WAVES_PER_EU)))
#else
#define SIMUS_OCCUPANCY
#endif

// LDS of one k_synth block in bytes, term by term as the kernel declares it:
// scatterer chunk, transmit-reduction rows (two buffers), reduced values,
// receive accumulators of the tile, elevation table, work-item slot.
constexpr int synth_lds(int bs, int sc, int tt, int groups, bool pair, bool table_lds, int jt)
{
    const int nt = sc * tt * groups;
    const int rs = bs / groups / 2 + 4;
    return 16 * groups * sc + 8 * 2 * nt * rs + 8 * 2 * (pair ? 2 : 1) * nt +
           4 * jt * tt * bs * (pair ? 1 : 2) + 16 * (table_lds ? 2 * DELTA_NT : 1) + 4;
}

// LDS is allocated to blocks in 2 KiB granules of the CU's 160 KiB (measured:
// a 53,124-byte block runs three per CU, a 54,020-byte one two).
constexpr int LDS_PER_CU = 163840;
constexpr int LDS_GRANULE = 2048;

// Blocks per CU that the registers allow: paired kernels take about 155
// VGPRs (three waves per SIMD), unpaired ones about 175 (two); at least one.
constexpr int synth_blocks_per_cu(int bs, bool pair)
{
    const int b = 4 * (pair ? 3 : 2) / (bs / 64);
    return b < 1 ? 1 : b;
}

// Bins per tile: the longest tile, up to 32, whose blocks fit the CU's LDS
// at that occupancy.  Longer tiles amortise each pair's set-up (an FP64
// distance, ten transcendentals).  Single transmits, 128 elements: 27 bins
// (config 2: 9.32 ms; 26 bins 9.42, 18 bins with the 512-interval table 9.70;
// 28 bins leave two blocks per CU: 11.7).
constexpr int synth_jt(int bs, int tt, bool pair, bool table_lds, int groups = 1)
{
    const int sc = tt == 2 ? 4 : SIMUS_SC1;
    const int limit = LDS_PER_CU / synth_blocks_per_cu(bs, pair) / LDS_GRANULE * LDS_GRANULE;
    // at most 32 bins for 256-thread blocks, 16 for 512 and 6 for 1024 (whose
    // 128-VGPR bound spills with 8 or more)
    int jt = bs <= 256 ? 32 : bs == 512 ? 16 : 6;
    while (jt > 1 && synth_lds(bs, sc, tt, groups, pair, table_lds, jt) > limit) --jt;
    return jt;
}

// DPP lane exchanges within rows of 16 lanes (gfx9 encodings).
enum : int {
    DPP_XOR1 = 0xB1,          // quad_perm [1,0,3,2]
    DPP_XOR2 = 0x4E,          // quad_perm [2,3,0,1]
    DPP_HALF_MIRROR = 0x141,  // lane i <-> 7 - i within 8
    DPP_MIRROR = 0x140        // lane i <-> 15 - i within 16
};

// Value of v in the lane selected by CTRL (all source lanes are active
// wherever this is used).
template <int CTRL>
__device__ __forceinline__ float dpp(float v)
{
    return __int_as_float(__builtin_amdgcn_mov_dpp(__float_as_int(v), CTRL, 0xF, 0xF, true));
}

// Sum over an aligned group of GL lanes (GL a power of two <= 64); every
// lane of the group receives the total.
template <int GL>
__device__ __forceinline__ float group_sum(float v)
{
    if (GL >= 2) v += dpp<DPP_XOR1>(v);
    if (GL >= 4) v += dpp<DPP_XOR2>(v);
    if (GL >= 8) v += dpp<DPP_HALF_MIRROR>(v);
    if (GL >= 16) v += dpp<DPP_MIRROR>(v);
    if (GL >= 32) v += __shfl_xor(v, 16);
    if (GL >= 64) v += __shfl_xor(v, 32);
    return v;
}

// EL: elevation term evaluated directly (0), from the table (1), or absent
// (2, 2-D acoustics).  NG groups of BS / NG sub-element slots share the block
// (its LDS table and barriers); group g takes the g-th chunk of SC scatterers
// of each super-chunk of NG SC, so small probes still fill 256-thread blocks.
template <int BS, int SC, int JT, int TT, bool HASY, int EL, bool PAIR, int NG>
__global__ __launch_bounds__(BS) SIMUS_OCCUPANCY void k_synth(SynthArgs A)
{
    constexpr int BG = BS / NG;            // sub-element slots per group
    constexpr int NS = SC * TT;            // sums per bin and group
    constexpr int NT = NS * NG;            // sums per bin
    constexpr int HB = BG / 2;             // pair sums per row
    constexpr int RS = HB + 4;             // LDS row stride (float2)
    constexpr int GL = (BS / 2 / NT >= 64) ? 64 : (BS / 2 / NT < HB ? BS / 2 / NT : HB);   // lanes per sum
    constexpr int PER = HB / GL;           // values per lane
    constexpr int NA = PAIR ? 1 : 2;       // floats per accumulator slot
    static_assert(NT <= BS / 2 && GL >= 1 && HB % GL == 0, "sums must fit half the block");
    static_assert(BG >= 64 && BG % 64 == 0, "a group spans whole waves");

    __shared__ float4 s_sc[NG * SC];
    __shared__ float2 s_red[2][NT * RS];
    // reduced values c (PAIR: [0] = (Re c, -Im c) for even lanes,
    // [1] = (Im c, Re c) for odd lanes)
    __shared__ float2 s_c[2][PAIR ? 2 : 1][NT];
    __shared__ float s_acc[JT * TT * BS * NA];
    constexpr bool TABLE = EL == 1;
    __shared__ float4 s_tab[TABLE ? 2 * DELTA_NT : 1];
    static_assert(sizeof(s_sc) + sizeof(s_red) + sizeof(s_c) + sizeof(s_acc) + sizeof(s_tab) + sizeof(int) ==
                      (size_t)synth_lds(BS, SC, TT, NG, PAIR, TABLE, JT),
                  "synth_lds must follow the declarations");

    const int tid = threadIdx.x;
    const int n = tid % BG, grp = tid / BG;    // sub-element slot, group
    const bool active = n < A.M;
    const SubFrame fr = load_frame(A.sub, active ? n : 0);
    const int e = active ? n / A.nu : 0;
    DeltaParams P{};
    if (TABLE) {
        for (int i = tid; i < 2 * DELTA_NT; i += BS) s_tab[i] = A.dtab[i];
        P = *A.dpar;
    }

    // Tx reduction of one bin: rows s_red[buf] -> s_c[buf] (R_s applied).
    auto reduce = [&](int buf) {
        const int sid = tid / GL, lg = tid % GL;
        if (sid < NT) {
            // two independent partial sums shorten the dependency chain
            float2 acc = make_float2(0.f, 0.f), acc2 = make_float2(0.f, 0.f);
            const float2* row = &s_red[buf][sid * RS];
#pragma unroll
            for (int i = 0; i < PER; i += 2) {
                const float2 v = row[lg + i * GL];
                acc.x += v.x;
                acc.y += v.y;
                if (i + 1 < PER) {
                    const float2 u = row[lg + (i + 1) * GL];
                    acc2.x += u.x;
                    acc2.y += u.y;
                }
            }
            acc.x += acc2.x;
            acc.y += acc2.y;
            acc.x = group_sum<GL>(acc.x);
            acc.y = group_sum<GL>(acc.y);
            if (lg == 0) {
                const float R = s_sc[(sid / NS) * SC + sid % SC].w;
                const float cx = R * acc.x, cy = R * acc.y;
                if (PAIR) {
                    s_c[buf][0][sid] = make_float2(cx, -cy);
                    s_c[buf][1][sid] = make_float2(cy, cx);
                } else {
                    s_c[buf][0][sid] = make_float2(cx, cy);
                }
            }
        }
    };
    // Rx accumulation of local bin jj from s_c[buf] with the terms G of that
    // bin (element sums B when paired).
    auto receive = [&](int jj, int buf, const float2 (&G)[SC]) {
#pragma unroll
        for (int t = 0; t < TT; ++t) {
            const int slot = (jj * TT + t) * BS + tid;
            if (PAIR) {
                const float2* cv = s_c[buf][tid & 1] + grp * NS + t * SC;
                float x = s_acc[slot], y = 0.f;
#pragma unroll
                for (int s = 0; s < SC; ++s) {
                    const float2 c = cv[s];
                    x = fmaf(G[s].x, c.x, x);
                    y = fmaf(G[s].y, c.y, y);
                }
                s_acc[slot] = x + y;
            } else {
                float2 x = make_float2(s_acc[2 * slot], s_acc[2 * slot + 1]), y = make_float2(0.f, 0.f);
#pragma unroll
                for (int s = 0; s < SC; s += 2) {
                    x = cfma(G[s], s_c[buf][0][grp * NS + t * SC + s], x);
                    if (s + 1 < SC) y = cfma(G[s + 1], s_c[buf][0][grp * NS + t * SC + s + 1], y);
                }
                s_acc[2 * slot] = x.x + y.x;
                s_acc[2 * slot + 1] = x.y + y.y;
            }
        }
    };

    // Static launch: one item per block.  Persistent launch: blocks draw
    // items from a work counter until it passes n_items (every block exits).
    // Items are drawn costliest first; an item's partials sit at its id.
    __shared__ int s_item;
    int item = blockIdx.x;
    if (A.ticket) {
        if (tid == 0) s_item = atomicAdd(A.ticket, 1);
        __syncthreads();
        item = s_item;
    }
    while (item < A.n_items) {
        const int id = A.order[item];
        const Item it = A.items[id];
        const int bt = it.tile & 0xffff, tg = it.tile >> 16;
        const int jb0 = bt * JT;
        const int nb = min(JT, A.n_bins - jb0);
        const int t0 = tg * TT;

        for (int i = tid; i < JT * TT * BS * NA; i += BS) s_acc[i] = 0.f;

        for (int s0 = it.s_begin; s0 < it.s_end; s0 += NG * SC) {
            if (tid < NG * SC) {
                const int s = s0 + tid;
                float4 v = make_float4(0.f, 0.f, 1.f, 0.f);     // padding: R = 0
                if (s < it.s_end) v = make_float4(A.x[s], HASY ? A.y[s] : 0.f, A.z[s], A.refl[s]);
                s_sc[tid] = v;
            }
            __syncthreads();
            Geo g[SC];
#pragma unroll
            for (int s = 0; s < SC; ++s) {
                const float4 v = s_sc[grp * SC + s];
                g[s] = make_geo<HASY>(A.K, fr, v.x, v.y, v.z, A.j_lo + jb0);
                if (!active) g[s].E = make_float2(0.f, 0.f);
                if (TABLE) g[s].kap *= P.kscale;          // delta_fetch's argument
            }
            // one bin: terms of bin jj into Gc, Tx rows, barrier, reduction of
            // bin jj, receive of bin jj - 1 from Gp
            auto bin = [&](int jj, float2 (&Gc)[SC], const float2 (&Gp)[SC]) {
                const int jb = jb0 + jj;
                const int buf = jj & 1;
                const float jf = (float)(A.j_lo + jb);
                // j G: the sinc's 1/j is applied as 1/j^2 by the finaliser
                if constexpr (EL == 2) {
#pragma unroll
                    for (int s = 0; s < SC; ++s) Gc[s] = green_next_2d(g[s]);
                } else if constexpr (TABLE) {
                    // each term's table read is issued while the previous term
                    // is evaluated (one read ahead keeps three blocks per CU)
                    DeltaFetch fch[2];
                    fch[0] = delta_fetch(s_tab, P, jf * g[0].kap);
#pragma unroll
                    for (int s = 0; s < SC; ++s) {
                        if (s + 1 < SC) fch[(s + 1) & 1] = delta_fetch(s_tab, P, jf * g[s + 1].kap);
                        __builtin_amdgcn_sched_barrier(0);
                        Gc[s] = green_next_fetched(g[s], fch[s & 1]);
                    }
                } else {
#pragma unroll
                    for (int s = 0; s < SC; ++s) Gc[s] = green_next<HASY, TABLE>(A.K, g[s], jf, 1.f, s_tab, P);
                }
#pragma unroll
                for (int s = 0; s < SC; ++s) {
                    if (PAIR) {
                        Gc[s].x += dpp<DPP_XOR1>(Gc[s].x);
                        Gc[s].y += dpp<DPP_XOR1>(Gc[s].y);
                    }
                }
                // branch-free loads (clamped index, then select) keep the bin in
                // one basic block
                float2 W[TT];
#pragma unroll
                for (int t = 0; t < TT; ++t) {
                    const int tt = min(t0 + t, A.n_tx - 1);
                    const float2 w = A.W[((int64_t)jb * A.n_tx + tt) * A.N + e];
                    const bool use = active && t0 + t < A.n_tx;
                    W[t] = make_float2(use ? w.x : 0.f, use ? w.y : 0.f);
                }
                if (PAIR) {
                    // W B split over the pair: the even lane stores Re, the odd
                    // lane Im, together the float2 slot of the pair
                    float* red = reinterpret_cast<float*>(s_red[buf]);
#pragma unroll
                    for (int t = 0; t < TT; ++t) {
                        const float w1 = (tid & 1) ? W[t].y : W[t].x;
                        const float w2 = (tid & 1) ? W[t].x : -W[t].y;
#pragma unroll
                        for (int s = 0; s < SC; ++s)
                            red[2 * (grp * NS + t * SC + s) * RS + n] = fmaf(w1, Gc[s].x, w2 * Gc[s].y);
                    }
                } else {
                    // both lanes of a pair hold the same pair sum and store it
                    // to the same slot
#pragma unroll
                    for (int t = 0; t < TT; ++t)
#pragma unroll
                        for (int s = 0; s < SC; ++s) {
                            float2 p = cmul(W[t], Gc[s]);
                            p.x += dpp<DPP_XOR1>(p.x);
                            p.y += dpp<DPP_XOR1>(p.y);
                            s_red[buf][(grp * NS + t * SC + s) * RS + (n >> 1)] = p;
                        }
                }
                __syncthreads();
                reduce(buf);
                if (jj > 0) receive(jj - 1, buf ^ 1, Gp);
            };
            float2 G0[SC], G1[SC];
            for (int jj = 0; jj < nb; jj += 2) {
                bin(jj, G0, G1);
                if (jj + 1 < nb) bin(jj + 1, G1, G0);
            }
            __syncthreads();
            if (nb > 0) {
                if ((nb - 1) & 1) receive(nb - 1, 1, G1);
                else receive(nb - 1, 0, G0);
            }
            __syncthreads();
        }
        float* out = reinterpret_cast<float*>(A.part) + (int64_t)id * (JT * TT * BS * NA);
        for (int i = tid; i < JT * TT * BS * NA; i += BS) out[i] = s_acc[i];

        if (!A.ticket) break;
        __syncthreads();
        if (tid == 0) s_item = atomicAdd(A.ticket, 1);
        __syncthreads();
        item = s_item;
    }
}

SynthConfig synth_config(int M, int nu, int n_tx, bool has_y, bool table_lds, bool alt)
{
    SynthConfig c{};
    int bg = 64;
    while (bg < M) bg *= 2;
    // probes of fewer than 256 sub-elements: several groups per 256-thread
    // block share its elevation table and barriers
    c.groups = bg < 256 ? 256 / bg : 1;
    c.bs = bg * c.groups;
    // Transmits per group: a pair of transmits costs 1.8x a single one here
    // (fewer scatterers per chunk), so pairs pay for even counts and for 11
    // or more transmits; wider groups (4, 8: 2 scatterers per chunk, 8 or 4
    // bins per set-up) measured slower than single transmits.
    const bool pairs = n_tx >= 2 && (n_tx % 2 == 0 || n_tx >= 11);
    c.tt = (alt ? !pairs && n_tx >= 2 : pairs) ? 2 : 1;
    c.sc = c.tt == 2 ? 4 : SIMUS_SC1;
    c.pair = nu == 2;
    c.jt = synth_jt(c.bs, c.tt, c.pair, table_lds, c.groups);
    c.has_y = has_y;
    return c;
}

template <int BS, int SC, int TT, bool PAIR, int NG>
static SynthKernel synth_kernel_y(const SynthConfig& cfg)
{
    constexpr int JTT = synth_jt(BS, TT, PAIR, true, NG);    // table in LDS
    constexpr int JTN = synth_jt(BS, TT, PAIR, false, NG);   // no table
    if (cfg.sc != SC) return nullptr;
    const bool with_table = !cfg.has_y && !cfg.dim2 && cfg.table;
    if (cfg.jt != (with_table ? JTT : JTN)) return nullptr;
    if (cfg.has_y) return k_synth<BS, SC, JTN, TT, true, 0, PAIR, NG>;
    if (cfg.dim2) return k_synth<BS, SC, JTN, TT, false, 2, PAIR, NG>;
    if (cfg.table) return k_synth<BS, SC, JTT, TT, false, 1, PAIR, NG>;
    return k_synth<BS, SC, JTN, TT, false, 0, PAIR, NG>;
}

template <int BS, bool PAIR, int NG>
static SynthKernel synth_kernel_bs(const SynthConfig& cfg)
{
    switch (cfg.tt) {
    case 1: return synth_kernel_y<BS, SIMUS_SC1, 1, PAIR, NG>(cfg);
    case 2: return synth_kernel_y<BS, 4, 2, PAIR, NG>(cfg);
    default: return nullptr;
    }
}

template <bool PAIR>
static SynthKernel synth_kernel_pair(const SynthConfig& cfg)
{
    if (cfg.bs == 256 && cfg.groups == 1) return synth_kernel_bs<256, PAIR, 1>(cfg);
    if (cfg.bs == 256 && cfg.groups == 2) return synth_kernel_bs<256, PAIR, 2>(cfg);
    if (cfg.bs == 256 && cfg.groups == 4) return synth_kernel_bs<256, PAIR, 4>(cfg);
    if (cfg.bs == 512 && cfg.groups == 1) return synth_kernel_bs<512, PAIR, 1>(cfg);
    if (cfg.bs == 1024 && cfg.groups == 1) return synth_kernel_bs<1024, PAIR, 1>(cfg);
    return nullptr;
}

SynthKernel synth_kernel(const SynthConfig& cfg)
{
    return cfg.pair ? synth_kernel_pair<true>(cfg) : synth_kernel_pair<false>(cfg);
}

hipError_t launch_synth(const SynthConfig& cfg, const SynthArgs& a, hipStream_t st)
{
    if (cfg.grid <= 0) return hipSuccess;
    const SynthKernel k = synth_kernel(cfg);
    if (!k) return hipErrorInvalidValue;
    SynthArgs arg = a;
    void* args[] = {&arg};
    return hipLaunchKernel(reinterpret_cast<const void*>(k), dim3(cfg.grid), dim3(cfg.bs), args, 0, st);
}

// ---------------------------------------------------------------------------
// Finaliser: spec[p][t][e][b] = P_b sum_items sum_g sum_{mu<nu} part[item][jj][t%TT][g BG + e nu + mu]
// (Eqs. 33-34), divided by j^2, j = j_lo + b, when inv_j2 is set (partials
// of j G terms).  Items of phantom p are ordered (tg, bt, slice); the sum
// over slices is split over FIN_K lanes in a fixed pattern, so the result is
// deterministic.
// ---------------------------------------------------------------------------
constexpr int FIN_K = 8;
__global__ __launch_bounds__(256) void k_finalize(float2* __restrict__ spec, const float2* __restrict__ part,
                                                  const float2* __restrict__ pw, const int32_t* __restrict__ pbase,
                                                  const int32_t* __restrict__ nsl, int n_ph, int n_tx, int N, int nu,
                                                  int n_bins, int bs, int groups, int tt, int jt, int n_bt,
                                                  int j_lo, bool inv_j2)
{
    // FIN_K neighbouring lanes share one output: lane k sums the slices
    // k, k + FIN_K, ... in order, and a fixed butterfly combines the lanes,
    // so the result does not depend on scheduling
    const int bg = bs / groups;
    const int64_t total = (int64_t)n_ph * n_tx * n_bins * N;
    const int kl = threadIdx.x % FIN_K;
    const int64_t stride = (int64_t)gridDim.x * (blockDim.x / FIN_K);
    for (int64_t i = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) / FIN_K; i < total; i += stride) {
        const int e = (int)(i % N);
        int64_t r = i / N;
        const int b = (int)(r % n_bins);
        r /= n_bins;
        const int t = (int)(r % n_tx);
        const int p = (int)(r / n_tx);
        const int tg = t / tt, tl = t % tt, bt = b / jt, jj = b % jt;
        const int ns = nsl[p];
        const int64_t first = pbase[p] + ((int64_t)tg * n_bt + bt) * ns;
        float sx = 0.f, sy = 0.f;
        for (int sl = kl; sl < ns; sl += FIN_K) {
            const float2* src = part + (first + sl) * ((int64_t)jt * tt * bs) + (jj * tt + tl) * bs + e * nu;
            for (int g = 0; g < groups; ++g)
                for (int mu = 0; mu < nu; ++mu) {
                    sx += src[g * bg + mu].x;
                    sy += src[g * bg + mu].y;
                }
        }
#pragma unroll
        for (int m = 1; m < FIN_K; m <<= 1) {
            sx += __shfl_xor(sx, m, FIN_K);
            sy += __shfl_xor(sy, m, FIN_K);
        }
        if (kl == 0) {
            float2 w = pw[b];
            if (inv_j2) {
                // partials of j G terms (two per product): divide by j^2
                const float j = (float)(j_lo + b);
                const float s = 1.f / (j * j);
                w = make_float2(w.x * s, w.y * s);
            }
            spec[(((int64_t)p * n_tx + t) * N + e) * n_bins + b] =
                make_float2(w.x * sx - w.y * sy, w.x * sy + w.y * sx);
        }
    }
}

hipError_t launch_finalize(float2* spec, const float2* part, const float2* pw,
                           const int32_t* pbase, const int32_t* nsl, int n_ph, int n_tx, int N,
                           int nu, int n_bins, int bs, int groups, int tt, int jt, int n_bt,
                           int j_lo, bool inv_j2, hipStream_t st)
{
    if (groups < 1 || bs % groups) return hipErrorInvalidValue;
    const int64_t total = (int64_t)n_ph * n_tx * n_bins * N;
    if (total == 0) return hipSuccess;
    const int grid = (int)std::min<int64_t>((total * FIN_K + 255) / 256, 16384);
    hipLaunchKernelGGL(k_finalize, dim3(grid), dim3(256), 0, st, spec, part, pw, pbase, nsl, n_ph,
                       n_tx, N, nu, n_bins, bs, groups, tt, jt, n_bt, j_lo, inv_j2);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Inverse transform (Eq. 1): rf[c][q] = sum_b Re(spec[c][b] e^{-2 pi i j q / nfft}),
// j = j_lo + b.  Thread = sample q; the phase factor of bin j is stepped to
// bin j + 1 by one complex product with e^{2 pi i q / nfft} and re-anchored
// every IDFT_ANCHOR bins from the exact integer angle index j q mod nfft
// (hardware sine/cosine of turns in [-1/2, 1/2)), so rounding grows over at
// most IDFT_ANCHOR steps.  One block per (channel, 256 samples); the
// channel's spectrum is staged in LDS in chunks.
// ---------------------------------------------------------------------------
constexpr int DFT_CHUNK = 4096;
constexpr int IDFT_ANCHOR = 32;

__global__ __launch_bounds__(256) void k_idft(float* __restrict__ rf, const float2* __restrict__ spec,
                                              int64_t ch0, int n_bins, int j_lo, int nfft, int n_t)
{
    __shared__ float2 s_x[DFT_CHUNK];
    const int64_t ch = ch0 + blockIdx.y;
    const float2* X = spec + ch * n_bins;
    const int q = blockIdx.x * blockDim.x + threadIdx.x;
    const bool live = q < n_t;
    const int qn = (live ? q : 0) % nfft;
    const float inv_n = 1.f / (float)nfft;
    const int half = nfft / 2;
    auto turns = [&](int m) { return (float)(m >= half ? m - nfft : m) * inv_n; };
    // per-bin step of the phase: 2 pi q / nfft
    const float dc = cos_turns(turns(qn)), ds = sin_turns(turns(qn));
    int m = (int)(((int64_t)j_lo * qn) % nfft);   // j q mod nfft at the next bin
    float acc0 = 0.f, acc1 = 0.f;
    for (int c0 = 0; c0 < n_bins; c0 += DFT_CHUNK) {
        const int cn = min(DFT_CHUNK, n_bins - c0);
        __syncthreads();
        for (int b = threadIdx.x; b < cn; b += blockDim.x) s_x[b] = X[c0 + b];
        __syncthreads();
        for (int b0 = 0; b0 < cn; b0 += IDFT_ANCHOR) {
            const int nb = min(IDFT_ANCHOR, cn - b0);
            float ec = cos_turns(turns(m)), es = sin_turns(turns(m));
            int b = 0;
            for (; b + 1 < nb; b += 2) {
                const float2 x0 = s_x[b0 + b], x1 = s_x[b0 + b + 1];
                acc0 = fmaf(x0.x, ec, fmaf(x0.y, es, acc0));
                float c1 = ec * dc - es * ds, s1 = fmaf(es, dc, ec * ds);
                acc1 = fmaf(x1.x, c1, fmaf(x1.y, s1, acc1));
                ec = c1 * dc - s1 * ds;
                es = fmaf(s1, dc, c1 * ds);
            }
            if (b < nb) {
                const float2 x0 = s_x[b0 + b];
                acc0 = fmaf(x0.x, ec, fmaf(x0.y, es, acc0));
            }
            m = (int)(((int64_t)m + (int64_t)nb * qn) % nfft);
        }
    }
    if (live) rf[ch * n_t + q] = acc0 + acc1;
}

hipError_t launch_idft(float* rf, const float2* spec, int64_t n_chan, int n_bins, int j_lo,
                       int nfft, int n_t, hipStream_t st)
{
    if (n_chan == 0 || n_t == 0) return hipSuccess;
    for (int64_t c0 = 0; c0 < n_chan; c0 += 65535) {
        const unsigned nc = (unsigned)std::min<int64_t>(65535, n_chan - c0);
        hipLaunchKernelGGL(k_idft, dim3((n_t + 255) / 256, nc), dim3(256), 0, st, rf, spec, c0,
                           n_bins, j_lo, nfft, n_t);
        const hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}

__global__ void k_zero_i32(int32_t* p, int n)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = 0;
}

hipError_t launch_zero_i32(int32_t* p, int n, hipStream_t st)
{
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_zero_i32, dim3((n + 255) / 256), dim3(256), 0, st, p, n);
    return hipGetLastError();
}

}  // namespace simus
