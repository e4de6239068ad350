// Device-side argument blocks and launch entry points of libsimus kernels.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace simus {

// Constants of four Gaussians of the elevation aperture (Eq. 12; Eq. 18's
// by default), scaled by 1/h^2: the unrolled path of four-Gaussian sets.
struct Gauss4 {
    float a[4];    // Re(B_g) / h^2   (> 0)
    float a2[4];   // a^2
    float b[4];    // Im(B_g) / h^2
    float Ar[4];   // sqrt(pi) Re(A_g)
    float Ai[4];   // sqrt(pi) Im(A_g)
};

// Per-call model constants.  All "per bin" rates are multiplied by the
// absolute bin index j (f_j = j df).
struct ModelConst {
    double turns_per_bin_m;  // df / c: phase turns of exp(i k r) per bin per metre
    float att_per_bin_m;     // -(alpha_dB / 8.69) (df / 1e4) log2(e): log2 of exp(-k_a r) per bin per metre
    float sinc_per_bin;      // df b_sub / c: sinc argument in turns per bin per unit sin(theta)
    float q_per_bin;         // pi df / c: Im(alpha_g) shift per bin per (1/R_f - 1/r)
    float k_per_bin;         // 2 pi df / c
    float ka_per_bin;        // (alpha_dB / 8.69) df / 1e4: k_a per bin [Np/m]
    float b_sub;             // sub-element half-width b / nu
    float inv_rf;            // 1 / R_f (0 for an unfocused element)
    float zeta;              // baffle impedance ratio
    int32_t baffle;          // 0 soft, 1 rigid, 2 zeta
    int32_t dim2;            // 2-D acoustics: amplitude 1/sqrt(r), no elevation term
    int32_t ng;              // Gaussians of the elevation aperture (Eq. 12)
    Gauss4 g;                // the set when ng == 4
    const float4* gset;      // device [ng]: (Re B/h^2, Im B/h^2, sqrt(pi) Re A, sqrt(pi) Im A)
};

// The half-angle sinc of the pair set-up, sinc(theta / 2) with |theta / 2| <=
// pi sinc_per_bin, is its Taylor series when sinc_per_bin is below this limit
// (argument below 1); the matrix-core kernels assume it (the host sends other
// problems to the vector path).
constexpr float SINC_TAYLOR_LIMIT = 0.3f;

// Elevation-term table (y = 0): DELTA_NT cubic intervals in w = q / (|q| + L).
// 256 intervals: worst interpolation error 2.5e-6 of max |delta| over the
// 128-element workload's range (median 2.4e-7, the FP32 evaluation level;
// 512 intervals: 4.4e-7), and 8 KiB of LDS, which lets the single-transmit
// synthesis take 26 bins per tile instead of 18 at three blocks per CU.
constexpr int DELTA_NT = 256;
// float4 index of the first and second halves of interval k's coefficients:
// two arrays of DELTA_NT, so that lanes reading neighbouring intervals fall
// on different LDS banks
__host__ __device__ constexpr int dtab_a(int k) { return k; }
__host__ __device__ constexpr int dtab_b(int k) { return DELTA_NT + k; }

struct DeltaParams {
    float L;       // map scale
    float u0;      // -w_lo / dw
    float inv_dw;  // 1 / dw
    float umax;    // DELTA_NT - 2^-8
    float kscale;  // inv_dw / L: q -> b = q inv_dw / L (delta_fetch's argument)
    float dw;      // 1 / inv_dw
};

// Sub-element frames, device arrays of length M = nu N.
struct SubGeo {
    const double* xc;
    const double* zc;
    const float* tx;
    const float* tz;
    const float* nx;
    const float* nz;
};

// One work item of the synthesis: scatterers [s_begin, s_end) of a phantom,
// bin tile `bt`, transmit group `tg`.
struct Item {
    int32_t phantom;
    int32_t s_begin;
    int32_t s_end;
    int32_t tile;  // bt | (tg << 16)
};

struct SynthArgs {
    const float* x;
    const float* y;     // may be null (y = 0)
    const float* z;
    const float* refl;
    SubGeo sub;
    const float2* W;    // [n_bins][n_tx][N] transmit weights W e^{i w tau}
    const float2* WT;   // matrix-core path: [n_bins][n_tg][NE][16] the same weights by
                        // transmit group, element slot and column, zero-padded
    const Item* items;
    const int32_t* order; // [n_items] draw order: item ids, costliest first
    int32_t n_items;
    int32_t* ticket;    // persistent launch: work counter (zeroed before launch)
    float2* part;       // [n_items][JT][TT][BS] per-sub-element partial spectra
    const float4* dtab; // [2 * DELTA_NT] elevation table (y = 0 path), or null
    const DeltaParams* dpar;
    int32_t M, nu, N, n_tx, n_bins, j_lo;
    ModelConst K;
};

struct SynthConfig {
    int bs;      // threads per block: groups x sub-element slots (a power of 2 >= M)
    int groups;  // vector path: sub-element groups per block (1, 2 or 4)
    int tt;      // transmits per group
    int sc;      // scatterers per chunk
    int jt;      // bins per tile
    bool has_y;
    bool table;  // elevation term from the table (requires !has_y)
    bool dim2;   // 2-D acoustics: no elevation term (vector path skips the table)
    bool persistent;
    bool pair;   // nu = 2: element sums of lane pairs, one float accumulator per lane
    bool mfma;   // transmit contraction on the matrix cores (synth_mfma.hip)
    int ne;      // matrix-core path: element slots (64 or 128)
    int nx;      // matrix-core path: receive sums per column tile (2 or 3)
    bool wt;     // matrix-core path: the kernel reads the padded weight table WT
    bool bf;     // matrix-core path: products in bf16 high/low parts (k_synth_mb)
    int grid;    // blocks launched (persistent: resident blocks)
};

// Adjoint work item: scatterers [s_begin, s_end) (at most 256) of one
// phantom, bin range `range` (bins range * range_bins ...).
struct AdjItem {
    int32_t phantom;
    int32_t s_begin;
    int32_t s_end;
    int32_t range;
};

struct AdjArgs {
    const float* x;
    const float* y;      // may be null
    const float* z;
    const float* refl;
    SubGeo sub;
    const float2* W;     // [n_bins][n_tx][N]
    const float2* lam;   // [n_ph][n_bins][n_tx][N] residual spectra
    const float2* pw;    // [n_bins] S_P S_T
    const float2* WL;    // k_adjoint_mq: [n_ph][n_bins][128][16] W of 8 transmits, then Lam, zero-padded
    const AdjItem* items;
    float4* part;        // [n_ranges][S_total] (dR, dX, dY, dZ) before R_s
    const float4* dtab;
    const DeltaParams* dpar;
    int64_t S_total;
    int32_t M, nu, N, n_tx, n_bins, j_lo, range_bins;
    ModelConst K;
};

struct AdjConfig {
    int tt;          // transmits per group (matrix-core path: columns per half)
    int jt;          // bins per tile (matrix-core path: bins per set-up)
    int scatterers;  // scatterers per work item (256 on the vector path)
    bool has_y;
    bool table;
    bool mfma;       // matrix-core adjoint (adjoint_mfma.hip)
    bool pair;       // matrix-core path: nu = 2
    bool wl;         // matrix-core path: k_adjoint_mq (four bins per step, columns from WL)
    bool bf;         // k_adjoint_mq: products in bf16 high/low parts
};

AdjConfig adjoint_config(int n_tx, bool has_y);
hipError_t launch_adjoint(const AdjConfig& c, const AdjArgs& a, int n_items, hipStream_t st);
bool adjoint_mt_supported(int M, int N, int n_tx);
AdjConfig adjoint_mt_config(int M, int N, int n_tx, bool has_y);
hipError_t launch_adjoint_mt(const AdjConfig& c, const AdjArgs& a, int n_items, hipStream_t st);
hipError_t launch_wltable(float2* WL, const float2* W, const float2* lam, int n_ph, int n_bins, int n_tx,
                          int N, bool bf16, hipStream_t st);
hipError_t launch_adjoint_reduce(const float4* part, int n_ranges, int64_t S, const float* refl,
                                 float* dR, float* dX, float* dY, float* dZ, hipStream_t st);
hipError_t launch_dft_t(float2* lam, const float* rho, int64_t n_chan, int n_bins, int j_lo, int nfft,
                        int n_t, int n_tx, int N, hipStream_t st);

struct FieldArgs {
    const float* X;
    const float* Y;      // may be null
    const float* Z;
    SubGeo sub;
    const float2* W;     // [n_bins][N] transmit weights
    const float2* ptx;   // [n_bins] S_P sqrt(S_T)
    float* part;         // [n_ranges][n_pts] partial sums of |P|^2
    const float4* dtab;
    const DeltaParams* dpar;
    int64_t n_pts;
    int32_t M, nu, N, n_bins, j_lo, n_ranges;
    ModelConst K;
};

// Frequencies per (point, sub-element) set-up of the field kernel, at most:
// a block's frequency range is split into tiles of nearly equal size.  Timed
// on the 64-element, 256 x 256-point, 402-frequency field: 8 -> 1.74 ms,
// 16 -> 1.58 ms, 32 -> 1.66 ms (registers halve the occupancy); with the
// balanced ranges and tiles, 16 -> 1.48 ms, 24 -> 1.49 ms, 32 -> 1.70 ms.
// On the 128-element, 705-frequency field, whose 30 ranges of 23-24 bins
// took two tiles each at 16: 16 -> 9.57 ms, 20 -> 9.86, 24 -> 8.66 (107
// registers, four waves per SIMD), 28 -> 8.72.
constexpr int PFIELD_JT = 24;
hipError_t launch_pfield(const FieldArgs& a, bool has_y, bool table, int n_ranges, hipStream_t st);
hipError_t launch_pfield_reduce(const float* part, int n_ranges, int64_t n_pts, float dw, float* out,
                                hipStream_t st);

// Picks bs/tt/sc/jt for M = nu N sub-elements and a transmit count.
// table_lds: the synthesis holds the elevation table in LDS (y = 0, 3-D,
// table not disabled)
// alt: the other transmit-group size (single transmits instead of pairs, or
// pairs instead of single transmits), the alternative the autotuner tries
SynthConfig synth_config(int M, int nu, int n_tx, bool has_y, bool table_lds, bool alt = false);

hipError_t launch_wtable(float2* W, const double* delays, const float* apod, int n_bins, int n_tx,
                         int N, int j_lo, double df, hipStream_t st);
// The weights in the matrix-core kernels' layout: WT[b][g][e][c] = W of
// transmit 16 g + c and element e at bin b, zero for e >= N or a transmit
// past n_tx; ne element slots, n_tg groups of 16 columns.
hipError_t launch_wtable_mt(float2* WT, const double* delays, const float* apod, int n_bins, int n_tx,
                            int N, int ne, int tpg, int n_tg, int j_lo, double df, bool bf16, hipStream_t st);
// The synthesis kernel instance a configuration runs (nullptr if none), for
// the launch and for occupancy queries (blocks of cfg.bs threads, or 512 on
// the matrix-core path).
using SynthKernel = void (*)(SynthArgs);
SynthKernel synth_kernel(const SynthConfig& cfg);
hipError_t launch_synth(const SynthConfig& cfg, const SynthArgs& a, hipStream_t st);
bool mt_supported(int M, int N, int n_tx);
// alt: the alternative group width (16 instead of 32 transmit columns for
// 128 element slots, 64 instead of 32 for 64), which the autotuner tries
SynthConfig mt_config(int M, int N, int n_tx, bool has_y, bool alt = false, bool fp32 = false);
SynthKernel synth_mt_kernel(const SynthConfig& cfg);
hipError_t launch_synth_mt(const SynthConfig& cfg, const SynthArgs& a, hipStream_t st);
// inv_j2: the partials are of j G terms (both synthesis paths) and are
// divided by j^2, j = j_lo + bin.
// bs partial slots per (bin, transmit) of an item, in `groups` blocks of
// bs / groups slots, each holding nu slots per element
hipError_t launch_finalize(float2* spec, const float2* part, const float2* pw,
                           const int32_t* pbase, const int32_t* nsl, int n_ph, int n_tx, int N,
                           int nu, int n_bins, int bs, int groups, int tt, int jt, int n_bt,
                           int j_lo, bool inv_j2, hipStream_t st);
hipError_t launch_idft(float* rf, const float2* spec, int64_t n_chan, int n_bins, int j_lo,
                       int nfft, int n_t, hipStream_t st);
hipError_t launch_zero_i32(int32_t* p, int n, hipStream_t st);

// Scratch of simus_rf_noalloc: one static device array per GPU of this many
// bytes (noalloc.hip).  noalloc_scratch gives its device address on the
// current device (looked up on the device's first call, then kept).
constexpr size_t NOALLOC_SCRATCH_BYTES = size_t(64) << 20;
hipError_t noalloc_scratch(char** ptr);

// Range of sub-element-to-scatterer distances (as float bits, [0] = min,
// [1] = max) over all pairs, then the elevation table for the call's range
// of q = (pi f / c)(1/R_f - 1/r), f over the evaluated band.
hipError_t launch_rrange(uint32_t* rr, const float* x, const float* y, const float* z, int64_t n,
                         const SubGeo& sub, int M, hipStream_t st);
// unit: every interval holds delta = 1 (2-D acoustics, no elevation term).
// gset64: device [ng][4] FP64 (Re A, Im A, Re B, Im B) of the Gaussians.
hipError_t launch_dtable(float4* tab, DeltaParams* par, const uint32_t* rr, const ModelConst& K,
                         const double* gset64, double height, int j_first, int j_last, bool unit,
                         hipStream_t st);

}  // namespace simus
