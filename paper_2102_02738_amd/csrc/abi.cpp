// C ABI of libsimus (include/simus.h): validation, planning, workspace and
// kernel orchestration.  No C++ exception crosses the ABI.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <map>
#include <memory>
#include <mutex>
#include <string>
#include <vector>

#include "kernels.hpp"
#include "plan.hpp"
#include "simus.h"

namespace simus {
namespace {

thread_local std::string g_last_error;

int fail(int code, const std::string& msg)
{
    g_last_error = msg;
    return code;
}

void hip_check(hipError_t e, const char* what)
{
    if (e != hipSuccess)
        throw Error{SIMUS_EHIP, std::string(what) + ": " + hipGetErrorString(e)};
}

bool log_enabled()
{
    static const bool on = [] {
        const char* v = std::getenv("SIMUS_LOG");
        return v && v[0] && v[0] != '0';
    }();
    return on;
}

// ---------------------------------------------------------------- kernel timing
enum Kind { K_SYNTH, K_WTABLE, K_FINALIZE, K_IDFT, K_DFT, K_ADJ, K_ADJRED, K_PFIELD, K_GRAPH, K_COUNT };
const char* const kKindNames[K_COUNT] = {"synth",   "wtable",         "finalize", "idft", "dft",
                                         "adjoint", "adjoint_reduce", "pfield",   "graph"};

// Set while this thread captures a graph or runs simus_rf_noalloc: launches
// are then not bracketed by timing events (no event is created).
thread_local bool t_untimed = false;

struct Untimed {
    Untimed() { t_untimed = true; }
    ~Untimed() { t_untimed = false; }
};

struct Profiler {
    std::mutex mu;
    bool on = false;
    struct Rec {
        int kind;
        hipEvent_t a, b;
    };
    std::vector<Rec> pending;
    std::vector<hipEvent_t> pool;
    double total[K_COUNT] = {};
    int64_t count[K_COUNT] = {};

    hipEvent_t take()
    {
        if (!pool.empty()) {
            hipEvent_t e = pool.back();
            pool.pop_back();
            return e;
        }
        hipEvent_t e = nullptr;
        hip_check(hipEventCreate(&e), "hipEventCreate");
        return e;
    }
    // Waits for every pending record and folds it into the totals.
    void drain()
    {
        for (const Rec& r : pending) {
            float ms = 0.f;
            hip_check(hipEventSynchronize(r.b), "hipEventSynchronize");
            hip_check(hipEventElapsedTime(&ms, r.a, r.b), "hipEventElapsedTime");
            total[r.kind] += ms;
            count[r.kind] += 1;
            pool.push_back(r.a);
            pool.push_back(r.b);
        }
        pending.clear();
    }
};

Profiler g_prof;

// Runs `launch` (which enqueues one kernel on st), bracketed by events when
// timing is enabled.
template <class F>
hipError_t timed(Kind k, hipStream_t st, F&& launch)
{
    if (t_untimed) return launch();
    {
        std::lock_guard<std::mutex> lk(g_prof.mu);
        if (!g_prof.on) return launch();
    }
    hipEvent_t a, b;
    {
        std::lock_guard<std::mutex> lk(g_prof.mu);
        a = g_prof.take();
        b = g_prof.take();
    }
    hip_check(hipEventRecord(a, st), "hipEventRecord");
    const hipError_t e = launch();
    hip_check(hipEventRecord(b, st), "hipEventRecord");
    std::lock_guard<std::mutex> lk(g_prof.mu);
    g_prof.pending.push_back({k, a, b});
    return e;
}

// ---------------------------------------------------------------- workspace
// One device arena and one pinned staging buffer per (device, stream).  The
// staging buffer is rewritten only after the previous upload from it has
// completed (event), so no call waits on kernels.
struct Arena {
    char* dev = nullptr;
    size_t dev_cap = 0;
    char* host = nullptr;
    size_t host_cap = 0;
    hipEvent_t staged = nullptr;
    bool staged_pending = false;
};

std::mutex g_mu;
std::map<std::pair<int, uintptr_t>, Arena> g_arenas;

struct Layout {
    size_t size = 0;
    size_t add(size_t bytes)
    {
        const size_t off = size;
        size += (bytes + 255) & ~size_t(255);
        return off;
    }
};

Arena& arena_for(hipStream_t st, size_t dev_bytes, size_t host_bytes)
{
    int dev = 0;
    hip_check(hipGetDevice(&dev), "hipGetDevice");
    std::lock_guard<std::mutex> lk(g_mu);
    Arena& a = g_arenas[{dev, reinterpret_cast<uintptr_t>(st)}];
    if (!a.staged) hip_check(hipEventCreateWithFlags(&a.staged, hipEventDisableTiming), "hipEventCreate");
    if (a.staged_pending) {
        hip_check(hipEventSynchronize(a.staged), "hipEventSynchronize");
        a.staged_pending = false;
    }
    if (dev_bytes > a.dev_cap) {
        if (a.dev) {
            hip_check(hipStreamSynchronize(st), "hipStreamSynchronize");
            hip_check(hipFree(a.dev), "hipFree");
            a.dev = nullptr;
            a.dev_cap = 0;
        }
        const size_t cap = std::max(dev_bytes, size_t(1) << 20);
        if (hipMalloc(&a.dev, cap) != hipSuccess) {
            a.dev = nullptr;
            (void)hipGetLastError();
            throw Error{SIMUS_ENOMEM, "device workspace allocation failed"};
        }
        a.dev_cap = cap;
    }
    if (host_bytes > a.host_cap) {
        if (a.host) hip_check(hipHostFree(a.host), "hipHostFree");
        a.host = nullptr;
        a.host_cap = 0;
        const size_t cap = std::max(host_bytes, size_t(1) << 16);
        if (hipHostMalloc(reinterpret_cast<void**>(&a.host), cap, hipHostMallocDefault) != hipSuccess) {
            a.host = nullptr;
            (void)hipGetLastError();
            throw Error{SIMUS_ENOMEM, "pinned staging allocation failed"};
        }
        a.host_cap = cap;
    }
    return a;
}

void upload(Arena& a, size_t bytes, hipStream_t st)
{
    if (bytes == 0) return;
    hip_check(hipMemcpyAsync(a.dev, a.host, bytes, hipMemcpyHostToDevice, st), "hipMemcpyAsync");
    hip_check(hipEventRecord(a.staged, st), "hipEventRecord");
    a.staged_pending = true;
}

template <class T>
T* at(char* base, size_t off)
{
    return reinterpret_cast<T*>(base + off);
}

// ---------------------------------------------------------------- model constants
ModelConst model_constants(const Probe& P, const Band& B)
{
    ModelConst K{};
    const double df = B.df;
    K.turns_per_bin_m = df / P.c;
    // Eq. (40): k_a = alpha/8.69 * f / 1e4 [Np/m]; exp(-k_a r) = 2^(log2(e) * -k_a r)
    K.att_per_bin_m = (float)(-(P.alpha_db / 8.69) * (df / 1e4) * M_LOG2E);
    K.sinc_per_bin = (float)(df * (0.5 * P.width / P.nu) / P.c);
    K.q_per_bin = (float)(M_PI * df / P.c);
    K.k_per_bin = (float)(2 * M_PI * df / P.c);
    K.ka_per_bin = (float)((P.alpha_db / 8.69) * (df / 1e4));
    K.b_sub = (float)(0.5 * P.width / P.nu);
    K.inv_rf = std::isinf(P.elev_focus) ? 0.f : (float)(1.0 / P.elev_focus);
    K.zeta = (float)P.zeta;
    K.baffle = P.baffle;
    K.dim2 = P.dim2 ? 1 : 0;
    // the Gaussians of Eq. (12) (Eq. 18's four by default): the unrolled
    // constants when there are four; the device table (gset, set per launch
    // from the workspace) serves any count
    K.ng = (int32_t)P.gA.size();
    const double h2 = P.height * P.height;
    const double sq_pi = std::sqrt(M_PI);
    for (int g = 0; g < 4 && K.ng == 4; ++g) {
        const double a = P.gB[g].real() / h2;
        K.g.a[g] = (float)a;
        K.g.a2[g] = (float)(a * a);
        K.g.b[g] = (float)(P.gB[g].imag() / h2);
        K.g.Ar[g] = (float)(sq_pi * P.gA[g].real());
        K.g.Ai[g] = (float)(sq_pi * P.gA[g].imag());
    }
    K.gset = nullptr;
    return K;
}

struct Phantoms {
    int n = 0;
    std::vector<int64_t> off;
    int64_t total = 0;
};

Phantoms check_phantoms(int32_t n_ph, const int64_t* offs)
{
    if (n_ph < 1) throw Error{SIMUS_EINVAL, "n_phantoms must be >= 1"};
    if (!offs) throw Error{SIMUS_EINVAL, "scat_offsets must be non-NULL"};
    if (offs[0] != 0) throw Error{SIMUS_EINVAL, "scat_offsets[0] must be 0"};
    Phantoms ph;
    ph.n = n_ph;
    ph.off.assign(offs, offs + n_ph + 1);
    for (int p = 0; p < n_ph; ++p)
        if (offs[p + 1] < offs[p]) throw Error{SIMUS_EINVAL, "scat_offsets must be non-decreasing"};
    ph.total = offs[n_ph];
    if (ph.total >= (int64_t(1) << 31)) throw Error{SIMUS_EINVAL, "too many scatterers (>= 2^31)"};
    return ph;
}

// ---------------------------------------------------------------- common preparation
// Validated call description shared by the forward and adjoint paths.
struct Common {
    Probe P;
    Band B;
    SubElements S;
    Phantoms ph;
    ModelConst K;
    int n_tx = 0;
    bool has_y = false, table = false;
};

Common make_common(const simus_probe* probe, const simus_medium* medium, const simus_options* opt,
                   int32_t n_tx, const double* delays, const float* apod, int32_t n_ph,
                   const int64_t* offs, bool has_y)
{
    Common C;
    C.P = make_probe(probe, medium, opt);
    check_transmits(C.P, n_tx, delays, apod);
    C.ph = check_phantoms(n_ph, offs);
    if (opt->nfft <= 0) throw Error{SIMUS_EINVAL, "options.nfft must be > 0 (see simus_rf_grid)"};
    if (opt->n_t > opt->nfft) throw Error{SIMUS_EINVAL, "options.n_t must be <= nfft"};
    C.B = make_band(C.P, opt->nfft, opt->n_t);
    C.S = sub_elements(C.P);
    C.K = model_constants(C.P, C.B);
    C.n_tx = n_tx;
    C.has_y = has_y;
    if (C.P.dim2 && has_y) throw Error{SIMUS_EINVAL, "y must be NULL with SIMUS_FLAG_2D"};
    // 2-D: the (unit) table path carries the absent elevation term
    C.table = C.P.dim2 || (!C.has_y && !(opt->flags & SIMUS_FLAG_NO_DELTA_TABLE));
    return C;
}

void check_scatterers(const Common& C, const float* x, const float* y, const float* z, const float* refl)
{
    if (C.ph.total > 0 && (!x || !z || !refl)) throw Error{SIMUS_EINVAL, "x, z and refl must be non-NULL"};
    if (C.ph.total > 0 && C.has_y && !y) throw Error{SIMUS_EINVAL, "y must be non-NULL for this plan"};
    if (!C.has_y && y) throw Error{SIMUS_EINVAL, "y must be NULL for this plan (created without y)"};
}

Common make_common(const simus_probe* probe, const simus_medium* medium, const simus_options* opt,
                   int32_t n_tx, const double* delays, const float* apod, int32_t n_ph,
                   const int64_t* offs, const float* x, const float* y, const float* z,
                   const float* refl)
{
    Common C = make_common(probe, medium, opt, n_tx, delays, apod, n_ph, offs, y != nullptr);
    check_scatterers(C, x, y, z, refl);
    return C;
}

// Host tables uploaded by every call, and device tables built on the device.
struct CommonLayout {
    size_t xc, zc, tx, tz, nx, nz, dl, ap, pw, gs, gd;   // upload region
    size_t W, rr, dt, dp;                                // device-only region
};

void layout_upload(Layout& up, CommonLayout& L, const Common& C)
{
    const int M = C.P.M, TN = C.n_tx * C.P.N;
    L.xc = up.add(sizeof(double) * M);
    L.zc = up.add(sizeof(double) * M);
    L.tx = up.add(sizeof(float) * M);
    L.tz = up.add(sizeof(float) * M);
    L.nx = up.add(sizeof(float) * M);
    L.nz = up.add(sizeof(float) * M);
    L.dl = up.add(sizeof(double) * TN);
    L.ap = up.add(sizeof(float) * TN);
    L.pw = up.add(sizeof(float2) * std::max(C.B.n_bins, 1));
    L.gs = up.add(sizeof(float4) * C.K.ng);
    L.gd = up.add(sizeof(double) * 4 * C.K.ng);
}

void layout_device(Layout& dv, CommonLayout& L, const Common& C)
{
    L.W = dv.add(sizeof(float2) * size_t(std::max(C.B.n_bins, 1)) * C.n_tx * C.P.N);
    L.rr = dv.add(sizeof(uint32_t) * 4);
    L.dt = dv.add(sizeof(float4) * 2 * DELTA_NT);
    L.dp = dv.add(sizeof(DeltaParams));
}

void fill_upload(char* h, const CommonLayout& L, const Common& C, const double* delays,
                 const float* apod)
{
    for (int m = 0; m < C.P.M; ++m) {
        at<double>(h, L.xc)[m] = C.S.xc[m];
        at<double>(h, L.zc)[m] = C.S.zc[m];
        at<float>(h, L.tx)[m] = (float)C.S.tx[m];
        at<float>(h, L.tz)[m] = (float)C.S.tz[m];
        at<float>(h, L.nx)[m] = (float)C.S.nx[m];
        at<float>(h, L.nz)[m] = (float)C.S.nz[m];
    }
    for (int i = 0; i < C.n_tx * C.P.N; ++i) {
        at<double>(h, L.dl)[i] = delays[i];
        at<float>(h, L.ap)[i] = apod ? apod[i] : 1.f;
    }
    // the Gaussians of Eq. (12): scaled FP32 for the direct evaluation, FP64
    // for the elevation table
    const double h2 = C.P.height * C.P.height;
    for (int g = 0; g < C.K.ng; ++g) {
        const std::complex<double> A = C.P.gA[g], B = C.P.gB[g];
        at<float4>(h, L.gs)[g] = make_float4((float)(B.real() / h2), (float)(B.imag() / h2),
                                             (float)(std::sqrt(M_PI) * A.real()),
                                             (float)(std::sqrt(M_PI) * A.imag()));
        double* gd = at<double>(h, L.gd) + 4 * g;
        gd[0] = A.real();
        gd[1] = A.imag();
        gd[2] = B.real();
        gd[3] = B.imag();
    }
    // two-way spectral weight (Eqs. 28, 34); in 2-D with the factor 2b of Eq. (38)
    const double f2 = C.P.dim2 ? C.P.width : 1.0;
    for (int b = 0; b < C.B.n_bins; ++b) {
        const double w = 2 * M_PI * (C.B.j_lo + b) * C.B.df;
        const std::complex<double> v = pulse_spectrum(C.P, w) * transducer_spectrum(C.P, w) * f2;
        at<float2>(h, L.pw)[b] = make_float2((float)v.real(), (float)v.imag());
    }
}

// The call's model constants with the device address of its Gaussian table.
ModelConst dev_consts(const Common& C, char* d, const CommonLayout& L)
{
    ModelConst K = C.K;
    K.gset = at<float4>(d, L.gs);
    return K;
}

SubGeo sub_geo(char* d, const CommonLayout& L)
{
    return SubGeo{at<double>(d, L.xc), at<double>(d, L.zc), at<float>(d, L.tx),
                  at<float>(d, L.tz), at<float>(d, L.nx), at<float>(d, L.nz)};
}

// Transmit weights, and for y = 0 the elevation table of the call.
void launch_common(char* d, const CommonLayout& L, const Common& C, const float* x, const float* y,
                   const float* z, hipStream_t st)
{
    hip_check(timed(K_WTABLE, st, [&] {
                  return launch_wtable(at<float2>(d, L.W), at<double>(d, L.dl), at<float>(d, L.ap),
                                       C.B.n_bins, C.n_tx, C.P.N, C.B.j_lo, C.B.df, st);
              }),
              "wtable launch");
    if (C.table) {
        hip_check(launch_rrange(at<uint32_t>(d, L.rr), x, y, z, C.ph.total, sub_geo(d, L), C.P.M, st),
                  "range launch");
        hip_check(launch_dtable(at<float4>(d, L.dt), at<DeltaParams>(d, L.dp), at<uint32_t>(d, L.rr),
                                C.K, at<double>(d, L.gd), C.P.height, C.B.j_lo,
                                C.B.j_lo + std::max(C.B.n_bins, 1) - 1, C.P.dim2, st),
                  "table launch");
    }
}

// ---------------------------------------------------------------- forward spectra
// Everything the forward path decides on the host for a probe, a transmit
// sequence and a partition into phantoms: the launch configuration, the work
// items and the workspace layout.  `host` holds the upload region (tables,
// items) already filled.
struct FwdPlan {
    Common C;
    SynthConfig cfg{};
    bool use_mt = false;
    int slots = 0;    // partial slots per (item, bin, transmit): sub-elements or elements
    int fin_nu = 0;   // sub-elements summed by the finalisation (1 once summed per element)
    int n_bt = 0, n_items = 0;
    int64_t slice = 0;
    CommonLayout L{};
    size_t o_it = 0, o_or = 0, o_pb = 0, o_ns = 0, o_part = 0, o_tk = 0, o_spec = 0, o_wt = 0;
    size_t up_size = 0, dv_size = 0;
    std::vector<char> host;
};

// Workspace layout of a forward plan with n_items work items: the upload
// region (tables, items, draw order, per-phantom item bases and slice
// counts) first, then the device-only tables, partial spectra, work counter
// and, with own_spec, the spectra.  Sets F's offsets; returns the size.
size_t fwd_layout(FwdPlan& F, int n_items, bool own_spec)
{
    const Common& C = F.C;
    Layout up;
    layout_upload(up, F.L, C);
    F.o_it = up.add(sizeof(Item) * std::max(n_items, 1));
    F.o_or = up.add(sizeof(int32_t) * std::max(n_items, 1));
    F.o_pb = up.add(sizeof(int32_t) * C.ph.n);
    F.o_ns = up.add(sizeof(int32_t) * C.ph.n);
    Layout dv = up;
    layout_device(dv, F.L, C);
    F.o_part = dv.add(sizeof(float2) * size_t(std::max(n_items, 1)) * F.cfg.jt * F.cfg.tt * F.slots);
    F.o_tk = dv.add(sizeof(int32_t) * 4);
    // the matrix-core kernels' padded weights [n_bins][n_tg][NE][TT] (or
    // [n_bins][n_tg][TT][NE] split)
    const int n_tgw = (C.n_tx + F.cfg.tt - 1) / F.cfg.tt;
    F.o_wt = F.cfg.wt ? dv.add(sizeof(float2) * size_t(std::max(C.B.n_bins, 1)) * n_tgw * F.cfg.ne * F.cfg.tt) : 0;
    const size_t spec_bytes = sizeof(float2) * size_t(C.ph.n) * C.n_tx * C.P.N * std::max(C.B.n_bins, 1);
    F.o_spec = own_spec ? dv.add(spec_bytes) : 0;
    F.up_size = up.size;
    F.dv_size = dv.size;
    return dv.size;
}

// The synthesis grid: as many blocks as can be resident at once for the
// persistent launch, else one block per item.
void set_launch_grid(FwdPlan& F, const simus_options* opt)
{
    SynthConfig& cfg = F.cfg;
    // resident blocks draw items from a work counter (measurably faster than
    // a static grid on both paths); SIMUS_FLAG_STATIC asks for one block per
    // item on the vector path
    cfg.persistent = (F.use_mt || !(opt->flags & SIMUS_FLAG_STATIC)) && F.n_items > 0;
    if (cfg.persistent) {
        hipDeviceProp_t prop;
        int dev = 0;
        hip_check(hipGetDevice(&dev), "hipGetDevice");
        hip_check(hipGetDeviceProperties(&prop, dev), "hipGetDeviceProperties");
        const SynthKernel k = F.use_mt ? synth_mt_kernel(cfg) : synth_kernel(cfg);
        if (!k) throw Error{SIMUS_EINVAL, "no synthesis kernel for this configuration"};
        int per_cu = 0;
        hip_check(hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, reinterpret_cast<const void*>(k),
                                                               F.use_mt ? 512 : cfg.bs, 0),
                  "hipOccupancyMaxActiveBlocksPerMultiprocessor");
        cfg.grid = std::min(F.n_items, prop.multiProcessorCount * std::max(per_cu, 1));
    } else {
        cfg.grid = F.n_items;
    }
}

// max_dev_bytes > 0 bounds the workspace (simus_rf_noalloc's scratch): the
// scatterers per item grow until the plan fits, and a plan that does not fit
// even with one slice per phantom, bin tile and transmit group throws
// SIMUS_ETOOBIG.  Everything before the launch grid is host work only.
FwdPlan make_fwd_plan(Common C, const simus_options* opt, const double* delays, const float* apod,
                      bool own_spec, size_t max_dev_bytes = 0)
{
    FwdPlan F;
    F.C = std::move(C);
    const Common& Cc = F.C;
    const int M = Cc.P.M, N = Cc.P.N, n_tx = Cc.n_tx, n_ph = Cc.ph.n;
    F.use_mt = !(opt->flags & SIMUS_FLAG_NO_MFMA) && mt_supported(M, N, n_tx) &&
               Cc.K.sinc_per_bin < SINC_TAYLOR_LIMIT;
    SynthConfig& cfg = F.cfg;
    const bool alt = (opt->flags & SIMUS_FLAG_ALT_SHAPE) != 0;
    const bool fp32 = (opt->flags & SIMUS_FLAG_FP32_PRODUCTS) != 0;
    cfg = F.use_mt ? mt_config(M, N, n_tx, Cc.has_y, alt, fp32)
                   : synth_config(M, Cc.P.nu, n_tx, Cc.has_y, Cc.table && !Cc.P.dim2, alt);
    cfg.table = Cc.table;
    cfg.dim2 = Cc.P.dim2;   // the vector path skips the (unit) table in 2-D
    const int JT = cfg.jt, TT = cfg.tt, BS = cfg.bs, SC = cfg.sc;
    // element partials (matrix-core path, or paired lanes) or sub-element partials
    const bool per_element = F.use_mt || cfg.pair;
    F.slots = F.use_mt ? N : cfg.pair ? BS / 2 : BS;
    F.fin_nu = per_element ? 1 : Cc.P.nu;
    F.n_bt = (Cc.B.n_bins + JT - 1) / JT;
    const int n_tg = (n_tx + TT - 1) / TT;
    if (F.n_bt >= 65536 || n_tg >= 32768) throw Error{SIMUS_EINVAL, "problem too large for the tile index"};
    // scatterers per item: about 6000 items (matrix-core path: 3000) over the
    // whole call, enough for a short tail over the resident blocks; fewer,
    // longer items halve the partial spectra and the finaliser's work (12000
    // items measured 0.6 % slower per call on the vector path)
    int64_t slice = opt->tile_scat;
    if (slice <= 0) {
        const int64_t work = std::max<int64_t>(1, Cc.ph.total) * F.n_bt * n_tg;
        slice = F.use_mt ? (work + 2999) / 3000 : (work + 5999) / 6000;
    }
    // a multiple of the super-chunk (groups x chunk) that the kernel steps by
    const int SCG = SC * (F.use_mt ? 1 : std::max(cfg.groups, 1));
    auto round_slice = [&](int64_t sl) {
        sl = std::max<int64_t>(sl, 4 * SCG);
        sl = (sl + SCG - 1) / SCG * SCG;
        return std::min<int64_t>(sl, int64_t(1) << 30);
    };
    slice = round_slice(slice);
    auto count_items = [&](int64_t sl) {
        int64_t n = 0;
        for (int p = 0; p < n_ph; ++p) n += (Cc.ph.off[p + 1] - Cc.ph.off[p] + sl - 1) / sl;
        return n * F.n_bt * n_tg;
    };
    if (max_dev_bytes > 0) {
        int64_t s_max = 1;
        for (int p = 0; p < n_ph; ++p) s_max = std::max(s_max, Cc.ph.off[p + 1] - Cc.ph.off[p]);
        s_max = round_slice(s_max);
        for (;;) {
            const int64_t ni = count_items(slice);
            if (ni < (int64_t(1) << 30) && fwd_layout(F, (int)ni, own_spec) <= max_dev_bytes) break;
            if (slice >= s_max) {
                fwd_layout(F, (int)std::min<int64_t>(ni, int64_t(1) << 30), own_spec);
                throw Error{SIMUS_ETOOBIG, "the call needs " + std::to_string(F.dv_size) +
                                               " bytes of workspace; the no-allocation scratch holds " +
                                               std::to_string(max_dev_bytes)};
            }
            slice = std::min(s_max, round_slice(slice + slice / 4));
        }
    }
    if (count_items(slice) >= (int64_t(1) << 31)) throw Error{SIMUS_EINVAL, "too many work items"};
    F.slice = slice;

    std::vector<Item> items;
    std::vector<int32_t> pbase(n_ph), nsl(n_ph);
    for (int p = 0; p < n_ph; ++p) {
        const int64_t Sp = Cc.ph.off[p + 1] - Cc.ph.off[p];
        const int ns = (int)((Sp + slice - 1) / slice);
        pbase[p] = (int32_t)items.size();
        nsl[p] = ns;
        for (int tg = 0; tg < n_tg; ++tg)
            for (int bt = 0; bt < F.n_bt; ++bt)
                for (int sl = 0; sl < ns; ++sl) {
                    const int64_t s0 = Cc.ph.off[p] + int64_t(sl) * slice;
                    const int64_t s1 = std::min<int64_t>(s0 + slice, Cc.ph.off[p + 1]);
                    items.push_back(Item{p, (int32_t)s0, (int32_t)s1, bt | (tg << 16)});
                }
    }
    F.n_items = (int)items.size();
    // draw order: costliest items (scatterers x bins) first, so that the
    // persistent blocks finish on small items
    std::vector<int32_t> order(F.n_items);
    for (int i = 0; i < F.n_items; ++i) order[i] = i;
    auto cost = [&](int i) {
        const Item& q = items[i];
        return int64_t(q.s_end - q.s_begin) * std::min(JT, Cc.B.n_bins - (q.tile & 0xffff) * JT);
    };
    std::stable_sort(order.begin(), order.end(), [&](int a, int b) { return cost(a) > cost(b); });

    fwd_layout(F, F.n_items, own_spec);
    F.host.assign(F.up_size, 0);
    char* h = F.host.data();
    fill_upload(h, F.L, Cc, delays, apod);
    if (F.n_items) {
        std::memcpy(h + F.o_it, items.data(), sizeof(Item) * F.n_items);
        std::memcpy(h + F.o_or, order.data(), sizeof(int32_t) * F.n_items);
    }
    std::memcpy(h + F.o_pb, pbase.data(), sizeof(int32_t) * n_ph);
    std::memcpy(h + F.o_ns, nsl.data(), sizeof(int32_t) * n_ph);
    set_launch_grid(F, opt);
    return F;
}

// Enqueues the forward kernels of a plan on st (kernel launches only: no
// copies, allocations or host waits), with the workspace at device address d
// holding the plan's upload region.  Spectra go to spec_out, or to the
// workspace followed by the inverse transform into rf_out.
void enqueue_fwd(const FwdPlan& F, char* d, const float* x, const float* y, const float* z,
                 const float* refl, float* spec_out, float* rf_out, hipStream_t st)
{
    const Common& C = F.C;
    const SynthConfig& cfg = F.cfg;
    const int N = C.P.N, n_tx = C.n_tx, n_ph = C.ph.n;
    float2* spec = spec_out ? reinterpret_cast<float2*>(spec_out) : at<float2>(d, F.o_spec);
    launch_common(d, F.L, C, x, y, z, st);
    if (cfg.wt)
        hip_check(timed(K_WTABLE, st, [&] {
                      return launch_wtable_mt(at<float2>(d, F.o_wt), at<double>(d, F.L.dl), at<float>(d, F.L.ap),
                                              C.B.n_bins, n_tx, N, cfg.ne, cfg.tt, (n_tx + cfg.tt - 1) / cfg.tt,
                                              C.B.j_lo, C.B.df, cfg.bf, st);
                  }),
                  "matrix-core weight table launch");
    SynthArgs A{};
    A.x = x;
    A.y = y;
    A.z = z;
    A.refl = refl;
    A.sub = sub_geo(d, F.L);
    A.W = at<float2>(d, F.L.W);
    A.WT = cfg.wt ? at<float2>(d, F.o_wt) : nullptr;
    A.items = at<Item>(d, F.o_it);
    A.order = at<int32_t>(d, F.o_or);
    A.n_items = F.n_items;
    A.part = at<float2>(d, F.o_part);
    A.M = C.P.M;
    A.nu = C.P.nu;
    A.N = N;
    A.n_tx = n_tx;
    A.n_bins = C.B.n_bins;
    A.j_lo = C.B.j_lo;
    A.K = dev_consts(C, d, F.L);
    A.dtab = C.table ? at<float4>(d, F.L.dt) : nullptr;
    A.dpar = C.table ? at<DeltaParams>(d, F.L.dp) : nullptr;
    A.ticket = nullptr;
    if (cfg.persistent) {
        A.ticket = at<int32_t>(d, F.o_tk);
        hip_check(launch_zero_i32(A.ticket, 1, st), "zero launch");
    }
    if (log_enabled())
        std::fprintf(stderr,
                     "[simus] N=%d nu=%d M=%d T=%d P=%d S=%lld nfft=%d n_t=%d j_lo=%d bins=%d "
                     "BS=%d G=%d TT=%d SC=%d JT=%d slice=%lld items=%d grid=%d y=%d table=%d persistent=%d mfma=%d\n",
                     N, C.P.nu, C.P.M, n_tx, n_ph, (long long)C.ph.total, C.B.nfft, C.B.n_t, C.B.j_lo,
                     C.B.n_bins, cfg.bs, cfg.groups, cfg.tt, cfg.sc, cfg.jt, (long long)F.slice, F.n_items, cfg.grid,
                     (int)C.has_y, (int)C.table, (int)cfg.persistent, (int)F.use_mt);
    hip_check(timed(K_SYNTH, st, [&] {
                  return F.use_mt ? launch_synth_mt(cfg, A, st) : launch_synth(cfg, A, st);
              }),
              "synthesis launch");
    hip_check(timed(K_FINALIZE, st, [&] {
                  return launch_finalize(spec, A.part, at<float2>(d, F.L.pw), at<int32_t>(d, F.o_pb),
                                         at<int32_t>(d, F.o_ns), n_ph, n_tx, N, F.fin_nu, C.B.n_bins,
                                         F.slots, F.use_mt ? 1 : cfg.groups, cfg.tt, cfg.jt, F.n_bt,
                                         C.B.j_lo, true, st);
              }),
              "finalize launch");
    if (rf_out) {
        hip_check(timed(K_IDFT, st, [&] {
                      return launch_idft(rf_out, spec, int64_t(n_ph) * n_tx * N, C.B.n_bins,
                                         C.B.j_lo, C.B.nfft, C.B.n_t, st);
                  }),
                  "inverse transform launch");
    }
}

// One call: plan, upload through the stream's staging buffer, enqueue.
void forward_spectra(const simus_probe* probe, const simus_medium* medium,
                     const simus_options* opt, int32_t n_tx, const double* delays,
                     const float* apod, int32_t n_ph, const int64_t* offs, const float* x,
                     const float* y, const float* z, const float* refl, float* spec_out,
                     float* rf_out, hipStream_t st)
{
    if (!spec_out && !rf_out) throw Error{SIMUS_EINVAL, "output pointer must be non-NULL"};
    Common C = make_common(probe, medium, opt, n_tx, delays, apod, n_ph, offs, x, y, z, refl);
    const FwdPlan F = make_fwd_plan(std::move(C), opt, delays, apod, spec_out == nullptr);
    Arena& a = arena_for(st, F.dv_size, F.up_size);
    std::memcpy(a.host, F.host.data(), F.up_size);
    upload(a, F.up_size, st);
    enqueue_fwd(F, a.dev, x, y, z, refl, spec_out, rf_out, st);
}

// ---------------------------------------------------------------- adjoint
void backward(const simus_probe* probe, const simus_medium* medium, const simus_options* opt,
              int32_t n_tx, const double* delays, const float* apod, int32_t n_ph,
              const int64_t* offs, const float* x, const float* y, const float* z,
              const float* refl, const float* drf, float* dR, float* dX, float* dY, float* dZ,
              hipStream_t st)
{
    const Common C = make_common(probe, medium, opt, n_tx, delays, apod, n_ph, offs, x, y, z, refl);
    if (C.ph.total > 0 && !drf) throw Error{SIMUS_EINVAL, "drf must be non-NULL"};
    if (!dR && !dX && !dY && !dZ) return;
    if (C.ph.total == 0) return;
    const int N = C.P.N;
    const bool mt_ok = !(opt->flags & SIMUS_FLAG_NO_MFMA) && adjoint_mt_supported(C.P.M, N, n_tx) &&
                       C.K.sinc_per_bin < SINC_TAYLOR_LIMIT;
    // The matrix-core adjoint pads transmits to groups of 8 and elements to
    // 128 slots; below N n_tx = 384, or under 48 elements, the vector kernel
    // measured faster (50k scatterers, 128 elements: 1 transmit 32 vs 58 ms,
    // 3 transmits 73 vs 61; 64 elements: 4 transmits 31 vs 54, 6-8 equal;
    // 32 elements, 8 transmits: 26 vs 52).  SIMUS_FLAG_ALT_SHAPE takes the
    // other kernel where both apply.
    const bool mt_pref = N >= 48 && int64_t(N) * n_tx >= 384;
    const bool use_mt = mt_ok && (((opt->flags & SIMUS_FLAG_ALT_SHAPE) != 0) != mt_pref);
    AdjConfig cfg = use_mt ? adjoint_mt_config(C.P.M, N, n_tx, C.has_y) : adjoint_config(n_tx, C.has_y);
    cfg.table = C.table;
    cfg.bf = cfg.wl && !(opt->flags & SIMUS_FLAG_FP32_PRODUCTS);
    // items: (phantom, scatterer slice, bin range); about 3000 items (matrix-core
    // path: 4000), bin ranges a multiple of the bin tile
    const int slice = cfg.scatterers;
    int64_t n_sb = 0;
    for (int p = 0; p < n_ph; ++p) n_sb += (C.ph.off[p + 1] - C.ph.off[p] + slice - 1) / slice;
    const int64_t target = use_mt ? 4000 : 3000;
    int64_t rb = (int64_t(std::max(C.B.n_bins, 1)) * n_sb + target - 1) / target;
    rb = std::max<int64_t>(rb, cfg.jt);
    // k_adjoint_mq reads its columns (16 KiB per bin) from a table in global
    // memory: ranges of at most 96 bins, drawn range by range, keep the
    // table's part that resident blocks share within an XCD's L2 (5 plane
    // waves, 100k scatterers: 87.5 ms with 384-bin ranges drawn slice by
    // slice, 83.3 range by range, 82.8 with 96-bin ranges, 83.3 with 64)
    if (use_mt && cfg.wl) rb = std::min<int64_t>(rb, 96);
    rb = (rb + cfg.jt - 1) / cfg.jt * cfg.jt;
    const int range_bins = (int)std::min<int64_t>(rb, std::max(C.B.n_bins, 1));
    const int n_ranges = (std::max(C.B.n_bins, 1) + range_bins - 1) / range_bins;
    std::vector<AdjItem> items;
    for (int r = 0; r < n_ranges; ++r)
        for (int p = 0; p < n_ph; ++p)
            for (int64_t s0 = C.ph.off[p]; s0 < C.ph.off[p + 1]; s0 += slice)
                items.push_back(AdjItem{p, (int32_t)s0,
                                        (int32_t)std::min<int64_t>(s0 + slice, C.ph.off[p + 1]), r});
    const int n_items = (int)items.size();

    Layout up;
    CommonLayout L;
    layout_upload(up, L, C);
    const size_t o_it = up.add(sizeof(AdjItem) * std::max(n_items, 1));
    Layout dv = up;
    layout_device(dv, L, C);
    const size_t o_lam =
        dv.add(sizeof(float2) * size_t(n_ph) * std::max(C.B.n_bins, 1) * n_tx * N);
    const size_t o_part = dv.add(sizeof(float4) * size_t(n_ranges) * C.ph.total);
    const bool wl = use_mt && cfg.wl;
    const size_t o_wl = wl ? dv.add(sizeof(float2) * size_t(n_ph) * std::max(C.B.n_bins, 1) * 128 * 16) : 0;

    Arena& a = arena_for(st, dv.size, up.size);
    fill_upload(a.host, L, C, delays, apod);
    std::memcpy(a.host + o_it, items.data(), sizeof(AdjItem) * n_items);
    upload(a, up.size, st);
    char* d = a.dev;
    launch_common(d, L, C, x, y, z, st);
    hip_check(timed(K_DFT, st, [&] {
                  return launch_dft_t(at<float2>(d, o_lam), drf, int64_t(n_ph) * n_tx * N,
                                      C.B.n_bins, C.B.j_lo, C.B.nfft, C.B.n_t, n_tx, N, st);
              }),
              "residual transform launch");
    AdjArgs A{};
    A.x = x;
    A.y = y;
    A.z = z;
    A.refl = refl;
    A.sub = sub_geo(d, L);
    A.W = at<float2>(d, L.W);
    A.lam = at<float2>(d, o_lam);
    A.pw = at<float2>(d, L.pw);
    A.WL = wl ? at<float2>(d, o_wl) : nullptr;
    A.items = at<AdjItem>(d, o_it);
    A.part = at<float4>(d, o_part);
    A.dtab = C.table ? at<float4>(d, L.dt) : nullptr;
    A.dpar = C.table ? at<DeltaParams>(d, L.dp) : nullptr;
    A.S_total = C.ph.total;
    A.M = C.P.M;
    A.nu = C.P.nu;
    A.N = N;
    A.n_tx = n_tx;
    A.n_bins = C.B.n_bins;
    A.j_lo = C.B.j_lo;
    A.range_bins = range_bins;
    A.K = dev_consts(C, d, L);
    if (log_enabled())
        std::fprintf(stderr, "[simus] adjoint S=%lld T=%d bins=%d TT=%d JT=%d range=%d items=%d y=%d table=%d mfma=%d\n",
                     (long long)C.ph.total, n_tx, C.B.n_bins, cfg.tt, cfg.jt, range_bins, n_items,
                     (int)C.has_y, (int)C.table, (int)use_mt);
    if (wl)
        hip_check(launch_wltable(at<float2>(d, o_wl), A.W, A.lam, n_ph, C.B.n_bins, n_tx, N, cfg.bf, st),
                  "adjoint column table launch");
    hip_check(timed(K_ADJ, st, [&] {
                  return use_mt ? launch_adjoint_mt(cfg, A, n_items, st) : launch_adjoint(cfg, A, n_items, st);
              }),
              "adjoint launch");
    hip_check(timed(K_ADJRED, st, [&] {
                  return launch_adjoint_reduce(A.part, n_ranges, C.ph.total, refl, dR, dX, dY, dZ, st);
              }),
              "adjoint reduce launch");
}

// ---------------------------------------------------------------- RMS field
int pfield_nf_host(const Probe& P, const SubElements& S, const double* delays, int64_t n,
                   const float* X, const float* Y, const float* Z)
{
    // Section VII: dw = 2 pi / max(r / c + delay) over points and sub-elements,
    // N_f = ceil(2 wc / dw) = ceil(2 fc max(r / c + delay)).
    double tmax = 0;
    for (int64_t p = 0; p < n; ++p) {
        const double yy = Y ? double(Y[p]) : 0.0;
        for (int m = 0; m < P.M; ++m) {
            const double dx = double(X[p]) - S.xc[m], dz = double(Z[p]) - S.zc[m];
            tmax = std::max(tmax, std::sqrt(dx * dx + dz * dz + yy * yy) / P.c + delays[m / P.nu]);
        }
    }
    const double nf = std::ceil(2.0 * P.fc * tmax);
    if (!(nf >= 1) || nf > 1e6) throw Error{SIMUS_EINVAL, "field frequency count out of range"};
    return (int)nf;
}

void pfield(const simus_probe* probe, const simus_medium* medium, const simus_options* opt,
            int32_t n_f, const double* delays, const float* apod, int64_t n_pts, const float* X,
            const float* Y, const float* Z, float* out, hipStream_t st)
{
    Common C;
    C.P = make_probe(probe, medium, opt);
    check_transmits(C.P, 1, delays, apod);
    if (n_f < 1 || n_f > 1000000) throw Error{SIMUS_EINVAL, "n_f must be in [1, 1e6]"};
    if (n_pts < 0) throw Error{SIMUS_EINVAL, "n_pts must be >= 0"};
    if (n_pts > 0 && (!X || !Z || !out)) throw Error{SIMUS_EINVAL, "X, Z and p_rms must be non-NULL"};
    if (n_pts == 0) return;
    // nodes w_j = 2 wc j / N_f, j = 1 .. N_f (j = 0 carries S_P(0) = 0)
    C.B.nfft = 0;
    C.B.n_t = 0;
    C.B.j_lo = 1;
    C.B.n_bins = n_f;
    C.B.df = 2.0 * C.P.fc / n_f;
    C.S = sub_elements(C.P);
    C.K = model_constants(C.P, C.B);
    C.n_tx = 1;
    C.has_y = Y != nullptr;
    if (C.P.dim2 && C.has_y) throw Error{SIMUS_EINVAL, "Y must be NULL with SIMUS_FLAG_2D"};
    C.table = C.P.dim2 || (!C.has_y && !(opt->flags & SIMUS_FLAG_NO_DELTA_TABLE));
    C.ph.n = 1;
    C.ph.total = n_pts;
    // frequency ranges of nearly equal size, each split into tiles of at
    // most PFIELD_JT bins: as many ranges as tiles, up to about 6 rounds of
    // resident blocks (5 per CU) over the point blocks; past that, ranges of
    // a whole number of tiles each, so that the tiles stay nearly full
    const int64_t n_pb = (n_pts + 255) / 256;
    const int64_t n_tl = std::max<int64_t>(1, (n_f + PFIELD_JT - 1) / PFIELD_JT);
    const int64_t cap = std::max<int64_t>(1, (6 * 1280 + n_pb - 1) / n_pb);
    const int64_t tiles_per_range = (n_tl + cap - 1) / cap;
    const int n_ranges = (int)((n_tl + tiles_per_range - 1) / tiles_per_range);
    if (n_pb > 0x7fffffff || n_ranges > 65535) throw Error{SIMUS_EINVAL, "too many field points"};

    Layout up;
    CommonLayout L;
    layout_upload(up, L, C);
    const size_t o_ptx = up.add(sizeof(float2) * n_f);
    Layout dv = up;
    layout_device(dv, L, C);
    const size_t o_part = dv.add(sizeof(float) * size_t(n_ranges) * n_pts);
    Arena& a = arena_for(st, dv.size, up.size);
    fill_upload(a.host, L, C, delays, apod);
    // one-way P_Tx = S_P sqrt(S_T) (Eq. 28); in 2-D with the factor sqrt(2b) of Eq. (37)
    const double f1 = C.P.dim2 ? std::sqrt(C.P.width) : 1.0;
    for (int j = 1; j <= n_f; ++j) {
        const double w = 2 * M_PI * j * C.B.df;
        const std::complex<double> v = pulse_spectrum(C.P, w) * std::sqrt(transducer_spectrum(C.P, w)) * f1;
        at<float2>(a.host, o_ptx)[j - 1] = make_float2((float)v.real(), (float)v.imag());
    }
    upload(a, up.size, st);
    char* d = a.dev;
    launch_common(d, L, C, X, Y, Z, st);
    FieldArgs F{};
    F.X = X;
    F.Y = Y;
    F.Z = Z;
    F.sub = sub_geo(d, L);
    F.W = at<float2>(d, L.W);
    F.ptx = at<float2>(d, o_ptx);
    F.part = at<float>(d, o_part);
    F.dtab = C.table ? at<float4>(d, L.dt) : nullptr;
    F.dpar = C.table ? at<DeltaParams>(d, L.dp) : nullptr;
    F.n_pts = n_pts;
    F.M = C.P.M;
    F.nu = C.P.nu;
    F.N = C.P.N;
    F.n_bins = n_f;
    F.j_lo = 1;
    F.n_ranges = n_ranges;
    F.K = dev_consts(C, d, L);
    hip_check(timed(K_PFIELD, st, [&] { return launch_pfield(F, C.has_y, C.table, n_ranges, st); }),
              "field launch");
    const float dw = (float)(2.0 * M_PI * C.B.df);
    hip_check(launch_pfield_reduce(F.part, n_ranges, n_pts, dw, out, st), "field reduce launch");
}

template <class Fn>
int guarded(Fn&& fn)
{
    try {
        fn();
        return SIMUS_OK;
    } catch (const Error& e) {
        return fail(e.code, e.msg);
    } catch (const std::exception& e) {
        return fail(SIMUS_EINVAL, std::string("internal error: ") + e.what());
    } catch (...) {
        return fail(SIMUS_EINVAL, "internal error");
    }
}

}  // namespace
}  // namespace simus

using namespace simus;

// A forward plan: the host plan, its device workspace (upload region first)
// and the graph captured for the last pointer set.
struct simus_rf_plan_s {
    FwdPlan F;
    simus_options opt{};          // as created (the autotuner changes tile_scat, flags)
    std::vector<double> delays;   // host copies, for rebuilding the plan
    std::vector<float> apod;
    int device = 0;
    char* dev = nullptr;
    size_t dev_cap = 0;
    hipStream_t cap = nullptr;
    hipGraphExec_t exec = nullptr;
    const void* key[5] = {};
    std::mutex mu;

    ~simus_rf_plan_s()
    {
        int cur = 0;
        (void)hipGetDevice(&cur);
        (void)hipSetDevice(device);
        (void)hipDeviceSynchronize();
        if (exec) (void)hipGraphExecDestroy(exec);
        if (cap) (void)hipStreamDestroy(cap);
        if (dev) (void)hipFree(dev);
        (void)hipSetDevice(cur);
    }
};

namespace {

void check_plan_call(simus_rf_plan plan, const float* x, const float* y, const float* z,
                     const float* refl, const float* rf)
{
    if (!plan) throw Error{SIMUS_EINVAL, "plan must be non-NULL"};
    if (!rf) throw Error{SIMUS_EINVAL, "rf must be non-NULL"};
    check_scatterers(plan->F.C, x, y, z, refl);
    int cur = 0;
    hip_check(hipGetDevice(&cur), "hipGetDevice");
    if (cur != plan->device) throw Error{SIMUS_EINVAL, "plan belongs to another device"};
}

}  // namespace

extern "C" {

int simus_version(void) { return SIMUS_VERSION; }

const char* simus_last_error(void) { return g_last_error.c_str(); }

int simus_rf_grid(const simus_probe* probe, const simus_medium* medium, const simus_options* opt,
                  int32_t n_tx, const double* delays, int64_t n_scat, const float* x,
                  const float* y, const float* z, simus_grid* out)
{
    return guarded([&] {
        if (!out) throw Error{SIMUS_EINVAL, "out must be non-NULL"};
        const Probe P = make_probe(probe, medium, opt);
        check_transmits(P, n_tx, delays, nullptr);
        if (n_scat < 0) throw Error{SIMUS_EINVAL, "n_scat must be >= 0"};
        if (n_scat > 0 && (!x || !z)) throw Error{SIMUS_EINVAL, "x and z must be non-NULL"};
        if (P.dim2 && y) throw Error{SIMUS_EINVAL, "y must be NULL with SIMUS_FLAG_2D"};
        const SubElements S = sub_elements(P);
        check_domain(P, S, n_scat, x, y, z);
        int64_t nfft = opt->nfft;
        if (nfft <= 0) {
            const double rmax = max_distance(S, n_scat, x, y, z);
            double dmax = 0;
            for (int64_t i = 0; i < int64_t(n_tx) * P.N; ++i) dmax = std::max(dmax, delays[i]);
            const double tmax = 2 * rmax / P.c + dmax + 10.0 / P.fc;
            const int64_t need = std::max<int64_t>((int64_t)std::ceil(P.fs * tmax), opt->n_t);
            nfft = next_fft_size(need);
        }
        if (nfft > (int64_t(1) << 26)) throw Error{SIMUS_EINVAL, "nfft too large"};
        if (opt->n_t > nfft) throw Error{SIMUS_EINVAL, "options.n_t must be <= nfft"};
        const Band B = make_band(P, (int)nfft, opt->n_t);
        out->nfft = B.nfft;
        out->n_t = B.n_t;
        out->j_lo = B.j_lo;
        out->n_bins = B.n_bins;
        out->nu = P.nu;
        out->reserved = 0;
        out->df = B.df;
    });
}

int simus_rf_spectrum(const simus_probe* probe, const simus_medium* medium,
                      const simus_options* opt, int32_t n_tx, const double* delays,
                      const float* apod, int32_t n_ph, const int64_t* offs, const float* x,
                      const float* y, const float* z, const float* refl, float* spec,
                      void* hip_stream)
{
    return guarded([&] {
        if (!spec) throw Error{SIMUS_EINVAL, "spec must be non-NULL"};
        forward_spectra(probe, medium, opt, n_tx, delays, apod, n_ph, offs, x, y, z, refl, spec,
                        nullptr, static_cast<hipStream_t>(hip_stream));
    });
}

int simus_rf(const simus_probe* probe, const simus_medium* medium, const simus_options* opt,
             int32_t n_tx, const double* delays, const float* apod, int32_t n_ph,
             const int64_t* offs, const float* x, const float* y, const float* z,
             const float* refl, float* rf, void* hip_stream)
{
    return guarded([&] {
        if (!rf) throw Error{SIMUS_EINVAL, "rf must be non-NULL"};
        forward_spectra(probe, medium, opt, n_tx, delays, apod, n_ph, offs, x, y, z, refl, nullptr,
                        rf, static_cast<hipStream_t>(hip_stream));
    });
}

int simus_rf_noalloc(const simus_probe* probe, const simus_medium* medium,
                     const simus_options* opt, int32_t n_tx, const double* delays,
                     const float* apod, int32_t n_ph, const int64_t* offs, const float* x,
                     const float* y, const float* z, const float* refl, float* rf,
                     void* hip_stream)
{
    return guarded([&] {
        if (!rf) throw Error{SIMUS_EINVAL, "rf must be non-NULL"};
        Common C = make_common(probe, medium, opt, n_tx, delays, apod, n_ph, offs, x, y, z, refl);
        // host work only up to here: a call that cannot fit the scratch is
        // refused (SIMUS_ETOOBIG) before any HIP call
        const FwdPlan F = make_fwd_plan(std::move(C), opt, delays, apod, true, NOALLOC_SCRATCH_BYTES);
        char* d = nullptr;
        hip_check(noalloc_scratch(&d), "scratch address");
        const hipStream_t st = static_cast<hipStream_t>(hip_stream);
        // the plan's tables, from pageable host memory: the runtime copies
        // them out of F.host before the call returns (HIP's pageable-copy
        // semantics), so F.host may go when this function ends
        hip_check(hipMemcpyAsync(d, F.host.data(), F.up_size, hipMemcpyHostToDevice, st),
                  "hipMemcpyAsync");
        Untimed untimed;
        enqueue_fwd(F, d, x, y, z, refl, nullptr, rf, st);
    });
}

int simus_rf_backward(const simus_probe* probe, const simus_medium* medium,
                      const simus_options* opt, int32_t n_tx, const double* delays,
                      const float* apod, int32_t n_ph, const int64_t* offs, const float* x,
                      const float* y, const float* z, const float* refl, const float* drf,
                      float* drefl, float* dx, float* dy, float* dz, void* hip_stream)
{
    return guarded([&] {
        backward(probe, medium, opt, n_tx, delays, apod, n_ph, offs, x, y, z, refl, drf, drefl, dx,
                 dy, dz, static_cast<hipStream_t>(hip_stream));
    });
}

int simus_pfield_nf(const simus_probe* probe, const simus_medium* medium, const simus_options* opt,
                    const double* delays, int64_t n_pts, const float* X, const float* Y,
                    const float* Z, int32_t* n_f)
{
    return guarded([&] {
        if (!n_f) throw Error{SIMUS_EINVAL, "n_f must be non-NULL"};
        const Probe P = make_probe(probe, medium, opt);
        check_transmits(P, 1, delays, nullptr);
        if (n_pts < 1 || !X || !Z) throw Error{SIMUS_EINVAL, "at least one point (X, Z non-NULL) is required"};
        if (P.dim2 && Y) throw Error{SIMUS_EINVAL, "Y must be NULL with SIMUS_FLAG_2D"};
        const SubElements S = sub_elements(P);
        *n_f = pfield_nf_host(P, S, delays, n_pts, X, Y, Z);
    });
}

int simus_pfield(const simus_probe* probe, const simus_medium* medium, const simus_options* opt,
                 int32_t n_f, const double* delays, const float* apod, int64_t n_pts,
                 const float* X, const float* Y, const float* Z, float* p_rms, void* hip_stream)
{
    return guarded([&] {
        pfield(probe, medium, opt, n_f, delays, apod, n_pts, X, Y, Z, p_rms,
               static_cast<hipStream_t>(hip_stream));
    });
}

int simus_rf_plan_create(const simus_probe* probe, const simus_medium* medium,
                         const simus_options* opt, int32_t n_tx, const double* delays,
                         const float* apod, int32_t n_ph, const int64_t* offs, int32_t has_y,
                         void* hip_stream, simus_rf_plan* out)
{
    return guarded([&] {
        if (!out) throw Error{SIMUS_EINVAL, "plan must be non-NULL"};
        Common C = make_common(probe, medium, opt, n_tx, delays, apod, n_ph, offs, has_y != 0);
        std::unique_ptr<simus_rf_plan_s> pl(new simus_rf_plan_s);
        pl->F = make_fwd_plan(std::move(C), opt, delays, apod, true);
        pl->opt = *opt;
        // the plan holds its Gaussians in its probe (the caller's array may go)
        pl->opt.n_gauss = 0;
        pl->opt.gauss = nullptr;
        pl->delays.assign(delays, delays + size_t(n_tx) * pl->F.C.P.N);
        if (apod) pl->apod.assign(apod, apod + size_t(n_tx) * pl->F.C.P.N);
        hip_check(hipGetDevice(&pl->device), "hipGetDevice");
        if (hipMalloc(&pl->dev, pl->F.dv_size) != hipSuccess) {
            pl->dev = nullptr;
            (void)hipGetLastError();
            throw Error{SIMUS_ENOMEM, "plan workspace allocation failed"};
        }
        pl->dev_cap = pl->F.dv_size;
        const hipStream_t st = static_cast<hipStream_t>(hip_stream);
        hip_check(hipMemcpyAsync(pl->dev, pl->F.host.data(), pl->F.up_size, hipMemcpyHostToDevice, st),
                  "hipMemcpyAsync");
        hip_check(hipStreamSynchronize(st), "hipStreamSynchronize");
        *out = pl.release();
    });
}

int simus_rf_plan_execute(simus_rf_plan plan, const float* x, const float* y, const float* z,
                          const float* refl, float* rf, void* hip_stream)
{
    return guarded([&] {
        check_plan_call(plan, x, y, z, refl, rf);
        enqueue_fwd(plan->F, plan->dev, x, y, z, refl, nullptr, rf, static_cast<hipStream_t>(hip_stream));
    });
}

int simus_rf_plan_graph_launch(simus_rf_plan plan, const float* x, const float* y, const float* z,
                               const float* refl, float* rf, void* hip_stream)
{
    return guarded([&] {
        check_plan_call(plan, x, y, z, refl, rf);
        const hipStream_t st = static_cast<hipStream_t>(hip_stream);
        std::lock_guard<std::mutex> lk(plan->mu);
        const void* key[5] = {x, y, z, refl, rf};
        if (!plan->exec || !std::equal(key, key + 5, plan->key)) {
            if (plan->exec) {
                // an earlier launch of the old graph may still run
                hip_check(hipDeviceSynchronize(), "hipDeviceSynchronize");
                hip_check(hipGraphExecDestroy(plan->exec), "hipGraphExecDestroy");
                plan->exec = nullptr;
            }
            if (!plan->cap)
                hip_check(hipStreamCreateWithFlags(&plan->cap, hipStreamNonBlocking), "hipStreamCreate");
            hip_check(hipStreamBeginCapture(plan->cap, hipStreamCaptureModeThreadLocal),
                      "hipStreamBeginCapture");
            hipGraph_t g = nullptr;
            try {
                Untimed untimed;
                enqueue_fwd(plan->F, plan->dev, x, y, z, refl, nullptr, rf, plan->cap);
            } catch (...) {
                (void)hipStreamEndCapture(plan->cap, &g);
                if (g) (void)hipGraphDestroy(g);
                throw;
            }
            hip_check(hipStreamEndCapture(plan->cap, &g), "hipStreamEndCapture");
            const hipError_t e = hipGraphInstantiate(&plan->exec, g, nullptr, nullptr, 0);
            (void)hipGraphDestroy(g);
            if (e != hipSuccess) {
                plan->exec = nullptr;
                hip_check(e, "hipGraphInstantiate");
            }
            std::copy(key, key + 5, plan->key);
        }
        hip_check(timed(K_GRAPH, st, [&] { return hipGraphLaunch(plan->exec, st); }), "hipGraphLaunch");
    });
}

// ---- the autotuner's file cache: one text line per problem class,
// "<key> <shape flags> <scatterers per item / default x 1000> <ms>"
extern "C++" {
namespace {
std::mutex g_tune_mu;
std::string g_tune_path;
int64_t g_tune_hits = 0;

int ilog2(int64_t v)
{
    int b = 0;
    while (v > 1) {
        v >>= 1;
        ++b;
    }
    return b;
}

// The problem class of a plan: path, sub-elements, elements, transmits, y,
// elevation table, 2-D, the caller's flags other than the shape ones, and the
// binary logarithms of the bins, scatterers and phantoms.
std::string tune_key(const FwdPlan& F, int32_t flags)
{
    const Common& C = F.C;
    char buf[256];
    std::snprintf(buf, sizeof buf, "simus%d/%s/M%d/N%d/T%d/y%d/tab%d/2d%d/fl%d/b%d/s%d/p%d", SIMUS_VERSION,
                  F.use_mt ? "mt" : "vec", C.P.M, C.P.N, C.n_tx, C.has_y ? 1 : 0, C.table ? 1 : 0,
                  C.P.dim2 ? 1 : 0, flags, ilog2(std::max(C.B.n_bins, 1)),
                  ilog2(std::max<int64_t>(C.ph.total, 1)), ilog2(std::max(C.ph.n, 1)));
    return buf;
}

// The last line of the cache file for `key`, if any (false if the file does
// not exist or holds no such line).  Caller holds g_tune_mu.
bool tune_lookup(const std::string& key, int32_t* shape_flags, int32_t* mult_permille)
{
    FILE* f = std::fopen(g_tune_path.c_str(), "r");
    if (!f) return false;
    bool found = false;
    char line[512], k[300];
    while (std::fgets(line, sizeof line, f)) {
        int32_t fl = 0, mu = 0;
        double ms = 0;
        if (std::sscanf(line, "%299s %d %d %lf", k, &fl, &mu, &ms) == 4 && key == k && mu > 0) {
            *shape_flags = fl;
            *mult_permille = mu;
            found = true;
        }
    }
    std::fclose(f);
    return found;
}

// Appends one line (written whole); caller holds g_tune_mu.
void tune_store(const std::string& key, int32_t shape_flags, int32_t mult_permille, double ms)
{
    FILE* f = std::fopen(g_tune_path.c_str(), "a");
    if (!f) throw Error{SIMUS_EINVAL, "cannot append to the autotuner cache " + g_tune_path};
    char line[512];
    const int n = std::snprintf(line, sizeof line, "%s %d %d %.4f\n", key.c_str(), shape_flags, mult_permille, ms);
    const bool ok = n > 0 && std::fwrite(line, 1, (size_t)n, f) == (size_t)n;
    if (std::fclose(f) != 0 || !ok) throw Error{SIMUS_EINVAL, "cannot append to the autotuner cache " + g_tune_path};
}
}  // namespace
}  // extern "C++"

int simus_tune_cache(const char* path)
{
    return guarded([&] {
        if (path && std::strlen(path) > 4095) throw Error{SIMUS_EINVAL, "cache path longer than 4095 bytes"};
        std::lock_guard<std::mutex> lk(g_tune_mu);
        g_tune_path = path ? path : "";
    });
}

int64_t simus_tune_cache_hits(void)
{
    std::lock_guard<std::mutex> lk(g_tune_mu);
    return g_tune_hits;
}

int simus_rf_plan_autotune(simus_rf_plan plan, const float* x, const float* y, const float* z,
                           const float* refl, float* rf, void* hip_stream, int64_t* tile_scat,
                           int32_t* flags)
{
    return guarded([&] {
        check_plan_call(plan, x, y, z, refl, rf);
        const hipStream_t st = static_cast<hipStream_t>(hip_stream);
        std::lock_guard<std::mutex> lk(plan->mu);
        const double* dl = plan->delays.data();
        const float* ap = plan->apod.empty() ? nullptr : plan->apod.data();
        // The workspace's tables change below: earlier executions and graph
        // launches of the plan (on any stream) must have finished, and a
        // captured graph is dropped now.
        hip_check(hipDeviceSynchronize(), "hipDeviceSynchronize");
        if (plan->exec) {
            hip_check(hipGraphExecDestroy(plan->exec), "hipGraphExecDestroy");
            plan->exec = nullptr;
        }
        // Uploads a plan's tables into the workspace, growing it first if needed
        // (the old workspace is freed only once the new one exists); waits for
        // the stream.
        auto upload = [&](const FwdPlan& F) {
            if (F.dv_size > plan->dev_cap) {
                void* nd = nullptr;
                if (hipMalloc(&nd, F.dv_size) != hipSuccess) {
                    (void)hipGetLastError();
                    throw Error{SIMUS_ENOMEM, "plan workspace allocation failed"};
                }
                hip_check(hipStreamSynchronize(st), "hipStreamSynchronize");
                (void)hipFree(plan->dev);
                plan->dev = static_cast<char*>(nd);
                plan->dev_cap = F.dv_size;
            }
            hip_check(hipMemcpyAsync(plan->dev, F.host.data(), F.up_size, hipMemcpyHostToDevice, st),
                      "hipMemcpyAsync");
            hip_check(hipStreamSynchronize(st), "hipStreamSynchronize");
        };
        auto rebuild = [&](const simus_options& o) {
            FwdPlan F = make_fwd_plan(Common(plan->F.C), &o, dl, ap, true);
            upload(F);
            return F;
        };
        // candidates: the distinct tile shapes of the default rule and of
        // SIMUS_FLAG_ALT_SHAPE (kernel, element slots, transmit columns, bins
        // per item, product precision); 0.5x .. 2x the default
        // scatterers per item (0.5x, 1x, 2x on the matrix-core path, whose
        // runs are long); on the vector path with and without the persistent
        // launch
        // scatterers per item are tried, and cached, as multiples of the
        // default rule's count for the plan's flags
        const int64_t base = [&] {
            simus_options o = plan->opt;
            o.tile_scat = 0;
            return make_fwd_plan(Common(plan->F.C), &o, dl, ap, true).slice;
        }();
        const int32_t shape_bits = SIMUS_FLAG_ALT_SHAPE;
        std::vector<int32_t> shapes;
        std::vector<SynthConfig> seen;
        std::vector<bool> seen_mt;
        for (const int32_t bits : {0, SIMUS_FLAG_ALT_SHAPE}) {
            simus_options o = plan->opt;
            o.flags = (o.flags & ~shape_bits) | bits;
            const FwdPlan Fo = make_fwd_plan(Common(plan->F.C), &o, dl, ap, true);
            bool dup = false;
            for (size_t i = 0; i < seen.size(); ++i) {
                const SynthConfig& q = seen[i];
                dup = dup || (seen_mt[i] == Fo.use_mt && q.ne == Fo.cfg.ne && q.tt == Fo.cfg.tt &&
                              q.jt == Fo.cfg.jt && q.bs == Fo.cfg.bs && q.nx == Fo.cfg.nx &&
                              q.groups == Fo.cfg.groups && q.pair == Fo.cfg.pair && q.wt == Fo.cfg.wt &&
                              q.bf == Fo.cfg.bf);
            }
            if (dup) continue;
            seen.push_back(Fo.cfg);
            seen_mt.push_back(Fo.use_mt);
            shapes.push_back(o.flags);
        }
        // a choice stored for this problem class
        const int32_t user_flags = plan->opt.flags & ~(shape_bits | SIMUS_FLAG_STATIC);
        const std::string key = tune_key(plan->F, user_flags);
        {
            std::lock_guard<std::mutex> lk(g_tune_mu);
            int32_t cf = 0, mu = 0;
            if (!g_tune_path.empty() && tune_lookup(key, &cf, &mu)) {
                simus_options o = plan->opt;
                o.flags = user_flags | (cf & (shape_bits | SIMUS_FLAG_STATIC));
                o.tile_scat = (int32_t)std::min<int64_t>(
                    std::max<int64_t>(1, std::llround(base * (mu / 1000.0))), int64_t(1) << 30);
                FwdPlan F = make_fwd_plan(Common(plan->F.C), &o, dl, ap, true);
                o.tile_scat = (int32_t)F.slice;
                upload(F);
                plan->F = std::move(F);
                plan->opt = o;
                ++g_tune_hits;
                if (tile_scat) *tile_scat = o.tile_scat;
                if (flags) *flags = o.flags;
                return;
            }
        }
        std::vector<simus_options> cands;
        for (const int32_t shape_flags : shapes)
            for (double m : {0.5, 1.0, 1.5, 2.0}) {
                if (plan->F.use_mt && m == 1.5) continue;
                for (int persist = 0; persist < 2; ++persist) {
                    if (plan->F.use_mt && !persist) continue;   // always persistent there
                    simus_options o = plan->opt;
                    o.flags = shape_flags;
                    o.tile_scat = (int32_t)std::min<int64_t>(
                        std::max<int64_t>(1, std::llround(base * m)), int64_t(1) << 30);
                    o.flags = persist ? (o.flags & ~SIMUS_FLAG_STATIC) : (o.flags | SIMUS_FLAG_STATIC);
                    cands.push_back(o);
                }
            }
        hipEvent_t ev[2] = {nullptr, nullptr};
        hip_check(hipEventCreate(&ev[0]), "hipEventCreate");
        hip_check(hipEventCreate(&ev[1]), "hipEventCreate");
        double best_ms = 0;
        simus_options best = plan->opt;
        try {
            for (size_t c = 0; c < cands.size(); ++c) {
                const FwdPlan F = rebuild(cands[c]);
                // a warm-up run, then three timed runs (one when a run takes
                // over 50 ms)
                float ms = 0.f;
                for (int pass = 0; pass < 2; ++pass) {
                    const int reps = pass == 0 ? 1 : ms > 50.f ? 1 : 3;
                    hip_check(hipEventRecord(ev[0], st), "hipEventRecord");
                    for (int r = 0; r < reps; ++r)
                        enqueue_fwd(F, plan->dev, x, y, z, refl, nullptr, rf, st);
                    hip_check(hipEventRecord(ev[1], st), "hipEventRecord");
                    hip_check(hipEventSynchronize(ev[1]), "hipEventSynchronize");
                    hip_check(hipEventElapsedTime(&ms, ev[0], ev[1]), "hipEventElapsedTime");
                    ms /= reps;
                }
                if (c == 0 || ms < best_ms) {
                    best_ms = ms;
                    best = cands[c];
                    best.tile_scat = F.slice;
                }
            }
        } catch (...) {
            (void)hipEventDestroy(ev[0]);
            (void)hipEventDestroy(ev[1]);
            // the plan keeps its own configuration: put its tables back (the
            // workspace only grew, so it still fits them)
            try {
                upload(plan->F);
            } catch (...) {
            }
            throw;
        }
        hip_check(hipEventDestroy(ev[0]), "hipEventDestroy");
        hip_check(hipEventDestroy(ev[1]), "hipEventDestroy");
        FwdPlan F = make_fwd_plan(Common(plan->F.C), &best, dl, ap, true);
        try {
            upload(F);
        } catch (...) {
            try {
                upload(plan->F);
            } catch (...) {
            }
            throw;
        }
        plan->F = std::move(F);
        plan->opt = best;
        if (tile_scat) *tile_scat = best.tile_scat;
        if (flags) *flags = best.flags;
        std::lock_guard<std::mutex> lk_cache(g_tune_mu);
        if (!g_tune_path.empty())
            tune_store(key, best.flags & (shape_bits | SIMUS_FLAG_STATIC),
                       (int32_t)std::llround(1000.0 * (double)best.tile_scat / (double)std::max<int64_t>(base, 1)),
                       best_ms);
    });
}

void simus_rf_plan_destroy(simus_rf_plan plan) { delete plan; }

int simus_spectrum_to_rf(int32_t nfft, int32_t n_t, int32_t j_lo, int32_t n_bins, int64_t n_chan,
                         const float* spec, float* rf, void* hip_stream)
{
    return guarded([&] {
        if (nfft < 2 || nfft % 2) throw Error{SIMUS_EINVAL, "nfft must be even and >= 2"};
        if (n_t < 0 || n_t > nfft) throw Error{SIMUS_EINVAL, "n_t must be in [0, nfft]"};
        if (n_bins < 0 || j_lo < 0 || int64_t(j_lo) + n_bins > nfft / 2 + 1)
            throw Error{SIMUS_EINVAL, "bins must lie in [0, nfft/2]"};
        if (n_chan < 0) throw Error{SIMUS_EINVAL, "n_chan must be >= 0"};
        if (n_chan > 0 && n_t > 0 && (!spec || !rf)) throw Error{SIMUS_EINVAL, "spec and rf must be non-NULL"};
        const hipStream_t st = static_cast<hipStream_t>(hip_stream);
        hip_check(timed(K_IDFT, st, [&] {
                      return launch_idft(rf, reinterpret_cast<const float2*>(spec), n_chan, n_bins,
                                         j_lo, nfft, n_t, st);
                  }),
                  "inverse transform launch");
    });
}

int simus_profile_enable(int on)
{
    return guarded([&] {
        std::lock_guard<std::mutex> lk(g_prof.mu);
        g_prof.on = on != 0;
    });
}

int simus_profile_read(const char* kernel, double* total_ms, int64_t* launches)
{
    return guarded([&] {
        if (!kernel) throw Error{SIMUS_EINVAL, "kernel name must be non-NULL"};
        int k = -1;
        for (int i = 0; i < K_COUNT; ++i)
            if (std::strcmp(kernel, kKindNames[i]) == 0) k = i;
        if (k < 0) throw Error{SIMUS_EINVAL, std::string("unknown kernel name: ") + kernel};
        std::lock_guard<std::mutex> lk(g_prof.mu);
        g_prof.drain();
        if (total_ms) *total_ms = g_prof.total[k];
        if (launches) *launches = g_prof.count[k];
    });
}

void simus_profile_reset(void)
{
    std::lock_guard<std::mutex> lk(g_prof.mu);
    try {
        g_prof.drain();
    } catch (...) {
    }
    for (int i = 0; i < K_COUNT; ++i) {
        g_prof.total[i] = 0;
        g_prof.count[i] = 0;
    }
}

void simus_release_workspace(void)
{
    std::lock_guard<std::mutex> lk(g_mu);
    for (auto& kv : g_arenas) {
        Arena& a = kv.second;
        int cur = 0;
        (void)hipGetDevice(&cur);
        (void)hipSetDevice(kv.first.first);
        if (a.staged) (void)hipEventSynchronize(a.staged);
        (void)hipDeviceSynchronize();
        if (a.dev) (void)hipFree(a.dev);
        if (a.host) (void)hipHostFree(a.host);
        if (a.staged) (void)hipEventDestroy(a.staged);
        (void)hipSetDevice(cur);
    }
    g_arenas.clear();
}

}  // extern "C"
