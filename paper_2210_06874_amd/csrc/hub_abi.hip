// C ABI of the hot path: argument validation, context and workspace management,
// kernel launches and the host side of the conjugate-gradient driver.
#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <unordered_map>

#include "hub_kernels.hpp"

using namespace hub;

namespace {

constexpr int kThreads51 = 512;     // workgroup size of the L = 51 kernels
// the minimum-norm choice of the Omelyan-Mryglod-Folk second-order integrator
constexpr double kOmelyanLambda = 0.1931833275037836;
constexpr int kHalfBelow = 256;     // two workgroups per slice below this many slices
// FP32 operators at L = 51 and 102 by a degree-5 polynomial of delta kappa K (exp_poly_ratios: the
// Chebyshev series of e^z on [-x, x], x = 3 |delta kappa|, truncated) while x <= 0.25 and its error
// bound is at most kPolyTol (1.1e-8 at x = 0.25, 1.9e-9 at the paper's x = 0.1875), a third of
// FP32's unit roundoff or less; larger steps take the FFT kernels.  The degree-6 Taylor polynomial
// reaches the same accuracy with one sweep more (5-8 % slower).  Two workgroups per slice split
// the 51 columns, four the 102 (each range plus its halos fits 32 lanes); 512 threads: 16 strips
// of 3-4 rows (L = 51; 768 and 1024 measured slower in CG) or 6-7 rows (L = 102).
// FP64 operators at L = 102 by the degree-9 series (2.9e-17 at x = 0.1875; kPolyTol64 is a third
// of FP64's unit roundoff), five workgroups per slice (20-21 columns and 5 halos a side fit 32
// lanes; six, 17 columns each, measured 13 % slower): there the transforms need the three-kernel
// split path.  At L = 51 the FP64 stencil (four
// workgroups per slice) measured 21.4 us per application against 17.9 us for the in-LDS
// transforms, so FP64 at L = 51 keeps those.
constexpr double kPolyMaxX = 0.25;
constexpr int kPolyDeg = 5;
constexpr double kPolyTol = 2e-8;
constexpr int kPolyDeg64 = 9;
constexpr double kPolyTol64 = 4e-17;
constexpr int kThreadsPoly = 512;
template <typename R>
constexpr int poly_deg() { return sizeof(R) == sizeof(float) ? kPolyDeg : kPolyDeg64; }
template <typename R>
constexpr int poly_split(int L) { return sizeof(R) == sizeof(double) ? 5 : (L == 51 ? 2 : 4); }
// row groups: FP64 holds 4 rows per lane in two groups of 51 rows and 5 halos a side (7 rows per
// lane, all 102 rows in one group, spilled in the CG kernels)
template <typename R>
constexpr int poly_rsplit(int) { return sizeof(R) == sizeof(double) ? 2 : 1; }

thread_local char g_err[512] = "";

hub_status fail(hub_status s, const char* fmt, ...) {
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(g_err, sizeof(g_err), fmt, ap);
    va_end(ap);
    return s;
}

#define HIP_OR_FAIL(expr)                                                                  \
    do {                                                                                   \
        hipError_t e_ = (expr);                                                            \
        if (e_ != hipSuccess)                                                              \
            return fail(e_ == hipErrorOutOfMemory ? HUB_ERR_NOMEM : HUB_ERR_DEVICE,        \
                        "%s failed: %s", #expr, hipGetErrorString(e_));                    \
    } while (0)

hub_status launch_check(const char* what) {
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return fail(HUB_ERR_DEVICE, "launch of %s failed: %s", what, hipGetErrorString(e));
    return HUB_OK;
}

// Device scratch of hub_force_noalloc: the per-right-hand-side forces before their sum.
// One copy per GPU, held until the process ends.  Host code never passes the array's name to
// a kernel (on the host it is only a stand-in for the symbol): hub_create looks up each
// device's own address once, with that device current, and the entry point uses that.
constexpr long long kNoAllocScratchDoubles = 1LL << 23;      // 64 MiB
static __device__ __align__(256) double scratch[kNoAllocScratchDoubles];
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
double* g_scratch_ptr[kMaxDevices] = {};
hipError_t g_scratch_err[kMaxDevices] = {};
bool g_scratch_tried[kMaxDevices] = {};

// With `dev` current: look up this device's scratch address (first call per device only).
void lookup_scratch(int dev) {
    if (dev < 0 || dev >= kMaxDevices) return;
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (g_scratch_tried[dev]) return;
    g_scratch_tried[dev] = true;
    void* ptr = nullptr;
    g_scratch_err[dev] = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
    if (g_scratch_err[dev] == hipSuccess) g_scratch_ptr[dev] = static_cast<double*>(ptr);
}

// hub_log_det: dense V x V limit (L <= 24), and the largest |beta| (3|kappa| + |mu|) it accepts.
// That is the log of the bound on the transfer product's largest singular value; the product's
// roundoff grows like 2^-53 e^{that}, about 4e-4 of its largest entry at 29.
constexpr int kLogDetMaxV = 1152;
constexpr double kLogDetMaxGrowth = 29.0;

// Split-path tiles: about this many complex entries per row block and per column block
// (both sublattices), rounded to an even division of L.
constexpr int kSplitRowElems = 2048;
constexpr int kSplitColElems = 2048;
constexpr int kThreadsSplit = 256;  // workgroup size of the compile-time split kernels

constexpr SplitGeom split_geom(int L) {
    SplitGeom g{};
    int rb0 = std::max(1, std::min(L, kSplitRowElems / L));
    g.nrb = (L + rb0 - 1) / rb0;
    g.rb = (L + g.nrb - 1) / g.nrb;
    int cb0 = std::max(1, std::min(L, kSplitColElems / L));
    g.ncb = (L + cb0 - 1) / cb0;
    g.cb = (L + g.ncb - 1) / g.ncb;
    return g;
}

template <typename R>
size_t fused_lds(const hub_ctx* c) { return (size_t)(c->V + c->L) * sizeof(cx<R>); }

template <typename R>
OpTab<R> op_tab(const hub_ctx* c);
template <>
OpTab<double> op_tab<double>(const hub_ctx* c) {
    return {reinterpret_cast<const cx<double>*>(c->roots64), c->etab64, c->plan, c->L, c->V, c->Nt, c->N};
}
template <>
OpTab<float> op_tab<float>(const hub_ctx* c) {
    return {reinterpret_cast<const cx<float>*>(c->roots32), c->etab32, c->plan, c->L, c->V, c->Nt, c->N};
}

// Raise a kernel's dynamic-LDS limit once per (device, kernel), and again for a larger
// size.  A failure here surfaces as a launch error of that kernel.
template <typename K>
void allow_lds(K kern, size_t bytes) {
    static std::mutex mu;
    static std::unordered_map<const void*, size_t> granted[64];
    if (bytes <= 65536) return;
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= 64) dev = 0;
    const void* key = reinterpret_cast<const void*>(kern);
    std::lock_guard<std::mutex> lock(mu);
    auto it = granted[dev].find(key);
    if (it != granted[dev].end() && it->second >= bytes) return;
    if (hipFuncSetAttribute(key, hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes) == hipSuccess)
        granted[dev][key] = bytes;
}

// Which operator kernel runs for nrhs right-hand sides, and how many reduction slots
// (blocks per right-hand side) it has.
enum class OpKind { Generic, Whole51, Half51, Poly, Split, Linear, Sub102 };

// Workgroup size of the sublattice-at-a-time kernel.  Its 84 KB tile allows one workgroup
// per compute unit, so the waves per CU are the workgroup's own: twelve (three per SIMD)
// hide more latency than eight, at the price of a few register spills outside the
// butterfly loops; sixteen spill more.
constexpr int kThreadsSub = 768;

constexpr int kLinBatch = 3;        // sites per thread with loads in flight together
constexpr int kLinTarget = 256;     // fewest workgroups per launch worth splitting slices for

// Linear form: chunks per slice.  Enough workgroups to fill the chip (kLinTarget), and
// chunks small enough for one batch of loads per thread, while the reduction slots per
// right-hand side (Nt * chunks, summed by every workgroup of the next CG kernel) stay
// at most 1024; every chunk holds at least one wavefront of sites.
int lin_nch(const hub_ctx* c, int nrhs) {
    const int slices = nrhs * c->Nt;
    int n = std::max((kLinTarget + slices - 1) / slices, (c->V + kLinBatch * kLinThreads - 1) / (kLinBatch * kLinThreads));
    n = std::min(n, std::max(1, 1024 / c->Nt));
    n = std::min(n, (c->V + 63) / 64);
    return std::max(1, n);
}

// R: the precision of the launch (FP32 slices at L = 102 exceed LDS but one sublattice
// fits; FP64 ones take the split path).
template <typename R>
OpKind op_kind(const hub_ctx* c, int nrhs) {
    if (c->form == HUB_FORM_LINEAR) return OpKind::Linear;
    // FP32 at L = 51 or 102 with small delta kappa: the polynomial stencil; the persistent CG launch
    // is built from the L = 102 sublattice kernel, so with its modes (1, 2) on those operators stay
    // that kernel
    if (c->specialized && c->poly && sizeof(R) == sizeof(float) && !(c->L == 102 && c->persist_mode))
        return OpKind::Poly;
    if (c->specialized && c->poly64 && sizeof(R) == sizeof(double)) return OpKind::Poly;
    if (c->path == HUB_PATH_SPLIT) {
        if (!c->split_forced && c->specialized && c->L == 102 && sizeof(R) == sizeof(float)) return OpKind::Sub102;
        return OpKind::Split;
    }
    if (c->L == 51 && c->specialized) return nrhs * c->Nt < kHalfBelow ? OpKind::Half51 : OpKind::Whole51;
    return OpKind::Generic;
}

template <typename R>
int op_slots(const hub_ctx* c, int nrhs) {
    switch (op_kind<R>(c, nrhs)) {
        case OpKind::Half51: return 2 * c->Nt;
        case OpKind::Poly: return poly_split<R>(c->L) * poly_rsplit<R>(c->L) * c->Nt;
        case OpKind::Split: return 2 * c->Nt * split_geom(c->L).nrb;
        case OpKind::Linear: return c->Nt * lin_nch(c, nrhs);
        default: return c->Nt;
    }
}

// The split path with L and its tiles known at compile time.
template <typename R, int L, int RB, int CB, class Src, class Epi, class Ctl>
hub_status run_split_ct(hub_ctx* c, int nrhs, const OpTab<R>& T, const Src& src, const Epi& epi, const Ctl& ctl,
                        hipStream_t st) {
    cx<R>* W = reinterpret_cast<cx<R>*>(c->split_w);
    const size_t lds_rows = (size_t)(RB * L + L) * sizeof(cx<R>);
    const size_t lds_cols = (size_t)(2 * L * CB + L) * sizeof(cx<R>);
    auto k1 = k_split_rows_fwd_ct<R, L, RB, kThreadsSplit, Src, Ctl>;
    auto k2 = k_split_cols_ct<R, L, CB, kThreadsSplit, Ctl>;
    auto k3 = k_split_rows_inv_ct<R, L, RB, kThreadsSplit, Epi, Ctl>;
    allow_lds(k1, lds_rows);
    allow_lds(k2, lds_cols);
    allow_lds(k3, lds_rows);
    const int nrow_blocks = nrhs * c->Nt * 2 * (L / RB);
    hipLaunchKernelGGL(k1, dim3(nrow_blocks), dim3(kThreadsSplit), lds_rows, st, T, src, W, ctl);
    hub_status s = launch_check("k_split_rows_fwd_ct");
    if (s != HUB_OK) return s;
    hipLaunchKernelGGL(k2, dim3(nrhs * c->Nt * (L / CB)), dim3(kThreadsSplit), lds_cols, st, T, W, ctl);
    s = launch_check("k_split_cols_ct");
    if (s != HUB_OK) return s;
    hipLaunchKernelGGL(k3, dim3(nrow_blocks), dim3(kThreadsSplit), lds_rows, st, T, static_cast<const cx<R>*>(W),
                       epi, ctl);
    return launch_check("k_split_rows_inv_ct");
}

// The polynomial stencil at a compile-time L: poly_split<R>(L) x poly_rsplit<R>(L) workgroups
// per slice.
template <typename R, int L, class Src, class Epi, class Ctl>
hub_status launch_poly(const hub_ctx* c, int nrhs, const OpTab<R>& T, const PolyCoef<R>& pc, const Src& src,
                       const Epi& epi, const Ctl& ctl, hipStream_t st) {
    constexpr int NS = poly_split<R>(L), RS = poly_rsplit<R>(L);
    auto kern = k_exp_poly<R, L, kThreadsPoly, poly_deg<R>(), NS, RS, Src, Epi, Ctl>;
    hipLaunchKernelGGL(kern, dim3(NS * RS * nrhs * c->Nt), dim3(kThreadsPoly), 0, st, T, pc, src, epi, ctl);
    return launch_check(L == 51 ? "k_exp_poly<51>" : "k_exp_poly<102>");
}

// The polynomial stencil with the context's polynomial (OpKind::Poly).
template <typename R, class Src, class Epi, class Ctl>
hub_status run_poly(hub_ctx* c, int nrhs, const OpTab<R>& T, const Src& src, const Epi& epi, const Ctl& ctl,
                    hipStream_t st) {
    constexpr bool f32 = sizeof(R) == sizeof(float);
    PolyCoef<R> pc{};
    pc.scale = (R)(std::exp(c->delta * c->mu) * (f32 ? c->poly_a0 : c->poly64_a0));
    for (int k = 1; k <= poly_deg<R>(); ++k)
        pc.c[k] = (R)(c->delta * c->kappa * (f32 ? c->poly_ratio[k] : c->poly64_ratio[k]));
    if constexpr (f32) {
        if (c->L == 51) return launch_poly<R, 51>(c, nrhs, T, pc, src, epi, ctl, st);
    }
    if (c->L != 102) return fail(HUB_ERR_ARG, "internal: no polynomial stencil at L = %d", c->L);
    return launch_poly<R, 102>(c, nrhs, T, pc, src, epi, ctl, st);
}

// The compile-time L = 51 transform kernels: two workgroups per slice below kHalfBelow slices
// (OpKind::Half51), else one (OpKind::Whole51).
template <typename R, class Src, class Epi, class Ctl>
hub_status run_fused51(hub_ctx* c, int nrhs, OpKind kind, const OpTab<R>& T, const Src& src, const Epi& epi,
                       const Ctl& ctl, hipStream_t st) {
    const size_t lds = fused_lds<R>(c);
    if (kind == OpKind::Half51) {
        auto kern = k_fused_ct<R, 51, kThreads51, true, Src, Epi, Ctl>;
        allow_lds(kern, lds);
        hipLaunchKernelGGL(kern, dim3(2 * nrhs * c->Nt), dim3(kThreads51), lds, st, T, src, epi, ctl);
        return launch_check("k_fused_ct<51, half>");
    }
    auto kern = k_fused_ct<R, 51, kThreads51, false, Src, Epi, Ctl>;
    allow_lds(kern, lds);
    hipLaunchKernelGGL(kern, dim3(nrhs * c->Nt), dim3(kThreads51), lds, st, T, src, epi, ctl);
    return launch_check("k_fused_ct<51>");
}

// The kernels of one OpKind between a source functor and an epilogue functor.
template <typename R, class Src, class Epi, class Ctl>
hub_status run_kind(hub_ctx* c, int nrhs, OpKind kind, const OpTab<R>& T, const Src& src, const Epi& epi,
                    const Ctl& ctl, hipStream_t st) {
    const size_t lds = fused_lds<R>(c);
    switch (kind) {
        case OpKind::Sub102: {
            if constexpr (sizeof(R) == sizeof(float)) {
                auto kern = k_fused_sub<R, 102, kThreadsSub, Src, Epi, Ctl>;
                const size_t lds_sub = (size_t)(c->L * c->L + c->L) * sizeof(cx<R>);
                allow_lds(kern, lds_sub);
                hipLaunchKernelGGL(kern, dim3(nrhs * c->Nt), dim3(kThreadsSub), lds_sub, st, T, src, epi, ctl);
                return launch_check("k_fused_sub<102>");
            }
            return fail(HUB_ERR_ARG, "internal: sublattice kernel is FP32 only");
        }
        case OpKind::Half51:
        case OpKind::Whole51:
            return run_fused51<R>(c, nrhs, kind, T, src, epi, ctl, st);
        case OpKind::Poly:
            return run_poly<R>(c, nrhs, T, src, epi, ctl, st);
        case OpKind::Generic: {
            auto kern = k_fused<R, Src, Epi, Ctl>;
            allow_lds(kern, lds);
            hipLaunchKernelGGL(kern, dim3(nrhs * c->Nt), dim3(kThreads), lds, st, T, src, epi, ctl);
            return launch_check("k_fused");
        }
        case OpKind::Linear:
            return fail(HUB_ERR_ARG, "internal: the linear form has its own kernels");
        case OpKind::Split:
            break;
    }
    if (!c->split_w) return fail(HUB_ERR_ARG, "internal: split path without its scratch vector");
    if (c->specialized && c->L == 102) {
        constexpr SplitGeom G102 = split_geom(102);
        static_assert(102 % G102.rb == 0 && 102 % G102.cb == 0, "tiles must divide L");
        return run_split_ct<R, 102, G102.rb, G102.cb>(c, nrhs, T, src, epi, ctl, st);
    }
    const SplitGeom G = split_geom(c->L);
    cx<R>* W = reinterpret_cast<cx<R>*>(c->split_w);
    const size_t lds_rows = (size_t)(G.rb * c->L + c->L) * sizeof(cx<R>);
    const size_t lds_cols = (size_t)(2 * c->L * G.cb + c->L) * sizeof(cx<R>);
    auto k1 = k_split_rows_fwd<R, Src, Ctl>;
    auto k2 = k_split_cols<R, Ctl>;
    auto k3 = k_split_rows_inv<R, Epi, Ctl>;
    allow_lds(k1, lds_rows);
    allow_lds(k2, lds_cols);
    allow_lds(k3, lds_rows);
    const int nrow_blocks = nrhs * c->Nt * 2 * G.nrb;
    hipLaunchKernelGGL(k1, dim3(nrow_blocks), dim3(kThreads), lds_rows, st, T, G, src, W, ctl);
    hub_status s = launch_check("k_split_rows_fwd");
    if (s != HUB_OK) return s;
    hipLaunchKernelGGL(k2, dim3(nrhs * c->Nt * G.ncb), dim3(kThreads), lds_cols, st, T, G, W, ctl);
    s = launch_check("k_split_cols");
    if (s != HUB_OK) return s;
    hipLaunchKernelGGL(k3, dim3(nrow_blocks), dim3(kThreads), lds_rows, st, T, G, static_cast<const cx<R>*>(W),
                       epi, ctl);
    return launch_check("k_split_rows_inv");
}

// Apply E between a source functor and an epilogue functor over nrhs right-hand sides.
template <typename R, class Src, class Epi, class Ctl>
hub_status run_op(hub_ctx* c, int nrhs, const Src& src, const Epi& epi, const Ctl& ctl_in, hipStream_t st) {
    const OpTab<R> T = op_tab<R>(c);
    const OpKind kind = op_kind<R>(c, nrhs);
    const Ctl ctl = ctl_in.with_slots(op_slots<R>(c, nrhs));
    // the paired x update (EpiUpdate kXSkip / kXPair) is built into the polynomial stencil and,
    // for FP64, the L = 51 transform kernels only (cg_impl pairs nothing else)
    if constexpr (EpiXMode<Epi>::value != kXPlain) {
        if (kind == OpKind::Poly) return run_poly<R>(c, nrhs, T, src, epi, ctl, st);
        if constexpr (sizeof(R) == sizeof(double)) {
            if (kind == OpKind::Half51 || kind == OpKind::Whole51)
                return run_fused51<R>(c, nrhs, kind, T, src, epi, ctl, st);
        }
        return fail(HUB_ERR_ARG, "internal: no paired x update for this kernel");
    } else {
        return run_kind<R>(c, nrhs, kind, T, src, epi, ctl, st);
    }
}

// Linear form: one stencil launch between a source and an output functor.
template <typename R>
LinTab<R> lin_tab(const hub_ctx* c, int nrhs) {
    const int nch = lin_nch(c, nrhs);
    return {c->L, c->L * c->L, c->V, c->Nt, nch, (c->V + nch - 1) / nch, c->N, (R)(c->delta * c->kappa)};
}

template <typename R, bool DAG, class Ph, class Src, class Out, class Ctl>
hub_status run_lin(hub_ctx* c, int nrhs, const Ph& ph, const Src& src, const Out& out, const Ctl& ctl_in,
                   hipStream_t st) {
    const LinTab<R> T = lin_tab<R>(c, nrhs);
    const Ctl ctl = ctl_in.with_slots(op_slots<R>(c, nrhs));
    hipLaunchKernelGGL((k_lin<R, DAG, kLinBatch, Ph, Src, Out, Ctl>), dim3(nrhs * c->Nt * T.nch),
                       dim3(kLinThreads), 0, st, T, ph, src, out, ctl);
    return launch_check(DAG ? "k_lin<dag>" : "k_lin");
}

bool overlaps(const void* a, size_t abytes, const void* b, size_t bbytes) {
    const char* x = static_cast<const char*>(a);
    const char* y = static_cast<const char*>(b);
    return x < y + bbytes && y < x + abytes;
}

// in: nrhs vectors of `elem`-byte entries; out: nrhs vectors (out_per_rhs) or one array of
// N entries of out_elem bytes; phi: N entries of phi_elem bytes.  The output may overlap
// neither input (other workgroups still read them while it is written).
// Every call runs on the current device, which must be the one the context was created on
// (its tables, scratch and the caller's arrays live there).
hub_status check_device(const hub_ctx* c) {
    int dev = -1;
    if (hipGetDevice(&dev) != hipSuccess) return fail(HUB_ERR_DEVICE, "hipGetDevice failed");
    if (dev != c->device)
        return fail(HUB_ERR_ARG, "the context lives on device %d but device %d is current", c->device, dev);
    return HUB_OK;
}

hub_status check_vec_args(const hub_ctx* c, const void* phi, const void* in, const void* out, int nrhs,
                          size_t elem, size_t out_elem, bool out_per_rhs, size_t phi_elem) {
    if (!c) return fail(HUB_ERR_ARG, "ctx is NULL");
    if (!phi || !in || !out) return fail(HUB_ERR_ARG, "NULL array argument");
    if (nrhs < 1 || nrhs > c->nrhs_max)
        return fail(HUB_ERR_ARG, "nrhs=%d outside [1, nrhs_max=%d]", nrhs, c->nrhs_max);
    const size_t in_bytes = (size_t)nrhs * c->N * elem;
    const size_t out_bytes = (size_t)(out_per_rhs ? nrhs : 1) * c->N * out_elem;
    if (overlaps(in, in_bytes, out, out_bytes)) return fail(HUB_ERR_ARG, "input and output overlap");
    if (overlaps(phi, (size_t)c->N * phi_elem, out, out_bytes)) return fail(HUB_ERR_ARG, "phi and output overlap");
    return check_device(c);
}

template <typename R>
hub_status apply_M_impl(hub_ctx* c, const R* phi, const void* in, void* out, int nrhs, void* stream) {
    hub_status s = check_vec_args(c, phi, in, out, nrhs, sizeof(cx<R>), sizeof(cx<R>), true, sizeof(R));
    if (s != HUB_OK) return s;
    const cx<R>* v = static_cast<const cx<R>*>(in);
    if (c->form == HUB_FORM_LINEAR)
        return run_lin<R, false>(c, nrhs, PhAngle<R>{phi}, LSrcVec<R>{v}, LOutStore<R>{static_cast<cx<R>*>(out)},
                                 CtlPlain{}, static_cast<hipStream_t>(stream));
    return run_op<R>(c, nrhs, SrcPhasePrev<R>{v, PhAngle<R>{phi}}, EpiM<R>{v, static_cast<cx<R>*>(out)},
                     CtlPlain{}, static_cast<hipStream_t>(stream));
}

template <typename R>
hub_status apply_Mdag_impl(hub_ctx* c, const R* phi, const void* in, void* out, int nrhs, void* stream) {
    hub_status s = check_vec_args(c, phi, in, out, nrhs, sizeof(cx<R>), sizeof(cx<R>), true, sizeof(R));
    if (s != HUB_OK) return s;
    const cx<R>* v = static_cast<const cx<R>*>(in);
    if (c->form == HUB_FORM_LINEAR)
        return run_lin<R, true>(c, nrhs, PhAngle<R>{phi}, LSrcVec<R>{v}, LOutStore<R>{static_cast<cx<R>*>(out)},
                                CtlPlain{}, static_cast<hipStream_t>(stream));
    return run_op<R>(c, nrhs, SrcNext<R>{v}, EpiMdag<R>{v, static_cast<cx<R>*>(out), PhAngle<R>{phi}},
                     CtlPlain{}, static_cast<hipStream_t>(stream));
}

// ----------------------------------------------------------------------------- time slabs
// A view of the context over the nt slices of one time slab: the kernels index vectors by the
// slab's own slices, while the tables and buffers stay the context's (its buffers hold at least
// nrhs_max * N >= nrhs * nt * V entries).
hub_ctx slab_view(const hub_ctx* c, int nt) {
    hub_ctx v = *c;
    v.Nt = nt;
    v.N = (long long)nt * c->V;
    return v;
}

// Slab arguments: 0 <= t0, nt >= 1, t0 + nt <= Nt; arrays as in check_vec_args with nt slices;
// the halo ([nrhs][V] entries of `elem` bytes, and phi_halo [V] when given) may not overlap out.
hub_status check_slab_args(const hub_ctx* c, int t0, int nt, const void* phi, size_t phi_elem, const void* in,
                           size_t elem, const void* halo, const void* phi_halo, bool need_phi_halo, const void* out,
                           size_t out_elem, bool out_per_rhs, int nrhs) {
    if (!c) return fail(HUB_ERR_ARG, "ctx is NULL");
    if (c->form != HUB_FORM_EXP) return fail(HUB_ERR_ARG, "time slabs are available for HUB_FORM_EXP only");
    if (t0 < 0 || nt < 1 || (long long)t0 + nt > c->Nt)
        return fail(HUB_ERR_ARG, "slab t0=%d nt=%d outside [0, Nt=%d]", t0, nt, c->Nt);
    if (!phi || !in || !halo || !out || (need_phi_halo && !phi_halo)) return fail(HUB_ERR_ARG, "NULL array argument");
    if (nrhs < 1 || nrhs > c->nrhs_max)
        return fail(HUB_ERR_ARG, "nrhs=%d outside [1, nrhs_max=%d]", nrhs, c->nrhs_max);
    const size_t ns = (size_t)nt * c->V;
    const size_t out_bytes = (size_t)(out_per_rhs ? nrhs : 1) * ns * out_elem;
    if (overlaps(in, (size_t)nrhs * ns * elem, out, out_bytes)) return fail(HUB_ERR_ARG, "input and output overlap");
    if (overlaps(phi, ns * phi_elem, out, out_bytes)) return fail(HUB_ERR_ARG, "phi and output overlap");
    if (overlaps(halo, (size_t)nrhs * c->V * elem, out, out_bytes)) return fail(HUB_ERR_ARG, "halo and output overlap");
    if (need_phi_halo && overlaps(phi_halo, (size_t)c->V * phi_elem, out, out_bytes))
        return fail(HUB_ERR_ARG, "phi halo and output overlap");
    return check_device(c);
}

template <typename R>
hub_status apply_M_slab_impl(hub_ctx* c, int t0, int nt, const R* phi, const void* in, const R* phi_halo,
                             const void* in_halo, void* out, int nrhs, void* stream) {
    hub_status s = check_slab_args(c, t0, nt, phi, sizeof(R), in, sizeof(cx<R>), in_halo, phi_halo, true, out,
                                   sizeof(cx<R>), true, nrhs);
    if (s != HUB_OK) return s;
    hub_ctx view = slab_view(c, nt);
    const cx<R>* v = static_cast<const cx<R>*>(in);
    return run_op<R>(&view, nrhs,
                     SrcPhasePrevSlab<R>{v, PhAngle<R>{phi}, static_cast<const cx<R>*>(in_halo), PhAngle<R>{phi_halo}},
                     EpiMSlab<R>{v, static_cast<cx<R>*>(out), t0}, CtlPlain{}, static_cast<hipStream_t>(stream));
}

template <typename R>
hub_status apply_Mdag_slab_impl(hub_ctx* c, int t0, int nt, const R* phi, const void* in, const void* in_halo,
                                void* out, int nrhs, void* stream) {
    hub_status s = check_slab_args(c, t0, nt, phi, sizeof(R), in, sizeof(cx<R>), in_halo, nullptr, false, out,
                                   sizeof(cx<R>), true, nrhs);
    if (s != HUB_OK) return s;
    hub_ctx view = slab_view(c, nt);
    const cx<R>* v = static_cast<const cx<R>*>(in);
    return run_op<R>(&view, nrhs, SrcNextSlab<R>{v, static_cast<const cx<R>*>(in_halo)},
                     EpiMdagSlab<R>{v, static_cast<cx<R>*>(out), PhAngle<R>{phi}, t0, c->Nt}, CtlPlain{},
                     static_cast<hipStream_t>(stream));
}

// Solver workspace, allocated on the first solve.  After a failed allocation the
// buffers already obtained stay with the context (hub_destroy frees them) and a later
// call allocates only the missing ones.
hub_status ensure_cg_workspace(hub_ctx* c) {
    if (c->cg_ready) return HUB_OK;
    const size_t vbytes = (size_t)c->nrhs_max * c->N * sizeof(cx<double>);
    const size_t pbytes = (size_t)c->nrhs_max * c->max_partials * sizeof(double);
    struct Need {
        void** p;
        size_t bytes;
    } need[] = {{&c->cg_rhi, vbytes},
                {&c->cg_tmp, vbytes},
                {&c->cg_x, vbytes},
                {&c->cg_r, vbytes},
                {&c->cg_p, vbytes},
                {&c->cg_t, vbytes},
                {&c->ph64, (size_t)c->N * sizeof(cx<double>)},
                {&c->ph32, (size_t)c->N * sizeof(cx<float>)},
                {reinterpret_cast<void**>(&c->scal), (size_t)c->nrhs_max * sizeof(CgScalars)},
                {reinterpret_cast<void**>(&c->cg_pr), 3 * pbytes},
                {reinterpret_cast<void**>(&c->cg_pt), pbytes}};
    for (const Need& n : need)
        if (!*n.p) HIP_OR_FAIL(hipMalloc(n.p, n.bytes));
    if (!c->scal_host)
        HIP_OR_FAIL(hipHostMalloc(reinterpret_cast<void**>(&c->scal_host), (size_t)c->nrhs_max * sizeof(CgScalars),
                                  hipHostMallocDefault));
    if (!c->cg_event) HIP_OR_FAIL(hipEventCreateWithFlags(&c->cg_event, hipEventDisableTiming));
    if (!c->persist_bar) HIP_OR_FAIL(hipMalloc(reinterpret_cast<void**>(&c->persist_bar), 4 * sizeof(unsigned)));
    if (!c->persist_flag_host)
        HIP_OR_FAIL(hipHostMalloc(reinterpret_cast<void**>(&c->persist_flag_host), 4 * sizeof(unsigned),
                                  hipHostMallocDefault));
    c->cg_ready = true;
    return HUB_OK;
}

// Persistent launch of n FP32 CG iterations at L = 102 (k_cg_persist_sub), when the context
// allows it and every workgroup of a device-filling grid is co-resident.  Returns HUB_OK with
// *done = false when the two-kernel path must run instead (not applicable, or the cooperative
// launch was refused: then never tried again on this context).
hub_status try_persistent(hub_ctx* c, int nrhs, long long from, long long n, const PersistArgs<float>& base,
                          hipStream_t st, bool* done) {
    *done = false;
    if (c->persist_mode != 1 || !c->persist_ok || c->form != HUB_FORM_EXP || op_kind<float>(c, nrhs) != OpKind::Sub102)
        return HUB_OK;
    auto kern = k_cg_persist_sub<float, 102, kThreadsSub>;
    const size_t lds = (size_t)(c->L * c->L + c->L) * sizeof(cx<float>);
    allow_lds(kern, lds);
    if (c->persist_grid < 0) {
        int per_cu = 0, cus = 0;
        if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, reinterpret_cast<const void*>(kern), kThreadsSub,
                                                         lds) != hipSuccess ||
            hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, c->device) != hipSuccess) {
            (void)hipGetLastError();
            per_cu = 0;
        }
        c->persist_grid = per_cu * cus;
    }
    if (c->persist_grid < 8) {
        c->persist_ok = false;
        return HUB_OK;
    }
    const int items = nrhs * c->Nt;
    const int grid = std::min(items, c->persist_grid);
    hipLaunchKernelGGL(k_zero_u32, dim3(1), dim3(64), 0, st, c->persist_bar, 4);
    hub_status s = launch_check("k_zero_u32");
    if (s != HUB_OK) return s;
    PersistArgs<float> a = base;
    a.it0 = from;
    a.n_iter = (int)n;
    a.bar = c->persist_bar;
    a.spin = c->persist_spin;
    const OpTab<float> T = op_tab<float>(c);
    void* args[] = {const_cast<OpTab<float>*>(&T), &a};
    const hipError_t e = hipLaunchCooperativeKernel(reinterpret_cast<const void*>(kern), dim3(grid),
                                                    dim3(kThreadsSub), args, (unsigned)lds, st);
    if (e != hipSuccess) {
        (void)hipGetLastError();
        c->persist_ok = false;          // not co-resident after all: the two-kernel path from now on
        return HUB_OK;
    }
    c->persist_launches += 1;
    *done = true;
    return HUB_OK;
}

// The solver proper, templated on the precision of the inner iterations.
template <typename Rlo>
hub_status cg_impl(hub_ctx* c, const double* phi, const cx<double>* chi, cx<double>* xhi, int nrhs,
                   const hub_cg_opts& o, hub_cg_info* info, hipStream_t st) {
    const bool lin = c->form == HUB_FORM_LINEAR;
    // Phases: e^{i phi} tabulated once per solve in FP64, and in FP32 for FP32 iterations of
    // the exponential form on the transform kernels.  FP32 iterations of the bandwidth-bound
    // stencils (the linear form, the polynomial stencil of the exponential form) read an FP32
    // copy of the angles instead, half the bytes of a table, and evaluate the phase per use on
    // the hardware sin/cos units.
    const bool angles = lin || (sizeof(Rlo) == sizeof(float) && op_kind<Rlo>(c, nrhs) == OpKind::Poly);
    // iterations on the stencils (the polynomial one, the linear form's) and FP64 ones on the
    // L = 51 transform kernels update x every other iteration (EpiUpdate, LOutUpdate)
    const OpKind it_kind = op_kind<Rlo>(c, nrhs);
    const bool paired = lin || it_kind == OpKind::Poly ||
                        (sizeof(Rlo) == sizeof(double) && (it_kind == OpKind::Half51 || it_kind == OpKind::Whole51));
    cx<double>* ph64 = static_cast<cx<double>*>(c->ph64);
    const cx<Rlo>* ph_lo = reinterpret_cast<const cx<Rlo>*>(ph64);
    const Rlo* phi_lo = reinterpret_cast<const Rlo*>(phi);
    hipLaunchKernelGGL(k_phase_table<double>, dim3(1024), dim3(kThreads), 0, st, phi, ph64, c->N);
    hub_status s0 = launch_check("k_phase_table<double>");
    if (s0 != HUB_OK) return s0;
    if constexpr (sizeof(Rlo) == sizeof(float)) {
        if (!angles) {
            hipLaunchKernelGGL(k_phase_table<float>, dim3(1024), dim3(kThreads), 0, st, phi,
                               static_cast<cx<float>*>(c->ph32), c->N);
            s0 = launch_check("k_phase_table<float>");
            ph_lo = reinterpret_cast<const cx<Rlo>*>(c->ph32);
        } else {
            float* phi32 = static_cast<float*>(c->ph32);       // N floats in the table's space
            hipLaunchKernelGGL(k_to_float, dim3(1024), dim3(kThreads), 0, st, phi, phi32, c->N);
            s0 = launch_check("k_to_float");
            phi_lo = reinterpret_cast<const Rlo*>(phi32);
        }
        if (s0 != HUB_OK) return s0;
    }
    const PhTable<Rlo> tab_lo{ph_lo};
    const PhTable<double> tab64{ph64};
    const PhAngle<Rlo> ang_lo{phi_lo};
    cx<double>* rhi = static_cast<cx<double>*>(c->cg_rhi);
    cx<double>* tmp = static_cast<cx<double>*>(c->cg_tmp);
    cx<Rlo>* xlo = static_cast<cx<Rlo>*>(c->cg_x);
    cx<Rlo>* rlo = static_cast<cx<Rlo>*>(c->cg_r);
    cx<Rlo>* p = static_cast<cx<Rlo>*>(c->cg_p);
    cx<Rlo>* tv = static_cast<cx<Rlo>*>(c->cg_t);
    CgScalars* sc = c->scal;
    const int zero_start = o.use_x0 ? 0 : 1;
    const int blocks = nrhs * c->Nt;

    // ||r||^2 partials of iterations i, i-1, i+1 rotate through three buffers (index i mod 3)
    const int slots = op_slots<Rlo>(c, nrhs);   // the iteration kernels' reduction slots
    auto pr = [&](long long i) { return c->cg_pr + (size_t)(i % 3) * nrhs * slots; };
    double* pt = c->cg_pt;

    RedArgs ra{c->partials, c->counters + 1, c->Nt, nrhs};
    hipLaunchKernelGGL(k_cg_init<Rlo>, dim3(blocks), dim3(kThreads), 0, st, chi, xhi, rhi, xlo, rlo, p, c->V,
                       c->Nt, zero_start, FinInit{sc, o.tol, pr(0), pr(2), slots}, ra);
    hub_status s = launch_check("k_cg_init");
    if (s != HUB_OK) return s;
    // the persistent launches' barrier state and abort flag start clear (the host reads the
    // flag with the scalars at every check)
    hipLaunchKernelGGL(k_zero_u32, dim3(1), dim3(64), 0, st, c->persist_bar, 4);
    s = launch_check("k_zero_u32");
    if (s != HUB_OK) return s;

    auto reliable_update = [&](long long i) -> hub_status {
        hipLaunchKernelGGL(k_fold_solution<Rlo>, dim3(512, nrhs), dim3(kThreads), 0, st, xhi, xlo, c->N,
                           static_cast<const CgScalars*>(sc));
        hub_status r = launch_check("k_fold_solution");
        if (r != HUB_OK) return r;
        const RedArgs red{c->partials, c->counters + 3, 0, nrhs};
        const CtlAtomic<FinResidual> fin_ctl{sc, GATE_NOTDONE, red, FinResidual{sc, pr(i), pr(i + 2), slots}};
        if (lin) {
            r = run_lin<double, true>(c, nrhs, tab64, LSrcVec<double>{xhi}, LOutStore<double>{tmp},
                                      CtlGate{sc, GATE_NOTDONE}, st);
            if (r != HUB_OK) return r;
            return run_lin<double, false>(c, nrhs, tab64, LSrcVec<double>{tmp}, LOutResidual<Rlo>{chi, rhi, rlo},
                                          fin_ctl, st);
        }
        r = run_op<double>(c, nrhs, SrcNext<double>{xhi}, EpiMdag<double, PhTable<double>>{xhi, tmp, tab64},
                           CtlGate{sc, GATE_NOTDONE}, st);
        if (r != HUB_OK) return r;
        return run_op<double>(c, nrhs, SrcPhasePrev<double, PhTable<double>>{tmp, tab64},
                              EpiResidual<Rlo>{tmp, chi, rhi, rlo}, fin_ctl, st);
    };

    if (!zero_start) {
        hipLaunchKernelGGL(k_zero_trivial, dim3(blocks), dim3(kThreads), 0, st, xhi, c->V, c->Nt,
                           static_cast<const CgScalars*>(sc));
        s = launch_check("k_zero_trivial");
        if (s != HUB_OK) return s;
        s = reliable_update(0);
        if (s != HUB_OK) return s;
    }

    // Iterations i = from .. from + n - 1: one persistent launch where it applies, else two
    // kernels each.
    c->persist_launches = 0;
    auto queue_iters = [&](long long from, long long n) -> hub_status {
        if (n <= 0) return HUB_OK;
        if constexpr (sizeof(Rlo) == sizeof(float)) {
            if (!lin) {
                const PersistArgs<float> pa{c->cg_pr, pt, sc, slots, nrhs, 0, 0, rlo, p, tv, xlo, tab_lo, nullptr, 0};
                bool done = false;
                const hub_status q = try_persistent(c, nrhs, from, n, pa, st, &done);
                if (q != HUB_OK || done) return q;
            }
        }
        // the phases as the iterations take them: FP32 angles (stencils), else the FP64 table
        const auto ph = [&] {
            if constexpr (sizeof(Rlo) == sizeof(float)) return ang_lo;
            else return tab_lo;
        }();
        using Ph = std::decay_t<decltype(ph)>;
        for (long long i = from; i < from + n; ++i) {
            const CtlSearch k1{pr(i), pr(i + 2), pt, sc, slots};
            const CtlUpdate k2{pr(i), pr(i + 2), pt, pr(i + 1), sc, slots};
            const CtlUpdateT<kXSkip> k2s{pr(i), pr(i + 2), pt, pr(i + 1), sc, slots};
            const CtlUpdateT<kXPair> k2p{pr(i), pr(i + 2), pt, pr(i + 1), sc, slots};
            // paired x updates: iteration j of its block (blocks of reliable_every iterations, the
            // last cut by max_iter) skips x when j is even and adds both terms when j is odd; an
            // even j that ends its block updates x plainly, so no term is pending at the reliable
            // update
            int xm = kXPlain;
            if (paired) {
                const long long b0 = i - i % o.reliable_every, j = i - b0;
                const long long len = std::min<long long>(o.reliable_every, o.max_iter - b0);
                xm = (j % 2 == 1) ? kXPair : (j + 1 < len ? kXSkip : kXPlain);
            }
            hub_status q;
            if (lin) {
                q = run_lin<Rlo, true>(c, nrhs, ph, LSrcSearch<Rlo>{rlo, p}, LOutSearch<Rlo>{tv}, k1, st);
                if (q != HUB_OK) return q;
                if (xm == kXSkip)
                    q = run_lin<Rlo, false>(c, nrhs, ph, LSrcVec<Rlo>{tv}, LOutUpdate<Rlo, kXSkip>{p, xlo, rlo}, k2s, st);
                else if (xm == kXPair)
                    q = run_lin<Rlo, false>(c, nrhs, ph, LSrcVec<Rlo>{tv}, LOutUpdate<Rlo, kXPair>{p, xlo, rlo}, k2p, st);
                else
                    q = run_lin<Rlo, false>(c, nrhs, ph, LSrcVec<Rlo>{tv}, LOutUpdate<Rlo>{p, xlo, rlo}, k2, st);
            } else if (paired) {
                q = run_op<Rlo>(c, nrhs, SrcSearchNext<Rlo>{rlo, p}, EpiSearchMdag<Rlo, Ph>{rlo, p, tv, ph}, k1, st);
                if (q != HUB_OK) return q;
                if (xm == kXSkip)
                    q = run_op<Rlo>(c, nrhs, SrcPhasePrev<Rlo, Ph>{tv, ph}, EpiUpdate<Rlo, kXSkip>{tv, p, xlo, rlo}, k2s,
                                    st);
                else if (xm == kXPair)
                    q = run_op<Rlo>(c, nrhs, SrcPhasePrev<Rlo, Ph>{tv, ph}, EpiUpdate<Rlo, kXPair>{tv, p, xlo, rlo}, k2p,
                                    st);
                else
                    q = run_op<Rlo>(c, nrhs, SrcPhasePrev<Rlo, Ph>{tv, ph}, EpiUpdate<Rlo>{tv, p, xlo, rlo}, k2, st);
            } else if (angles) {
                q = run_op<Rlo>(c, nrhs, SrcSearchNext<Rlo>{rlo, p},
                                EpiSearchMdag<Rlo, PhAngle<Rlo>>{rlo, p, tv, ang_lo}, k1, st);
                if (q != HUB_OK) return q;
                q = run_op<Rlo>(c, nrhs, SrcPhasePrev<Rlo, PhAngle<Rlo>>{tv, ang_lo},
                                EpiUpdate<Rlo>{tv, p, xlo, rlo}, k2, st);
            } else {
                q = run_op<Rlo>(c, nrhs, SrcSearchNext<Rlo>{rlo, p},
                                EpiSearchMdag<Rlo, PhTable<Rlo>>{rlo, p, tv, tab_lo}, k1, st);
                if (q != HUB_OK) return q;
                q = run_op<Rlo>(c, nrhs, SrcPhasePrev<Rlo, PhTable<Rlo>>{tv, tab_lo},
                                EpiUpdate<Rlo>{tv, p, xlo, rlo}, k2, st);
            }
            if (q != HUB_OK) return q;
        }
        return HUB_OK;
    };

    hub_status result = HUB_OK;
    long long it = 0;                  // iterations queued so far
    const int every = o.reliable_every;
    // The host reads the scalars of each reliable update while the device already runs the
    // first iterations of the next block, so the device does not idle during the read.  Those
    // iterations are harmless when the host then stops: every kernel of a finished right-hand
    // side is idle, and otherwise they touch only the iteration vectors, never x or the
    // scalars' host copy, which describe the state at the reliable update.
    const long long lookahead = std::min<long long>(4, every);
    // stagnation watch: per rhs, the best true ||r||^2 seen and the consecutive stalled updates
    std::vector<double> best(nrhs, HUGE_VAL);
    std::vector<int> seen(nrhs, 0), stalled(nrhs, 0), logged(nrhs, 0);
    for (;;) {
        HIP_OR_FAIL(hipMemcpyAsync(c->scal_host, sc, nrhs * sizeof(CgScalars), hipMemcpyDeviceToHost, st));
        HIP_OR_FAIL(hipMemcpyAsync(c->persist_flag_host, c->persist_bar, 4 * sizeof(unsigned), hipMemcpyDeviceToHost,
                                   st));
        HIP_OR_FAIL(hipEventRecord(c->cg_event, st));
        const long long at = it;       // iterations behind the scalars being read
        const long long head = std::min<long long>(lookahead, o.max_iter - it);
        s = queue_iters(it, head);
        if (s != HUB_OK) return s;
        it += head;
        HIP_OR_FAIL(hipEventSynchronize(c->cg_event));
        if (c->persist_launches > 0 && c->persist_flag_host[2] != 0u) {
            (void)hipStreamSynchronize(st);
            return fail(HUB_ERR_DEVICE, "a grid barrier of the persistent CG launch gave up waiting "
                                        "(spin limit %lld polls); x is undefined", c->persist_spin);
        }
        bool all_done = true, bad = false, all_stalled = true;
        for (int r = 0; r < nrhs; ++r) {
            const CgScalars& h = c->scal_host[r];
            all_done &= h.done != 0;
            bad |= h.nonfinite != 0;
            if (o.history_host && h.reliable > logged[r] && h.reliable <= o.history_len) {
                // each host check follows exactly one reliable update
                o.history_host[(size_t)r * o.history_len + h.reliable - 1] =
                    std::sqrt(h.true_rr / (h.chichi > 0 ? h.chichi : 1.0));
                logged[r] = h.reliable;
            }
            if (h.done) continue;
            if (h.reliable > seen[r]) {
                // a stalled update: the iterated residual had met tol, the true one made no
                // 1 % progress (the attainable-accuracy floor); slow progress is not a stall
                seen[r] = h.reliable;
                if (h.true_rr < 0.98 * best[r]) {
                    best[r] = h.true_rr;
                    stalled[r] = 0;
                } else if (h.rec_rr <= h.tol2) {
                    stalled[r] += 1;
                } else {
                    stalled[r] = 0;
                }
            }
            all_stalled &= stalled[r] >= o.stall_updates;
        }
        if (bad) {
            result = fail(HUB_ERR_NONFINITE, "CG breakdown: non-finite or non-positive scalar");
            break;
        }
        if (all_done) break;
        if (o.stall_updates > 0 && all_stalled) {
            result = fail(HUB_ERR_NOCONV, "CG stagnated at its attainable accuracy: %d reliable updates "
                                          "without progress (tol=%g)",
                          o.stall_updates, o.tol);
            break;
        }
        if (at >= o.max_iter) {
            result = fail(HUB_ERR_NOCONV, "CG did not reach tol=%g within max_iter=%d", o.tol, o.max_iter);
            break;
        }
        const long long n = std::min<long long>(every - head, o.max_iter - it);
        s = queue_iters(it, n);
        if (s != HUB_OK) return s;
        it += n;
        s = reliable_update(it);
        if (s != HUB_OK) return s;
    }
    // the iterations queued ahead end before the call returns
    HIP_OR_FAIL(hipStreamSynchronize(st));
    if (c->persist_launches > 0) {
        HIP_OR_FAIL(hipMemcpy(c->persist_flag_host, c->persist_bar, 4 * sizeof(unsigned), hipMemcpyDeviceToHost));
        if (c->persist_flag_host[2] != 0u)
            return fail(HUB_ERR_DEVICE, "a grid barrier of the persistent CG launch gave up waiting "
                                        "(spin limit %lld polls); x is undefined", c->persist_spin);
    }
    if (info) {
        for (int r = 0; r < nrhs; ++r) {
            const CgScalars& h = c->scal_host[r];
            const double cc = h.chichi > 0 ? h.chichi : 1.0;
            info[r].iters = h.iters;
            info[r].reliable_updates = h.reliable;
            info[r].true_rel_res = std::sqrt(h.true_rr / cc);
            info[r].recursive_rel_res = std::sqrt(h.rec_rr / cc);
            info[r].persistent_launches = (int32_t)c->persist_launches;
        }
    }
    return result;
}

}  // namespace

extern "C" {

const char* hub_last_error(void) { return g_err; }

hub_status hub_create(const hub_params* prm, void* stream, hub_ctx** out) {
    if (!out) return fail(HUB_ERR_ARG, "out is NULL");
    *out = nullptr;
    if (!prm) return fail(HUB_ERR_ARG, "params is NULL");
    if (prm->L < 1 || prm->L > 1024) return fail(HUB_ERR_ARG, "L=%d outside [1, 1024]", prm->L);
    if (prm->Nt < 1) return fail(HUB_ERR_ARG, "Nt=%d < 1", prm->Nt);
    if (prm->nrhs_max < 1) return fail(HUB_ERR_ARG, "nrhs_max=%d < 1", prm->nrhs_max);
    if (!std::isfinite(prm->beta) || !std::isfinite(prm->kappa) || !std::isfinite(prm->mu))
        return fail(HUB_ERR_ARG, "beta, kappa and mu must be finite");
    if (prm->path < HUB_PATH_AUTO || prm->path > HUB_PATH_SPLIT) return fail(HUB_ERR_ARG, "bad path %d", prm->path);
    if (prm->form != HUB_FORM_EXP && prm->form != HUB_FORM_LINEAR) return fail(HUB_ERR_ARG, "bad form %d", prm->form);
    const bool lin = prm->form == HUB_FORM_LINEAR;
    if (lin && prm->mu != 0.0) return fail(HUB_ERR_ARG, "the linear form is defined at mu = 0 only");
    FftPlan plan{};
    if (!lin && !make_plan(prm->L, &plan))
        return fail(HUB_ERR_ARG, "L=%d has a prime factor above 17", prm->L);
    const long long N = 2LL * prm->L * prm->L * prm->Nt;
    if ((long long)prm->nrhs_max * N >= (1LL << 40)) return fail(HUB_ERR_ARG, "problem too large");
    // every launch grid must fit a 32-bit block index: at most 2 * max(nrb, ncb) blocks per
    // slice for the transforms (at least the polynomial stencil's 2 at L = 51 and 4 at L = 102), at
    // most max(Nt, 1024) blocks per right-hand side for the linear stencil
    const SplitGeom g = split_geom(prm->L);
    const long long grid_per_rhs = lin ? std::max<long long>(prm->Nt, 1024)
                                       : 2LL * prm->Nt * std::max(g.nrb, g.ncb);
    if ((long long)prm->nrhs_max * grid_per_rhs > INT32_MAX)
        return fail(HUB_ERR_ARG, "nrhs_max * Nt = %lld slices exceed one launch grid",
                    (long long)prm->nrhs_max * prm->Nt);

    hub_ctx* c = new hub_ctx();
    c->L = prm->L;
    c->Nt = prm->Nt;
    c->V = 2 * prm->L * prm->L;
    c->N = N;
    c->nrhs_max = prm->nrhs_max;
    c->beta = prm->beta;
    c->kappa = prm->kappa;
    c->mu = prm->mu;
    c->delta = prm->beta / prm->Nt;
    c->plan = plan;
    c->form = prm->form;
    auto bail = [&](hub_status s) {
        hub_destroy(c);
        return s;
    };
    if (hipGetDevice(&c->device) != hipSuccess) return bail(fail(HUB_ERR_DEVICE, "no HIP device"));
    lookup_scratch(c->device);      // the no-allocation entry point's scratch on this device
    if (hipDeviceGetAttribute(&c->max_lds, hipDeviceAttributeMaxSharedMemoryPerBlock, c->device) != hipSuccess)
        return bail(fail(HUB_ERR_DEVICE, "cannot query LDS size"));
    c->lds_fused64 = (int)fused_lds<double>(c);
    c->lds_fused32 = (int)fused_lds<float>(c);
    const int reserve = 1024;   // static LDS of the reduction
    const bool fits = lin || c->lds_fused64 + reserve <= c->max_lds;
    if (prm->path == HUB_PATH_FUSED && !fits)
        return bail(fail(HUB_ERR_ARG, "fused path needs %d B of LDS, device has %d", c->lds_fused64, c->max_lds));
    c->path = (prm->path == HUB_PATH_SPLIT || (prm->path == HUB_PATH_AUTO && !fits)) ? HUB_PATH_SPLIT
                                                                                      : HUB_PATH_FUSED;
    c->split_forced = prm->path == HUB_PATH_SPLIT;
    {
        const double x = 3.0 * std::fabs(c->delta * c->kappa);
        if (!lin && prm->path == HUB_PATH_AUTO && (c->L == 51 || c->L == 102) && x <= kPolyMaxX) {
            c->poly_err = exp_poly_ratios(x, kPolyDeg, &c->poly_a0, c->poly_ratio);
            c->poly = c->poly_err >= 0.0 && c->poly_err <= kPolyTol;
            if (c->L == 102) {
                c->poly64_err = exp_poly_ratios(x, kPolyDeg64, &c->poly64_a0, c->poly64_ratio);
                c->poly64 = c->poly64_err >= 0.0 && c->poly64_err <= kPolyTol64;
            }
        }
    }

    std::vector<double> roots, etab;
    if (!lin) build_tables(plan, c->delta * c->kappa, c->delta * prm->mu, roots, etab);
    std::vector<float> roots32(roots.begin(), roots.end()), etab32(etab.begin(), etab.end());
    hipStream_t st = static_cast<hipStream_t>(stream);
#define CREATE_OR_BAIL(expr)                                                                   \
    do {                                                                                       \
        hipError_t e_ = (expr);                                                                \
        if (e_ != hipSuccess)                                                                  \
            return bail(fail(e_ == hipErrorOutOfMemory ? HUB_ERR_NOMEM : HUB_ERR_DEVICE,       \
                             "%s failed: %s", #expr, hipGetErrorString(e_)));                  \
    } while (0)
    if (!lin) {
        CREATE_OR_BAIL(hipMalloc(&c->roots64, roots.size() * sizeof(double)));
        CREATE_OR_BAIL(hipMalloc(&c->roots32, roots.size() * sizeof(float)));
        CREATE_OR_BAIL(hipMalloc(&c->etab64, etab.size() * sizeof(double)));
        CREATE_OR_BAIL(hipMalloc(&c->etab32, etab.size() * sizeof(float)));
        CREATE_OR_BAIL(hipMemcpyAsync(c->roots64, roots.data(), roots.size() * sizeof(double), hipMemcpyHostToDevice, st));
        CREATE_OR_BAIL(hipMemcpyAsync(c->roots32, roots32.data(), roots32.size() * sizeof(float), hipMemcpyHostToDevice, st));
        CREATE_OR_BAIL(hipMemcpyAsync(c->etab64, etab.data(), etab.size() * sizeof(double), hipMemcpyHostToDevice, st));
        CREATE_OR_BAIL(hipMemcpyAsync(c->etab32, etab32.data(), etab32.size() * sizeof(float), hipMemcpyHostToDevice, st));
    }

    const SplitGeom G = split_geom(c->L);
    c->max_partials = std::max(2 * c->Nt, c->Nt * 2 * G.nrb);
    c->max_partials = std::max(c->max_partials, c->Nt * lin_nch(c, 1));
    c->max_partials = std::max(c->max_partials, c->Nt * poly_split<double>(c->L) * poly_rsplit<double>(c->L));
    CREATE_OR_BAIL(hipMalloc(&c->partials, (size_t)c->nrhs_max * c->max_partials * sizeof(double)));
    CREATE_OR_BAIL(hipMalloc(&c->counters, kNumCounters * sizeof(unsigned int)));
    CREATE_OR_BAIL(hipMemsetAsync(c->counters, 0, kNumCounters * sizeof(unsigned int), st));
    CREATE_OR_BAIL(hipMalloc(&c->red_out, 8 * sizeof(double)));
    // the split path's scratch vector, unless the stencils take every operator (then FP64 runs the
    // polynomial stencil, FP32 that or the sublattice kernel)
    if (c->path == HUB_PATH_SPLIT && !lin && !c->poly64)
        CREATE_OR_BAIL(hipMalloc(&c->split_w, (size_t)c->nrhs_max * c->N * sizeof(cx<double>)));
    // per-right-hand-side forces before their sum (exponential form, nrhs > 1)
    if (c->nrhs_max > 1 && !lin)
        CREATE_OR_BAIL(hipMalloc(&c->force_tmp, (size_t)c->nrhs_max * c->N * sizeof(double)));
    CREATE_OR_BAIL(hipStreamSynchronize(st));   // host vectors above go out of scope
#undef CREATE_OR_BAIL
    *out = c;
    return HUB_OK;
}

void hub_destroy(hub_ctx* c) {
    if (!c) return;
    int prev = -1;
    const bool switched = hipGetDevice(&prev) == hipSuccess && prev != c->device &&
                          hipSetDevice(c->device) == hipSuccess;
    (void)hipDeviceSynchronize();
    void* dev[] = {c->roots64, c->roots32, c->etab64, c->etab32, c->partials, c->counters, c->red_out,
                   c->split_w, c->cg_rhi, c->cg_tmp, c->cg_x, c->cg_r, c->cg_p, c->cg_t,
                   c->ph64, c->ph32, c->scal, c->cg_pr, c->cg_pt, c->force_tmp,
                   c->tr_chi, c->tr_x, c->tr_pi, c->tr_phi0, c->tr_g, c->tr_E, c->ld_x, c->ld_y};
    for (void* p : dev)
        if (p) (void)hipFree(p);
    if (c->scal_host) (void)hipHostFree(c->scal_host);
    if (c->persist_flag_host) (void)hipHostFree(c->persist_flag_host);
    if (c->persist_bar) (void)hipFree(c->persist_bar);
    if (c->tr_E_host) (void)hipHostFree(c->tr_E_host);
    if (c->cg_event) (void)hipEventDestroy(c->cg_event);
    delete c;
    if (switched) (void)hipSetDevice(prev);
}

hub_status hub_apply_M(hub_ctx* c, const double* phi, const void* in, void* out, int32_t nrhs, void* st) {
    return apply_M_impl<double>(c, phi, in, out, nrhs, st);
}
hub_status hub_apply_Mdag(hub_ctx* c, const double* phi, const void* in, void* out, int32_t nrhs, void* st) {
    return apply_Mdag_impl<double>(c, phi, in, out, nrhs, st);
}
hub_status hub_apply_M_c64(hub_ctx* c, const float* phi, const void* in, void* out, int32_t nrhs, void* st) {
    return apply_M_impl<float>(c, phi, in, out, nrhs, st);
}
hub_status hub_apply_Mdag_c64(hub_ctx* c, const float* phi, const void* in, void* out, int32_t nrhs, void* st) {
    return apply_Mdag_impl<float>(c, phi, in, out, nrhs, st);
}

hub_status hub_cg_solve(hub_ctx* c, const double* phi, const void* chi, void* x, int32_t nrhs,
                        const hub_cg_opts* opts, hub_cg_info* info, void* stream) {
    hub_status s = check_vec_args(c, phi, chi, x, nrhs, sizeof(cx<double>), sizeof(cx<double>), true, sizeof(double));
    if (s != HUB_OK) return s;
    if (!opts) return fail(HUB_ERR_ARG, "opts is NULL");
    if (!(opts->tol > 0.0) || !std::isfinite(opts->tol)) return fail(HUB_ERR_ARG, "tol must be > 0");
    if (opts->max_iter < 1) return fail(HUB_ERR_ARG, "max_iter must be >= 1");
    if (opts->reliable_every < 1) return fail(HUB_ERR_ARG, "reliable_every must be >= 1");
    if (opts->prec != HUB_PREC_FP64 && opts->prec != HUB_PREC_MIXED) return fail(HUB_ERR_ARG, "bad prec");
    if (opts->use_x0 != 0 && opts->use_x0 != 1) return fail(HUB_ERR_ARG, "use_x0 must be 0 or 1");
    if (opts->stall_updates < 0) return fail(HUB_ERR_ARG, "stall_updates must be >= 0");
    if (opts->history_len < 0 || (opts->history_len > 0 && !opts->history_host))
        return fail(HUB_ERR_ARG, "history_len must be >= 0, with history_host set when > 0");
    s = ensure_cg_workspace(c);
    if (s != HUB_OK) return s;
    hipStream_t st = static_cast<hipStream_t>(stream);
    const cx<double>* chi_c = static_cast<const cx<double>*>(chi);
    cx<double>* x_c = static_cast<cx<double>*>(x);
    if (opts->prec == HUB_PREC_MIXED) return cg_impl<float>(c, phi, chi_c, x_c, nrhs, *opts, info, st);
    return cg_impl<double>(c, phi, chi_c, x_c, nrhs, *opts, info, st);
}

hub_status hub_force(hub_ctx* c, const double* phi, const void* x, double* g, int32_t nrhs, void* stream) {
    hub_status s = check_vec_args(c, phi, x, g, nrhs, sizeof(cx<double>), sizeof(double), false, sizeof(double));
    if (s != HUB_OK) return s;
    hipStream_t st = static_cast<hipStream_t>(stream);
    const cx<double>* xv = static_cast<const cx<double>*>(x);
    if (c->form == HUB_FORM_LINEAR) {
        const int blocks = (int)std::min<long long>((c->N + kThreads - 1) / kThreads, 4096);
        hipLaunchKernelGGL(k_lin_force, dim3(blocks), dim3(kThreads), 0, st, lin_tab<double>(c, 1), phi, xv, g, nrhs);
        return launch_check("k_lin_force");
    }
    if (nrhs == 1)
        return run_op<double>(c, 1, SrcNext<double>{xv}, EpiForce{xv, {phi}, g, 0}, CtlPlain{}, st);
    s = run_op<double>(c, nrhs, SrcNext<double>{xv}, EpiForce{xv, {phi}, c->force_tmp, c->N}, CtlPlain{}, st);
    if (s != HUB_OK) return s;
    hipLaunchKernelGGL(k_sum_rhs, dim3(1024), dim3(kThreads), 0, st, c->force_tmp, g, c->N, nrhs);
    return launch_check("k_sum_rhs");
}

hub_status hub_apply_M_slab(hub_ctx* c, int32_t t0, int32_t nt, const double* phi, const void* in,
                            const double* phi_halo, const void* in_halo, void* out, int32_t nrhs, void* st) {
    return apply_M_slab_impl<double>(c, t0, nt, phi, in, phi_halo, in_halo, out, nrhs, st);
}
hub_status hub_apply_Mdag_slab(hub_ctx* c, int32_t t0, int32_t nt, const double* phi, const void* in,
                               const void* in_halo, void* out, int32_t nrhs, void* st) {
    return apply_Mdag_slab_impl<double>(c, t0, nt, phi, in, in_halo, out, nrhs, st);
}
hub_status hub_apply_M_slab_c64(hub_ctx* c, int32_t t0, int32_t nt, const float* phi, const void* in,
                                const float* phi_halo, const void* in_halo, void* out, int32_t nrhs, void* st) {
    return apply_M_slab_impl<float>(c, t0, nt, phi, in, phi_halo, in_halo, out, nrhs, st);
}
hub_status hub_apply_Mdag_slab_c64(hub_ctx* c, int32_t t0, int32_t nt, const float* phi, const void* in,
                                   const void* in_halo, void* out, int32_t nrhs, void* st) {
    return apply_Mdag_slab_impl<float>(c, t0, nt, phi, in, in_halo, out, nrhs, st);
}

hub_status hub_force_slab(hub_ctx* c, int32_t t0, int32_t nt, const double* phi, const void* x,
                          const void* x_halo, double* g, int32_t nrhs, void* stream) {
    hub_status s = check_slab_args(c, t0, nt, phi, sizeof(double), x, sizeof(cx<double>), x_halo, nullptr, false, g,
                                   sizeof(double), false, nrhs);
    if (s != HUB_OK) return s;
    hipStream_t st = static_cast<hipStream_t>(stream);
    hub_ctx view = slab_view(c, nt);
    const cx<double>* xv = static_cast<const cx<double>*>(x);
    const SrcNextSlab<double> src{xv, static_cast<const cx<double>*>(x_halo)};
    if (nrhs == 1) return run_op<double>(&view, 1, src, EpiForceSlab{xv, {phi}, g, 0, t0, c->Nt}, CtlPlain{}, st);
    s = run_op<double>(&view, nrhs, src, EpiForceSlab{xv, {phi}, c->force_tmp, view.N, t0, c->Nt}, CtlPlain{}, st);
    if (s != HUB_OK) return s;
    hipLaunchKernelGGL(k_sum_rhs, dim3(1024), dim3(kThreads), 0, st, static_cast<const double*>(c->force_tmp), g,
                       view.N, nrhs);
    return launch_check("k_sum_rhs");
}

hub_status hub_force_noalloc(hub_ctx* c, const double* phi, const void* x, double* g, int32_t nrhs, void* stream) {
    hub_status s = check_vec_args(c, phi, x, g, nrhs, sizeof(cx<double>), sizeof(double), false, sizeof(double));
    if (s != HUB_OK) return s;
    if (c->form == HUB_FORM_LINEAR || nrhs == 1) return hub_force(c, phi, x, g, nrhs, stream);   // no scratch
    if ((long long)nrhs * c->N > kNoAllocScratchDoubles)
        return fail(HUB_ERR_ARG, "nrhs * N = %lld exceeds the static scratch of %lld doubles",
                    (long long)nrhs * c->N, kNoAllocScratchDoubles);
    double* sp = (c->device >= 0 && c->device < kMaxDevices) ? g_scratch_ptr[c->device] : nullptr;
    if (!sp)
        return fail(HUB_ERR_DEVICE, "no static scratch on device %d: %s", c->device,
                    hipGetErrorString(c->device >= 0 && c->device < kMaxDevices ? g_scratch_err[c->device]
                                                                                 : hipErrorInvalidDevice));
    hipStream_t st = static_cast<hipStream_t>(stream);
    const cx<double>* xv = static_cast<const cx<double>*>(x);
    s = run_op<double>(c, nrhs, SrcNext<double>{xv}, EpiForce{xv, {phi}, sp, c->N}, CtlPlain{}, st);
    if (s != HUB_OK) return s;
    hipLaunchKernelGGL(k_sum_rhs, dim3(1024), dim3(kThreads), 0, st, static_cast<const double*>(sp), g, c->N, nrhs);
    return launch_check("k_sum_rhs");
}

hub_status hub_log_det(hub_ctx* c, const double* phi, double* out_dev, void* stream) {
    if (!c) return fail(HUB_ERR_ARG, "ctx is NULL");
    if (!phi || !out_dev) return fail(HUB_ERR_ARG, "NULL array argument");
    if (c->form != HUB_FORM_EXP) return fail(HUB_ERR_ARG, "hub_log_det is available for HUB_FORM_EXP only");
    if (c->V > kLogDetMaxV) return fail(HUB_ERR_ARG, "V=%d above the dense limit %d of hub_log_det", c->V, kLogDetMaxV);
    const double growth = std::fabs(c->beta) * (3.0 * std::fabs(c->kappa) + std::fabs(c->mu));
    if (growth > kLogDetMaxGrowth)
        return fail(HUB_ERR_ARG, "|beta| (3|kappa| + |mu|) = %g above %g: the unstabilised transfer product "
                                 "would lose the determinant", growth, kLogDetMaxGrowth);
    if (overlaps(phi, (size_t)c->N * sizeof(double), out_dev, 2 * sizeof(double)))
        return fail(HUB_ERR_ARG, "phi and output overlap");
    if (hub_status d = check_device(c); d != HUB_OK) return d;
    const size_t mb = (size_t)c->V * c->V * sizeof(cx<double>);
    if (!c->ld_x) HIP_OR_FAIL(hipMalloc(&c->ld_x, mb));
    if (!c->ld_y) HIP_OR_FAIL(hipMalloc(&c->ld_y, mb));
    hipStream_t st = static_cast<hipStream_t>(stream);
    cx<double>* X = static_cast<cx<double>*>(c->ld_x);
    cx<double>* Y = static_cast<cx<double>*>(c->ld_y);
    hipLaunchKernelGGL(k_identity, dim3(256), dim3(kThreads), 0, st, X, c->V);
    hub_status s = launch_check("k_identity");
    if (s != HUB_OK) return s;
    // X <- E D_t X for t = 0 .. Nt-1: the V columns are the "slices" of one launch per slice
    hub_ctx view = slab_view(c, c->V);
    view.N = (long long)c->V * c->V;
    view.path = HUB_PATH_FUSED;           // a slice of V <= 1152 sites always fits LDS: no split scratch
    view.split_forced = false;
    for (int t = 0; t < c->Nt; ++t) {
        s = run_op<double>(&view, 1, SrcPhaseCol<double>{X, PhAngle<double>{phi + (size_t)t * c->V}},
                           EpiStore<double>{Y}, CtlPlain{}, st);
        if (s != HUB_OK) return s;
        std::swap(X, Y);
    }
    hipLaunchKernelGGL(k_add_identity, dim3((c->V + kThreads - 1) / kThreads), dim3(kThreads), 0, st, X, c->V);
    s = launch_check("k_add_identity");
    if (s != HUB_OK) return s;
    hipLaunchKernelGGL(k_lu_logdet, dim3(1), dim3(kLuThreads), 2 * c->V * sizeof(cx<double>), st, X, c->V, out_dev);
    return launch_check("k_lu_logdet");
}

hub_status hub_action(hub_ctx* c, const void* chi, const void* x, int32_t nrhs, double* S_dev, void* stream) {
    if (!c) return fail(HUB_ERR_ARG, "ctx is NULL");
    if (!chi || !x || !S_dev) return fail(HUB_ERR_ARG, "NULL array argument");
    if (nrhs < 1 || nrhs > c->nrhs_max) return fail(HUB_ERR_ARG, "nrhs=%d outside [1, %d]", nrhs, c->nrhs_max);
    if (hub_status d = check_device(c); d != HUB_OK) return d;
    hipStream_t st = static_cast<hipStream_t>(stream);
    RedArgs ra{c->partials, c->counters + 6, c->Nt, nrhs};
    hipLaunchKernelGGL(k_dot_re, dim3(nrhs * c->Nt), dim3(kThreads), 0, st, static_cast<const cx<double>*>(chi),
                       static_cast<const cx<double>*>(x), c->V, c->Nt, FinStore{S_dev, nrhs}, ra);
    return launch_check("k_dot_re");
}

hub_status hub_md_update(hub_ctx* c, double* phi, double* pi, const double* dSdphi, double U, double eps_pi,
                         double eps_phi, void* stream) {
    if (!c) return fail(HUB_ERR_ARG, "ctx is NULL");
    if (!phi || !pi || !dSdphi) return fail(HUB_ERR_ARG, "NULL array argument");
    if (!(U > 0.0) || !std::isfinite(U) || !std::isfinite(eps_pi) || !std::isfinite(eps_phi))
        return fail(HUB_ERR_ARG, "U must be > 0 and the step sizes finite");
    const size_t bytes = (size_t)c->N * sizeof(double);
    if (overlaps(phi, bytes, pi, bytes) || overlaps(phi, bytes, dSdphi, bytes) || overlaps(pi, bytes, dSdphi, bytes))
        return fail(HUB_ERR_ARG, "phi, pi and dSdphi must not overlap");
    if (hub_status d = check_device(c); d != HUB_OK) return d;
    hipStream_t st = static_cast<hipStream_t>(stream);
    hipLaunchKernelGGL(k_md_update, dim3(1024), dim3(kThreads), 0, st, phi, pi, dSdphi, c->N, 1.0 / (c->delta * U),
                       eps_pi, eps_phi);
    return launch_check("k_md_update");
}

hub_status hub_boson_energy(hub_ctx* c, const double* phi, const double* pi, double U, double* out_dev,
                            void* stream) {
    if (!c) return fail(HUB_ERR_ARG, "ctx is NULL");
    if (!phi || !pi || !out_dev) return fail(HUB_ERR_ARG, "NULL array argument");
    if (!(U > 0.0) || !std::isfinite(U)) return fail(HUB_ERR_ARG, "U must be > 0");
    if (hub_status d = check_device(c); d != HUB_OK) return d;
    hipStream_t st = static_cast<hipStream_t>(stream);
    RedArgs ra{c->partials, c->counters + 7, c->Nt, 1};
    hipLaunchKernelGGL(k_boson_energy, dim3(c->Nt), dim3(kThreads), 0, st, phi, pi, c->V, 1.0 / (c->delta * U),
                       FinStore{out_dev, 1}, ra);
    return launch_check("k_boson_energy");
}

hub_status hub_trajectory(hub_ctx* c, double* phi, const double* pi0, const void* rho, int32_t nrhs, double u,
                          const hub_traj_opts* o, hub_traj_info* info, void* stream) {
    if (!c) return fail(HUB_ERR_ARG, "ctx is NULL");
    if (!phi || !pi0 || !rho || !o) return fail(HUB_ERR_ARG, "NULL argument");
    if (nrhs < 1 || nrhs > c->nrhs_max) return fail(HUB_ERR_ARG, "nrhs=%d outside [1, %d]", nrhs, c->nrhs_max);
    if (!(o->U > 0.0) || !std::isfinite(o->U) || !(o->eps > 0.0) || !std::isfinite(o->eps) || o->n_md < 1)
        return fail(HUB_ERR_ARG, "U and eps must be finite and > 0, n_md >= 1");
    if (o->integrator != HUB_MD_LEAPFROG && o->integrator != HUB_MD_OMELYAN)
        return fail(HUB_ERR_ARG, "bad integrator %d", o->integrator);
    if (!std::isfinite(u)) return fail(HUB_ERR_ARG, "u must be finite");
    const size_t fb = (size_t)c->N * sizeof(double), vb = (size_t)nrhs * c->N * sizeof(cx<double>);
    if (overlaps(phi, fb, pi0, fb) || overlaps(phi, fb, rho, vb)) return fail(HUB_ERR_ARG, "phi overlaps pi0 or rho");
    if (hub_status d = check_device(c); d != HUB_OK) return d;
    // workspace, kept by the context (a failed allocation leaves the others for the next call)
    const size_t wb = (size_t)c->nrhs_max * c->N * sizeof(cx<double>);
    struct Need {
        void** p;
        size_t bytes;
    } need[] = {{&c->tr_chi, wb}, {&c->tr_x, wb}, {reinterpret_cast<void**>(&c->tr_pi), fb},
                {reinterpret_cast<void**>(&c->tr_phi0), fb}, {reinterpret_cast<void**>(&c->tr_g), fb},
                {reinterpret_cast<void**>(&c->tr_E), 2 * sizeof(double)}};
    for (const Need& n : need)
        if (!*n.p) HIP_OR_FAIL(hipMalloc(n.p, n.bytes));
    if (!c->tr_E_host)
        HIP_OR_FAIL(hipHostMalloc(reinterpret_cast<void**>(&c->tr_E_host), 2 * sizeof(double), hipHostMallocDefault));

    hipStream_t st = static_cast<hipStream_t>(stream);
    cx<double>* chi = static_cast<cx<double>*>(c->tr_chi);
    cx<double>* x = static_cast<cx<double>*>(c->tr_x);
    double* pi = c->tr_pi;
    double* g = c->tr_g;
    HIP_OR_FAIL(hipMemcpyAsync(c->tr_phi0, phi, fb, hipMemcpyDeviceToDevice, st));
    HIP_OR_FAIL(hipMemcpyAsync(pi, pi0, fb, hipMemcpyDeviceToDevice, st));
    bool restore = true;              // until the decision, a failure puts the start field back
    auto finish = [&](hub_status status) -> hub_status {
        if (restore) (void)hipMemcpyAsync(phi, c->tr_phi0, fb, hipMemcpyDeviceToDevice, st);
        const hipError_t e = hipStreamSynchronize(st);
        if (status == HUB_OK && e != hipSuccess)
            return fail(HUB_ERR_DEVICE, "hipStreamSynchronize failed: %s", hipGetErrorString(e));
        return status;
    };

    hub_status s = hub_apply_M(c, phi, rho, chi, nrhs, stream);     // heat bath chi = M rho
    if (s != HUB_OK) return finish(s);
    hub_cg_opts cg = o->cg;
    cg.history_host = nullptr;        // one history per solve would overwrite itself
    cg.history_len = 0;
    std::vector<hub_cg_info> ci(nrhs);
    int iters = 0, n_forces = 0;
    auto solve = [&](int use_x0) -> hub_status {
        cg.use_x0 = use_x0;
        const hub_status r = hub_cg_solve(c, phi, chi, x, nrhs, &cg, ci.data(), stream);
        int m = 0;
        for (const hub_cg_info& i : ci) m = std::max(m, (int)i.iters);
        iters += m;
        return r;
    };
    auto energy = [&](double* H) -> hub_status {
        hub_status r = hub_boson_energy(c, phi, pi, o->U, c->tr_E, stream);
        if (r != HUB_OK) return r;
        r = hub_action(c, chi, x, nrhs, c->tr_E + 1, stream);
        if (r != HUB_OK) return r;
        HIP_OR_FAIL(hipMemcpyAsync(c->tr_E_host, c->tr_E, 2 * sizeof(double), hipMemcpyDeviceToHost, st));
        HIP_OR_FAIL(hipStreamSynchronize(st));
        *H = c->tr_E_host[0] + c->tr_E_host[1];
        return HUB_OK;
    };
    // solve at the current field, then the force and one update (eps_pi, eps_phi)
    auto kick = [&](bool warm, double eps_pi, double eps_phi) -> hub_status {
        if (warm) {
            const hub_status r = solve(1);
            if (r != HUB_OK) return r;
        }
        hub_status r = hub_force(c, phi, x, g, nrhs, stream);
        if (r != HUB_OK) return r;
        ++n_forces;
        return hub_md_update(c, phi, pi, g, o->U, eps_pi, eps_phi, stream);
    };

    s = solve(0);
    if (s != HUB_OK) return finish(s);
    double H0 = 0.0, H1 = 0.0;
    s = energy(&H0);
    if (s != HUB_OK) return finish(s);
    const double eps = o->eps;
    const int n = o->n_md;
    if (o->integrator == HUB_MD_LEAPFROG) {
        s = kick(false, 0.5 * eps, eps);
        for (int k = 1; k <= n && s == HUB_OK; ++k)
            s = k < n ? kick(true, eps, eps) : kick(true, 0.5 * eps, 0.0);
    } else {
        const double lam = kOmelyanLambda;
        s = kick(false, lam * eps, 0.5 * eps);
        for (int k = 1; k <= n && s == HUB_OK; ++k) {
            s = kick(true, (1.0 - 2.0 * lam) * eps, 0.5 * eps);
            if (s == HUB_OK) s = k < n ? kick(true, 2.0 * lam * eps, 0.5 * eps) : kick(true, lam * eps, 0.0);
        }
    }
    if (s != HUB_OK) return finish(s);
    s = energy(&H1);
    if (s != HUB_OK) return finish(s);
    const double dH = H1 - H0;
    const bool accepted = dH <= 0.0 || u < std::exp(-dH);
    restore = !accepted;
    if (info) {
        info->accepted = accepted ? 1 : 0;
        info->n_forces = n_forces;
        info->cg_iters = iters;
        info->H0 = H0;
        info->H1 = H1;
        info->dH = dH;
    }
    return finish(HUB_OK);
}

hub_status hub_set_cg_launch(hub_ctx* c, int32_t persistent, int64_t barrier_spin_limit) {
    if (!c) return fail(HUB_ERR_ARG, "ctx is NULL");
    if (persistent < 0 || persistent > 2) return fail(HUB_ERR_ARG, "persistent must be 0, 1 or 2");
    if (barrier_spin_limit < 0) return fail(HUB_ERR_ARG, "barrier_spin_limit must be >= 0");
    c->persist_mode = persistent;
    c->persist_spin = barrier_spin_limit > 0 ? (long long)barrier_spin_limit : (1LL << 24);
    return HUB_OK;
}

hub_status hub_query(const hub_ctx* c, int32_t* path, int32_t* lds_bytes) {
    if (!c) return fail(HUB_ERR_ARG, "ctx is NULL");
    if (c->form == HUB_FORM_LINEAR) {
        if (path) *path = HUB_PATH_FUSED;
        if (lds_bytes) *lds_bytes = 0;
        return HUB_OK;
    }
    if (path) *path = c->path;
    if (lds_bytes) {
        const SplitGeom G = split_geom(c->L);
        *lds_bytes = c->path == HUB_PATH_FUSED ? c->lds_fused64
                                               : (int)((2 * c->L * G.cb + c->L) * sizeof(cx<double>));
    }
    return HUB_OK;
}

}  // extern "C"
