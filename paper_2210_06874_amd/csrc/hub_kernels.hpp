// Device kernels of the hot path: the operator kernels (fused one-slice-per-workgroup
// layout and the three-kernel split layout for slices larger than LDS), the
// source/epilogue functors that specialise them into M, M^dag, the CG steps, the
// reliable update and the force, and the deterministic last-block reductions.
#pragma once

#include <type_traits>

#include "hub_fft.hpp"
#include "hub_math.hpp"

namespace hub {

constexpr int kThreads = 256;

// Tables and sizes every operator kernel needs.
template <typename R>
struct OpTab {
    const cx<R>* roots;   // [L]
    const R* etab;        // [L*L][4]
    FftPlan plan;
    int L, V, Nt;
    long long N;
};

// Reduction plumbing shared by all kernels that reduce.
struct RedArgs {
    double* partials;        // [nrhs][slots]
    unsigned int* counter;
    int slots;               // partial slots per right-hand side
    int nrhs;
};

// Sum of a wave's 64 values in a fixed order, returned to every lane: each row of 16 lanes is
// summed into its lane 15 by DPP right shifts, the rows are combined into lane 63 by DPP row
// broadcasts, and lane 63's value is read back as a scalar.  Every lane must be active.
template <int CTRL, int ROWS>
__device__ __forceinline__ double dpp_move_f64(double v) {
    const unsigned long long b = (unsigned long long)__double_as_longlong(v);
    const unsigned lo = __builtin_amdgcn_update_dpp(0, (int)(unsigned)b, CTRL, ROWS, 0xf, false);
    const unsigned hi = __builtin_amdgcn_update_dpp(0, (int)(unsigned)(b >> 32), CTRL, ROWS, 0xf, false);
    return __longlong_as_double((long long)(((unsigned long long)hi << 32) | lo));
}
__device__ __forceinline__ double wave_sum(double v) {
    v += dpp_move_f64<0x111, 0xf>(v);            // row_shr:1
    v += dpp_move_f64<0x112, 0xf>(v);            // row_shr:2
    v += dpp_move_f64<0x114, 0xf>(v);            // row_shr:4
    v += dpp_move_f64<0x118, 0xf>(v);            // row_shr:8 (lane 15 of a row: the row's sum)
    v += dpp_move_f64<0x142, 0xa>(v);            // row_bcast:15 into rows 1 and 3
    v += dpp_move_f64<0x143, 0xc>(v);            // row_bcast:31 into rows 2 and 3 (lane 63: the sum)
    const unsigned long long b = (unsigned long long)__double_as_longlong(v);
    const unsigned lo = __builtin_amdgcn_readlane((int)(unsigned)b, 63);
    const unsigned hi = __builtin_amdgcn_readlane((int)(unsigned)(b >> 32), 63);
    return __longlong_as_double((long long)(((unsigned long long)hi << 32) | lo));
}

// Block-wide sum in a fixed order (result valid in thread 0).
__device__ __forceinline__ double block_sum(double v, double* lds) {
    v = wave_sum(v);
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    __syncthreads();
    if (lane == 0) lds[wave] = v;
    __syncthreads();
    double s = 0.0;
    if (threadIdx.x == 0) {
        const int nw = (blockDim.x + 63) >> 6;
        for (int w = 0; w < nw; ++w) s += lds[w];
    }
    return s;
}

// Block-wide sum in a fixed order, returned to every thread.
__device__ __forceinline__ double block_allsum(double v, double* lds) {
    const double s = block_sum(v, lds);
    __shared__ double bcast;
    if (threadIdx.x == 0) bcast = s;
    __syncthreads();
    return bcast;
}


// K sums of `n` partials each, returned to every thread, in a fixed order.  Up to
// kWaveSlots partials every wave forms the sums on its own (lane l adds slots l, l + 64,
// l + 128, ... in turn, then the wave sum): no LDS traffic and one barrier.  Above that thread
// t adds slots t, t + blockDim, ... and the wave sums meet in LDS (the order then depends on
// blockDim, the same in every block of a kernel).  Either way every block of a kernel forms the
// same sums.  Ends with a barrier, as callers may rely on.  `lds` needs K * (waves per block)
// doubles.
constexpr int kPartialsPerLane = 4;
constexpr int kWaveSlots = 64 * kPartialsPerLane;

// the first slot a thread adds and the stride to its next
__device__ __forceinline__ int2 partial_walk(int n) {
    return n <= kWaveSlots ? make_int2((int)threadIdx.x & 63, 64) : make_int2((int)threadIdx.x, (int)blockDim.x);
}

template <int K>
__device__ __forceinline__ void finish_partials(int n, double (&v)[K], double* lds, double (&out)[K]) {
#pragma unroll
    for (int k = 0; k < K; ++k) v[k] = wave_sum(v[k]);
    if (n <= kWaveSlots) {
#pragma unroll
        for (int k = 0; k < K; ++k) out[k] = v[k];
        __syncthreads();
        return;
    }
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int nw = (blockDim.x + 63) >> 6;
    __syncthreads();
    if (lane == 0) {
#pragma unroll
        for (int k = 0; k < K; ++k) lds[wave * K + k] = v[k];
    }
    __syncthreads();
#pragma unroll
    for (int k = 0; k < K; ++k) {
        double s = 0.0;
        for (int w = 0; w < nw; ++w) s += lds[w * K + k];
        out[k] = s;
    }
    __syncthreads();
}

template <int K>
__device__ __forceinline__ void sum_partials_k(const double* const (&p)[K], int n, double* lds, double (&out)[K]) {
    const int2 w = partial_walk(n);
    double v[K];
#pragma unroll
    for (int k = 0; k < K; ++k) v[k] = 0.0;
    for (int j = w.x; j < n; j += w.y) {
#pragma unroll
        for (int k = 0; k < K; ++k) v[k] += p[k][j];
    }
    finish_partials<K>(n, v, lds, out);
}

// The first kPartialsPerLane partials of each of K arrays that this thread adds (clamped into
// range), loaded ahead of a kernel's other global loads: the memory counter is waited on in
// issue order, so partials loaded after the prefetch of the operands would make every wave wait
// for all of those before it could form the CG scalars.
template <int K>
struct PartialsPre {
    double v[K][kPartialsPerLane];
    double tol2;                 // and the right-hand side's state, from the scalars
    int done, nonfinite, iters;
};

template <int K>
__device__ __forceinline__ PartialsPre<K> prefetch_partials(const double* const (&p)[K], int n,
                                                            const CgScalars& s) {
    PartialsPre<K> r;
    const int2 w = partial_walk(n);
#pragma unroll
    for (int k = 0; k < K; ++k)
#pragma unroll
        for (int i = 0; i < kPartialsPerLane; ++i) r.v[k][i] = p[k][min(w.x + w.y * i, n - 1)];
    r.tol2 = s.tol2;
    r.done = s.done;
    r.nonfinite = s.nonfinite;
    r.iters = s.iters;
    return r;
}

// sum_partials_k with each thread's first partials already loaded (same order, same sums).
template <int K>
__device__ __forceinline__ void sum_partials_pre(const double* const (&p)[K], int n, const PartialsPre<K>& pre,
                                                 double* lds, double (&out)[K]) {
    const int2 w = partial_walk(n);
    double v[K];
#pragma unroll
    for (int k = 0; k < K; ++k) {
        double a = 0.0;
#pragma unroll
        for (int i = 0; i < kPartialsPerLane; ++i)
            if (w.x + w.y * i < n) a += pre.v[k][i];
        v[k] = a;
    }
    for (int j = w.x + w.y * kPartialsPerLane; j < n; j += w.y) {
#pragma unroll
        for (int k = 0; k < K; ++k) v[k] += p[k][j];
    }
    finish_partials<K>(n, v, lds, out);
}

struct NoCtlPre {};

// What an operator kernel's block learns before it starts: whether it works at all,
// and the CG step scalars.
struct Scal {
    int open;
    double alpha, beta;
    double alpha_prev = 0.0;     // paired x updates (EpiUpdate kXPair): the previous iteration's alpha
    int pending = 0;             // and whether its alpha_prev * p is still to be added to x
};

// Store this block's partial, and let the block that arrives last sum every right-hand
// side's partials in slot order and call fin.finish(rhs, sum, lds) in all of its threads.
// Deterministic: the final sums
// never depend on arrival order.  `lds` needs 64 doubles.
//
// The partials and the arrival counter are device-scope relaxed atomics (coherent
// across XCDs without writing back or invalidating the L2s); the partial's store is
// complete (s_waitcnt) before the counter increment is issued, so the block that sees
// the final count reads every partial.
template <class Fin>
__device__ __forceinline__ void reduce_and_finalize(double acc, int rhs, int slot, const RedArgs& ra,
                                                    const Fin& fin, double* lds) {
    __shared__ int is_last;
    const double s = block_sum(acc, lds);
    if (threadIdx.x == 0) {
        __hip_atomic_store(&ra.partials[(long long)rhs * ra.slots + slot], s, __ATOMIC_RELAXED,
                           __HIP_MEMORY_SCOPE_AGENT);
        __atomic_signal_fence(__ATOMIC_SEQ_CST);
        __builtin_amdgcn_s_waitcnt(0);
        __atomic_signal_fence(__ATOMIC_SEQ_CST);
        const unsigned prev = __hip_atomic_fetch_add(ra.counter, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        is_last = (prev == gridDim.x * gridDim.y * gridDim.z - 1) ? 1 : 0;
    }
    __syncthreads();
    if (!is_last) return;
    for (int r = 0; r < ra.nrhs; ++r) {
        double v = 0.0;
        for (int j = threadIdx.x; j < ra.slots; j += blockDim.x)
            v += __hip_atomic_load(&ra.partials[(long long)r * ra.slots + j], __ATOMIC_RELAXED,
                                   __HIP_MEMORY_SCOPE_AGENT);
        fin.finish(r, block_allsum(v, lds), lds);
    }
    if (threadIdx.x == 0) __hip_atomic_store(ra.counter, 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// ----------------------------------------------------------------------------- gating
// Solver kernels skip right-hand sides whose solve is done; gating is uniform per block.
enum Gate : int { GATE_NONE = 0, GATE_NOTDONE = 1 };

__device__ __forceinline__ bool gate_open(const CgScalars* sc, int gate, int rhs) {
    return gate == GATE_NONE || sc[rhs].done == 0;
}

__device__ __forceinline__ int prev_slice(int t, int Nt) { return t == 0 ? Nt - 1 : t - 1; }
__device__ __forceinline__ int next_slice(int t, int Nt) { return t == Nt - 1 ? 0 : t + 1; }

// ----------------------------------------------------------------------------- phases
// Where the phases e^{i phi} come from: the angles themselves (evaluated per use), or
// a table of e^{i phi} computed once (the solver computes one per solve).
template <typename R>
struct PhAngle {
    using Pre = R;
    const R* phi;
    __device__ Pre fetch(long long k) const { return phi[k]; }
    __device__ cx<R> value(Pre a) const {
        R s, c;
        if constexpr (sizeof(R) == sizeof(float)) phase_sincos_fast(a, &s, &c);
        else phase_sincos(a, &s, &c);
        return {c, s};
    }
};

template <typename R>
struct PhTable {
    using Pre = cx<R>;
    const cx<R>* tab;
    __device__ Pre fetch(long long k) const { return tab[k]; }
    __device__ cx<R> value(Pre a) const { return a; }
};

// ----------------------------------------------------------------------------- sources
// A source functor names the slice that feeds destination slice t and produces its
// entries (before E acts) in two steps: fetch() issues the global loads into a
// per-entry record, make() turns the record into the complex entry.  Kernels that
// know their trip counts issue every fetch before the first make.
template <typename R, class Ph>
struct PrePh {
    cx<R> v;
    typename Ph::Pre ph;
};

template <typename R, class Ph = PhAngle<R>>
struct SrcPhasePrev {            // e^{i phi_{t-1}} v_{t-1}            (M)
    using Pre = PrePh<R, Ph>;
    const cx<R>* v;
    Ph ph;
    __device__ int slice(int t, int Nt) const { return prev_slice(t, Nt); }
    __device__ Pre fetch(int rhs, int ts, int i, const OpTab<R>& T) const {
        const long long k = (long long)ts * T.V + i;
        return {v[rhs * T.N + k], ph.fetch(k)};
    }
    __device__ cx<R> make(const Pre& a, const Scal&) const { return cmul(a.v, ph.value(a.ph)); }
};

template <typename R>
struct SrcNext {                 // v_{t+1}                            (M^dag, force)
    using Pre = cx<R>;
    const cx<R>* v;
    __device__ int slice(int t, int Nt) const { return next_slice(t, Nt); }
    __device__ Pre fetch(int rhs, int ts, int i, const OpTab<R>& T) const {
        return v[rhs * T.N + (long long)ts * T.V + i];
    }
    __device__ cx<R> make(const Pre& a, const Scal&) const { return a; }
};

template <typename R>
struct PrePair {
    cx<R> a, b;
};

template <typename R>
struct SrcSearchNext {           // (r + beta p)_{t+1}                 (CG: M^dag of the new direction)
    using Pre = PrePair<R>;
    const cx<R>* r;
    const cx<R>* p;
    __device__ int slice(int t, int Nt) const { return next_slice(t, Nt); }
    __device__ Pre fetch(int rhs, int ts, int i, const OpTab<R>& T) const {
        const long long k = rhs * T.N + (long long)ts * T.V + i;
        return {r[k], p[k]};
    }
    __device__ cx<R> make(const Pre& a, const Scal& s) const {
        const R b = (R)s.beta;
        return {a.a.re + b * a.b.re, a.a.im + b * a.b.im};
    }
};

// ----------------------------------------------------------------------------- epilogues
// An epilogue functor receives w = (E src)_{t,i} for destination slice t and site i.
// fetch() issues the loads the epilogue needs, store() writes its outputs and adds its
// contribution to the block's reduction.  early() does the part of the epilogue that
// does not need w (kernels call it for every entry before store(), as soon as the
// fetched operands have arrived, so its stores overlap the transform).  Only epilogues
// that declare kEarly = true have one.
template <class Epi, class = void>
struct EpiHasEarly : std::false_type {};
template <class Epi>
struct EpiHasEarly<Epi, std::void_t<decltype(Epi::kEarly)>> : std::bool_constant<Epi::kEarly> {};

// epilogues with a step for blocks that do no work (EpiUpdate's pending x term)
template <class Epi, class = void>
struct EpiHasClosed : std::false_type {};
template <class Epi>
struct EpiHasClosed<Epi, std::void_t<decltype(&Epi::closed)>> : std::true_type {};

// the x-update form of an epilogue (EpiUpdate's kXMode), kXPlain for every other
template <class Epi, class = void>
struct EpiXMode : std::integral_constant<int, 0> {};
template <class Epi>
struct EpiXMode<Epi, std::void_t<decltype(Epi::kXMode)>> : std::integral_constant<int, Epi::kXMode> {};

template <typename R, class Epi>
__device__ __forceinline__ void epi_early(const Epi& epi, int rhs, int t, int i, typename Epi::Pre& a,
                                          const OpTab<R>& T, const Scal& sc) {
    if constexpr (EpiHasEarly<Epi>::value) epi.early(rhs, t, i, a, T, sc);
}
template <typename R>
struct EpiM {                    // out_t = v_t - B_t w
    using Pre = cx<R>;
    const cx<R>* v;
    cx<R>* out;
    __device__ Pre fetch(int rhs, int t, int i, const OpTab<R>& T) const {
        return v[rhs * T.N + (long long)t * T.V + i];
    }
    __device__ void store(int rhs, int t, int i, cx<R> w, const Pre& a, const OpTab<R>& T, const Scal&,
                          double&) const {
        out[rhs * T.N + (long long)t * T.V + i] = (t == 0) ? a + w : a - w;
    }
};

template <typename R, class Ph = PhAngle<R>>
struct EpiMdag {                 // out_t = v_t - B_{t+1} e^{-i phi_t} w
    using Pre = PrePh<R, Ph>;
    const cx<R>* v;
    cx<R>* out;
    Ph ph;
    __device__ Pre fetch(int rhs, int t, int i, const OpTab<R>& T) const {
        const long long ks = (long long)t * T.V + i;
        return {v[rhs * T.N + ks], ph.fetch(ks)};
    }
    __device__ void store(int rhs, int t, int i, cx<R> w, const Pre& a, const OpTab<R>& T, const Scal&,
                          double&) const {
        const cx<R> pw = cmulc(w, ph.value(a.ph));
        out[rhs * T.N + (long long)t * T.V + i] = (t == T.Nt - 1) ? a.v + pw : a.v - pw;
    }
};

template <typename R, class Ph>
struct PreSearch {
    cx<R> r, p;
    typename Ph::Pre ph;
};

template <typename R, class Ph = PhAngle<R>>
struct EpiSearchMdag {           // CG: tv_t = (r + beta p)_t - B_{t+1} e^{-i phi_t} w ; acc |tv|^2
    using Pre = PreSearch<R, Ph>;
    const cx<R>* r;
    const cx<R>* p;
    cx<R>* tv;
    Ph ph;
    __device__ Pre fetch(int rhs, int t, int i, const OpTab<R>& T) const {
        const long long ks = (long long)t * T.V + i;
        const long long k = rhs * T.N + ks;
        return {r[k], p[k], ph.fetch(ks)};
    }
    __device__ void store(int rhs, int t, int i, cx<R> w, const Pre& a, const OpTab<R>& T, const Scal& sc,
                          double& acc) const {
        const R b = (R)sc.beta;
        const cx<R> pn = {a.r.re + b * a.p.re, a.r.im + b * a.p.im};
        const cx<R> pw = cmulc(w, ph.value(a.ph));
        const cx<R> o = (t == T.Nt - 1) ? pn + pw : pn - pw;
        tv[rhs * T.N + (long long)t * T.V + i] = o;
        acc += (double)o.re * (double)o.re + (double)o.im * (double)o.im;
    }
};

template <typename R>
struct PreUpdate {
    cx<R> tq, p, x, r;
};
template <typename R>
struct PreUpdateNoX {
    cx<R> tq, p, r;
};

// How the CG update step treats x (the update x_{i+1} = x_i + alpha_i p_i).  Plain: every
// iteration.  Paired: an even iteration of a block skips x (it leaves alpha_i p_i pending and
// keeps alpha_i in the scalars) and the odd one after it adds both terms, alpha_i p_i +
// alpha_{i+1} p_{i+1}, from the p_i it reads and the p_{i+1} it forms: x is read and written
// every other iteration, 16 of the step's 60 bytes per site-slice.  A right-hand side that falls
// idle after a skip adds its pending term in the next (paired) step; the host gives the last
// iteration of an odd-length block the plain form, so no term is pending at a reliable update.
constexpr int kXPlain = 0, kXSkip = 1, kXPair = 2;

template <typename R, int XM = kXPlain>
struct EpiUpdate {               // CG: p = r + beta p; x += alpha p (early); q = tv_t - B_t w; r -= alpha q; acc |r|^2
    using Pre = std::conditional_t<XM == kXSkip, PreUpdateNoX<R>, PreUpdate<R>>;
    static constexpr bool kEarly = true;
    static constexpr int kXMode = XM;
    const cx<R>* tv;
    cx<R>* p;
    cx<R>* x;
    cx<R>* r;
    __device__ Pre fetch(int rhs, int t, int i, const OpTab<R>& T) const {
        const long long k = rhs * T.N + (long long)t * T.V + i;
        if constexpr (XM == kXSkip) return {tv[k], p[k], r[k]};
        else return {tv[k], p[k], x[k], r[k]};
    }
    __device__ void early(int rhs, int t, int i, Pre& a, const OpTab<R>& T, const Scal& sc) const {
        const long long k = rhs * T.N + (long long)t * T.V + i;
        const R b = (R)sc.beta, al = (R)sc.alpha;
        const cx<R> pn = {a.r.re + b * a.p.re, a.r.im + b * a.p.im};
        p[k] = pn;
        if constexpr (XM == kXPlain) {
            x[k] = {a.x.re + al * pn.re, a.x.im + al * pn.im};
        } else if constexpr (XM == kXPair) {
            const R ap = (R)sc.alpha_prev;
            x[k] = {fmar(al, pn.re, fmar(ap, a.p.re, a.x.re)), fmar(al, pn.im, fmar(ap, a.p.im, a.x.im))};
        }
    }
    // a paired step of a right-hand side that went idle after the skip: add the pending term
    __device__ void closed(int rhs, int t, int i, const Pre& a, const OpTab<R>& T, const Scal& sc) const {
        if constexpr (XM == kXPair) {
            const long long k = rhs * T.N + (long long)t * T.V + i;
            const R ap = (R)sc.alpha_prev;
            x[k] = {fmar(ap, a.p.re, a.x.re), fmar(ap, a.p.im, a.x.im)};
        }
    }
    __device__ void store(int rhs, int t, int i, cx<R> w, const Pre& a, const OpTab<R>& T, const Scal& sc,
                          double& acc) const {
        const long long k = rhs * T.N + (long long)t * T.V + i;
        const R al = (R)sc.alpha;
        const cx<R> q = (t == 0) ? a.tq + w : a.tq - w;
        const cx<R> rn = {a.r.re - al * q.re, a.r.im - al * q.im};
        r[k] = rn;
        acc += (double)rn.re * (double)rn.re + (double)rn.im * (double)rn.im;
    }
};

template <typename Rlo>
struct EpiResidual {             // FP64: r_hi = chi - (y_t - B_t w) with y = M^dag x_hi; r_lo = r_hi; acc |r_hi|^2
    using Pre = PrePair<double>;
    const cx<double>* y;
    const cx<double>* chi;
    cx<double>* rhi;
    cx<Rlo>* rlo;
    __device__ Pre fetch(int rhs, int t, int i, const OpTab<double>& T) const {
        const long long k = rhs * T.N + (long long)t * T.V + i;
        return {y[k], chi[k]};
    }
    __device__ void store(int rhs, int t, int i, cx<double> w, const Pre& a, const OpTab<double>& T, const Scal&,
                          double& acc) const {
        const long long k = rhs * T.N + (long long)t * T.V + i;
        const cx<double> q = (t == 0) ? a.a + w : a.a - w;
        const cx<double> rv = a.b - q;
        rhi[k] = rv;
        rlo[k] = {(Rlo)rv.re, (Rlo)rv.im};
        acc += rv.re * rv.re + rv.im * rv.im;
    }
};

struct EpiForce {                // g_t = -2 B_{t+1} Im(e^{i phi_t} x_t conj(w)),  w = (E x_{t+1})
    using Pre = PrePh<double, PhAngle<double>>;
    const cx<double>* x;
    PhAngle<double> ph;
    double* g;                   // [nrhs or 1][Nt][V]
    long long g_rhs_stride;      // 0 when there is one right-hand side
    __device__ Pre fetch(int rhs, int t, int i, const OpTab<double>& T) const {
        const long long ks = (long long)t * T.V + i;
        return {x[rhs * T.N + ks], ph.fetch(ks)};
    }
    __device__ void store(int rhs, int t, int i, cx<double> w, const Pre& a, const OpTab<double>& T, const Scal&,
                          double&) const {
        const long long ks = (long long)t * T.V + i;
        const cx<double> z = cmulc(cmul(a.v, ph.value(a.ph)), w);
        const double bn = (t == T.Nt - 1) ? -1.0 : 1.0;
        g[rhs * g_rhs_stride + ks] = -2.0 * bn * z.im;
    }
};

// ----------------------------------------------------------------------------- time slabs
// One shard of a time-sharded vector: the kernels run over the slab's nt slices (OpTab's
// Nt and N are the slab's), the slice across the slab's edge comes from a halo buffer
// ([nrhs][V], one slice per right-hand side), and the antiperiodic sign is taken at the
// global slice t0 + t of a lattice of Ntg slices.  The halo branch is uniform per block.
template <typename R, class Ph = PhAngle<R>>
struct SrcPhasePrevSlab {        // e^{i phi_{t-1}} v_{t-1}; slab slice -1 is the halo (M)
    using Pre = PrePh<R, Ph>;
    const cx<R>* v;
    Ph ph;
    const cx<R>* vh;             // v at global slice t0 - 1
    Ph phh;                      // phi at global slice t0 - 1
    __device__ int slice(int t, int) const { return t - 1; }
    __device__ Pre fetch(int rhs, int ts, int i, const OpTab<R>& T) const {
        if (ts < 0) return {vh[(long long)rhs * T.V + i], phh.fetch(i)};
        const long long k = (long long)ts * T.V + i;
        return {v[rhs * T.N + k], ph.fetch(k)};
    }
    __device__ cx<R> make(const Pre& a, const Scal&) const { return cmul(a.v, ph.value(a.ph)); }
};

template <typename R>
struct SrcNextSlab {             // v_{t+1}; slab slice nt is the halo (M^dag, force)
    using Pre = cx<R>;
    const cx<R>* v;
    const cx<R>* vh;             // v at global slice t0 + nt
    __device__ int slice(int t, int) const { return t + 1; }
    __device__ Pre fetch(int rhs, int ts, int i, const OpTab<R>& T) const {
        if (ts >= T.Nt) return vh[(long long)rhs * T.V + i];
        return v[rhs * T.N + (long long)ts * T.V + i];
    }
    __device__ cx<R> make(const Pre& a, const Scal&) const { return a; }
};

template <typename R>
struct EpiMSlab {                // out_t = v_t - B_{t0+t} w
    using Pre = cx<R>;
    const cx<R>* v;
    cx<R>* out;
    int t0;
    __device__ Pre fetch(int rhs, int t, int i, const OpTab<R>& T) const {
        return v[rhs * T.N + (long long)t * T.V + i];
    }
    __device__ void store(int rhs, int t, int i, cx<R> w, const Pre& a, const OpTab<R>& T, const Scal&,
                          double&) const {
        out[rhs * T.N + (long long)t * T.V + i] = (t0 + t == 0) ? a + w : a - w;
    }
};

template <typename R>
struct EpiMdagSlab {             // out_t = v_t - B_{t0+t+1} e^{-i phi_t} w
    using Pre = PrePh<R, PhAngle<R>>;
    const cx<R>* v;
    cx<R>* out;
    PhAngle<R> ph;
    int t0, Ntg;
    __device__ Pre fetch(int rhs, int t, int i, const OpTab<R>& T) const {
        const long long ks = (long long)t * T.V + i;
        return {v[rhs * T.N + ks], ph.fetch(ks)};
    }
    __device__ void store(int rhs, int t, int i, cx<R> w, const Pre& a, const OpTab<R>& T, const Scal&,
                          double&) const {
        const cx<R> pw = cmulc(w, ph.value(a.ph));
        out[rhs * T.N + (long long)t * T.V + i] = (t0 + t == Ntg - 1) ? a.v + pw : a.v - pw;
    }
};

struct EpiForceSlab {            // g_t = -2 B_{t0+t+1} Im(e^{i phi_t} x_t conj(w)),  w = (E x_{t+1})
    using Pre = PrePh<double, PhAngle<double>>;
    const cx<double>* x;
    PhAngle<double> ph;
    double* g;                   // [nrhs or 1][nt][V]
    long long g_rhs_stride;      // 0 when there is one right-hand side
    int t0, Ntg;
    __device__ Pre fetch(int rhs, int t, int i, const OpTab<double>& T) const {
        const long long ks = (long long)t * T.V + i;
        return {x[rhs * T.N + ks], ph.fetch(ks)};
    }
    __device__ void store(int rhs, int t, int i, cx<double> w, const Pre& a, const OpTab<double>& T, const Scal&,
                          double&) const {
        const long long ks = (long long)t * T.V + i;
        const cx<double> z = cmulc(cmul(a.v, ph.value(a.ph)), w);
        const double bn = (t0 + t == Ntg - 1) ? -1.0 : 1.0;
        g[rhs * g_rhs_stride + ks] = -2.0 * bn * z.im;
    }
};

// ----------------------------------------------------------------------------- Sec. 3 weight
// The transfer-matrix product E D_{Nt-1} ... E D_0 applied to the V columns of a V x V matrix:
// one launch per slice, column j of the matrix is "slice" j of the launch.
template <typename R>
struct SrcPhaseCol {             // e^{i phi_t} X[:, j]   (ph points at slice t of phi)
    using Pre = PrePh<R, PhAngle<R>>;
    const cx<R>* X;
    PhAngle<R> ph;
    __device__ int slice(int j, int) const { return j; }
    __device__ Pre fetch(int, int j, int i, const OpTab<R>& T) const {
        return {X[(long long)j * T.V + i], ph.fetch(i)};
    }
    __device__ cx<R> make(const Pre& a, const Scal&) const { return cmul(a.v, ph.value(a.ph)); }
};

struct NoPre {};

template <typename R>
struct EpiStore {                // out = w
    using Pre = NoPre;
    cx<R>* out;
    __device__ Pre fetch(int, int, int, const OpTab<R>&) const { return {}; }
    __device__ void store(int rhs, int t, int i, cx<R> w, const Pre&, const OpTab<R>& T, const Scal&, double&) const {
        out[rhs * T.N + (long long)t * T.V + i] = w;
    }
};

// fetch + store in one call (kernels that do not prefetch)
template <typename R, class Epi>
__device__ __forceinline__ void epi_apply(const Epi& epi, int rhs, int t, int i, cx<R> w, const OpTab<R>& T,
                                          const Scal& sc, double& acc) {
    typename Epi::Pre a = epi.fetch(rhs, t, i, T);
    epi_early<R>(epi, rhs, t, i, a, T, sc);
    epi.store(rhs, t, i, w, a, T, sc, acc);
}

template <typename R, class Src>
__device__ __forceinline__ cx<R> src_apply(const Src& src, int rhs, int ts, int i, const OpTab<R>& T,
                                           const Scal& sc) {
    return src.make(src.fetch(rhs, ts, i, T), sc);
}

// ----------------------------------------------------------------------------- finalizers
// finish(r, total, lds) is called by every thread of the block that arrives last, once per
// right-hand side in order, with the right-hand side's total (the same in every thread).
// Finalizers without block-wide work act in thread 0 only.
struct FinResidual {             // after an FP64 residual recomputation (CG reliable update)
    CgScalars* sc;
    double* rr_cur;              // ||r||^2 partials the next CG iteration starts from, [nrhs][slots]
    double* rr_prev;             // and those of the iteration before
    int slots;
    __device__ void finish(int r, double rr, double* lds) const {
        if (sc[r].done) return;                  // uniform: read before any thread writes
        double* cur = rr_cur + (long long)r * slots;
        double* prev = rr_prev + (long long)r * slots;
        const double* const pc[1] = {cur};
        double sum[1];
        sum_partials_k<1>(pc, slots, lds, sum);
        const double rec = sum[0];
        // The recursion's beta for the next iteration is rec / ||r_i||^2 of the last iteration
        // that did work.  That value is kept in the scalars, not taken from the partials: an
        // idle iteration (iterated residual already below tol) carries ||r||^2 forward into
        // both partial buffers, which would turn the ratio into 1 and revive a stale, much
        // longer search direction at full weight.
        const double old = sc[r].rr_last;
        const bool ok = isfinite(rr);
        if (threadIdx.x == 0) {
            sc[r].reliable += 1;
            sc[r].rec_rr = rec;
            sc[r].true_rr = rr;
            if (!ok) sc[r].nonfinite = 1;
            else sc[r].rr = rr;
            if (ok && rr <= sc[r].tol2) sc[r].done = 1;
        }
        if (!ok) return;
        // The iteration continues from the recomputed residual: alpha uses ||r_true||^2,
        // while the search direction keeps the recursion's beta = rec / old (the previous
        // entry is set so that the ratio the next kernel forms is that beta).  A zero or
        // non-finite iterated residual restarts the recursion: beta = 0.  Every thread has
        // read the partials (sum_partials_k ends in a barrier) before they change.
        const double pv = (rec > 0.0 && isfinite(rec)) ? old * (rr / rec) : __builtin_huge_val();
        for (int j = threadIdx.x; j < slots; j += blockDim.x) {
            cur[j] = j == 0 ? rr : 0.0;
            prev[j] = j == 0 ? pv : 0.0;
        }
    }
};

struct FinInit {                 // ||chi||^2 and the starting state of every right-hand side
    CgScalars* sc;
    double tol;
    double* rr0;                 // ||r||^2 partials of iteration 0, [nrhs][slots]
    double* rr_prev;             // and of "iteration -1" (only their ratio with rr0 is used, times p = 0)
    int slots;
    __device__ void finish(int r, double cc, double*) const {
        if (threadIdx.x != 0) return;
        CgScalars s{};
        s.chichi = cc;
        s.tol2 = tol * tol * cc;
        s.rr = cc;
        s.true_rr = cc;
        s.rec_rr = cc;
        s.rr_last = cc;
        s.nonfinite = isfinite(cc) ? 0 : 1;
        s.done = (cc == 0.0) ? 1 : 0;
        sc[r] = s;
        rr0[(long long)r * slots] = cc;
        rr_prev[(long long)r * slots] = cc;
        for (int j = 1; j < slots; ++j) {
            rr0[(long long)r * slots + j] = 0.0;
            rr_prev[(long long)r * slots + j] = 0.0;
        }
    }
};

struct FinStore {                // out[0] = sum over right-hand sides (in order)
    double* out;
    int nrhs;
    __device__ void finish(int r, double v, double*) const {
        if (threadIdx.x == 0) out[0] = (r == 0) ? v : out[0] + v;
    }
};

// ----------------------------------------------------------------------------- block control
// An operator kernel asks its control policy, before anything else, whether the block
// works and with which CG scalars (begin), and hands it the block's reduction value at
// the end (end).  begin() and end() are called by every thread of the block.
// A kernel that prefetches calls prefetch(rhs) before its own loads and hands the result to
// begin(); the others call begin(rhs, slot, lds).
struct CtlPlain {                // operators and force: always work, nothing reduced
    static constexpr bool kEnd = false;
    using Pre = NoCtlPre;
    __device__ Pre prefetch(int) const { return {}; }
    __device__ Scal begin(int, int, double*, const Pre&) const { return {1, 0.0, 0.0}; }
    __device__ Scal begin(int, int, double*) const { return {1, 0.0, 0.0}; }
    __device__ void end(double, int, int, const Scal&, double*) const {}
    CtlPlain with_slots(int) const { return *this; }
};

struct CtlGate {                 // gate from the CG scalars, nothing reduced
    static constexpr bool kEnd = false;
    const CgScalars* sc;
    int gate;
    using Pre = NoCtlPre;
    __device__ Pre prefetch(int) const { return {}; }
    __device__ Scal begin(int rhs, int, double*) const { return {gate_open(sc, gate, rhs) ? 1 : 0, 0.0, 0.0}; }
    __device__ Scal begin(int rhs, int slot, double* lds, const Pre&) const { return begin(rhs, slot, lds); }
    __device__ void end(double, int, int, const Scal&, double*) const {}
    CtlGate with_slots(int) const { return *this; }
};

template <class Fin>
struct CtlAtomic {               // gate from the CG scalars; last-block finalize of the reduction
    static constexpr bool kEnd = true;
    const CgScalars* sc;
    int gate;
    RedArgs ra;
    Fin fin;
    using Pre = NoCtlPre;
    __device__ Pre prefetch(int) const { return {}; }
    __device__ Scal begin(int rhs, int, double*) const { return {gate_open(sc, gate, rhs) ? 1 : 0, 0.0, 0.0}; }
    __device__ Scal begin(int rhs, int slot, double* lds, const Pre&) const { return begin(rhs, slot, lds); }
    __device__ void end(double acc, int rhs, int slot, const Scal&, double* lds) const {
        reduce_and_finalize(acc, rhs, slot, ra, fin, lds);
    }
    CtlAtomic with_slots(int n) const {
        CtlAtomic c = *this;
        c.ra.slots = n;
        return c;
    }
};

// CG iteration i, first kernel: t = M^dag (r + beta p).  beta = rr_i / rr_{i-1} from the
// previous kernels' partials (summed in slot order by every block, so every block
// agrees); the block works while ||r_i||^2 > tol^2 ||chi||^2 and the solve is not done.
// Writes this block's partial of ||t||^2.
struct CtlSearch {
    static constexpr bool kEnd = true;
    const double* rr_i;          // [nrhs][slots]
    const double* rr_im1;
    double* tt_out;
    CgScalars* sc;
    int slots;
    using Pre = PartialsPre<2>;
    __device__ Pre prefetch(int rhs) const {
        const long long o = (long long)rhs * slots;
        const double* const p[2] = {rr_i + o, rr_im1 + o};
        return prefetch_partials<2>(p, slots, sc[rhs]);
    }
    __device__ Scal begin(int rhs, int slot, double* lds) const { return begin(rhs, slot, lds, prefetch(rhs)); }
    __device__ Scal begin(int rhs, int slot, double* lds, const Pre& pre) const {
        const long long o = (long long)rhs * slots;
        const double* const p[2] = {rr_i + o, rr_im1 + o};
        double sum[2];
        sum_partials_pre<2>(p, slots, pre, lds, sum);
        const double a = sum[0], b = sum[1];
        int open = (!pre.done && !pre.nonfinite && a > pre.tol2) ? 1 : 0;
        const double beta = a / b;
        if (open && !isfinite(beta)) {
            open = 0;
            if (slot == 0 && threadIdx.x == 0) sc[rhs].nonfinite = 1;
        }
        return {open, 0.0, beta};
    }
    __device__ void end(double acc, int rhs, int slot, const Scal&, double* lds) const {
        const double v = block_sum(acc, lds);
        if (threadIdx.x == 0) tt_out[(long long)rhs * slots + slot] = v;
    }
    CtlSearch with_slots(int) const { return *this; }
};

// CG iteration i, second kernel: q = M t, p = r + beta p, x += alpha p, r -= alpha q,
// alpha = rr_i / ||t||^2.  Writes this block's partial of ||r_{i+1}||^2, or carries the
// block's rr_i partial forward when the block is idle (so an idle solve stays idle).  XM is the
// x-update form of the matching EpiUpdate: a skipping step records alpha and whether it worked,
// a paired step reads them (two kernels later, so no block reads what another writes).
template <int XM = kXPlain>
struct CtlUpdateT {
    static constexpr bool kEnd = true;
    const double* rr_i;
    const double* rr_im1;
    const double* tt;
    double* rr_next;
    CgScalars* sc;
    int slots;
    struct Pre : PartialsPre<3> {
        double alpha_prev;
        int x_pending;
    };
    __device__ Pre prefetch(int rhs) const {
        const long long o = (long long)rhs * slots;
        const double* const p[3] = {rr_i + o, rr_im1 + o, tt + o};
        Pre pre;
        static_cast<PartialsPre<3>&>(pre) = prefetch_partials<3>(p, slots, sc[rhs]);
        pre.alpha_prev = XM == kXPair ? sc[rhs].alpha_prev : 0.0;
        pre.x_pending = XM == kXPair ? sc[rhs].x_pending : 0;
        return pre;
    }
    __device__ Scal begin(int rhs, int slot, double* lds) const { return begin(rhs, slot, lds, prefetch(rhs)); }
    __device__ Scal begin(int rhs, int slot, double* lds, const Pre& pre) const {
        const long long o = (long long)rhs * slots;
        const double* const p[3] = {rr_i + o, rr_im1 + o, tt + o};
        double sum[3];
        sum_partials_pre<3>(p, slots, pre, lds, sum);
        const double a = sum[0], b = sum[1], c = sum[2];
        int open = (!pre.done && !pre.nonfinite && a > pre.tol2) ? 1 : 0;
        const double alpha = a / c, beta = a / b;
        if (open && (!(c > 0.0) || !isfinite(alpha) || !isfinite(beta))) {
            open = 0;
            if (slot == 0 && threadIdx.x == 0) sc[rhs].nonfinite = 1;
        }
        if (open && slot == 0 && threadIdx.x == 0) {
            sc[rhs].iters = pre.iters + 1;
            sc[rhs].rr_last = a;
        }
        if (XM == kXSkip && slot == 0 && threadIdx.x == 0) {
            sc[rhs].x_pending = open;
            if (open) sc[rhs].alpha_prev = alpha;
        }
        return {open, alpha, beta, pre.alpha_prev, pre.x_pending};
    }
    __device__ void end(double acc, int rhs, int slot, const Scal& s, double* lds) const {
        const double v = block_sum(acc, lds);
        const long long k = (long long)rhs * slots + slot;
        if (threadIdx.x == 0) rr_next[k] = s.open ? v : rr_i[k];
    }
    CtlUpdateT with_slots(int) const { return *this; }
};
using CtlUpdate = CtlUpdateT<kXPlain>;

// ----------------------------------------------------------------------------- fused kernel
// One workgroup per (right-hand side, destination slice): the source slice lives in
// LDS, both sublattices are transformed, mixed by E(k) and transformed back, and the
// epilogue streams the result out.  Block -> slice mapping keeps consecutive slices on
// one XCD (workgroups are dealt round-robin over the 8 XCDs), so the neighbouring
// slice that an epilogue and the next workgroup's source share hits the same L2.
__device__ __forceinline__ int xcd_linear(int b, int total) {
    const int x = b & 7, j = b >> 3;
    const int per = total >> 3, rem = total & 7;
    return x * per + (x < rem ? x : rem) + j;
}

template <typename R>
__device__ __forceinline__ void mix_E(cx<R>* A, cx<R>* B, int LL, const R* __restrict__ etab) {
    for (int p = threadIdx.x; p < LL; p += blockDim.x) {
        const R c = etab[4 * p], sr = etab[4 * p + 1], si = etab[4 * p + 2];
        const cx<R> a = A[p], b = B[p];
        // A' = c a + sf b ;  B' = conj(sf) a + c b
        A[p] = {c * a.re + sr * b.re - si * b.im, c * a.im + sr * b.im + si * b.re};
        B[p] = {c * b.re + sr * a.re + si * a.im, c * b.im + sr * a.im - si * a.re};
    }
}

template <typename R, class Src, class Epi, class Ctl>
__global__ void __launch_bounds__(kThreads)
k_fused(const OpTab<R> T, const Src src, const Epi epi, const Ctl ctl) {
    extern __shared__ __align__(16) unsigned char smem[];
    __shared__ double red_lds[64];
    cx<R>* buf = reinterpret_cast<cx<R>*>(smem);
    cx<R>* roots = buf + T.V;
    const int L = T.L, LL = L * L, V = T.V;
    const int u = xcd_linear(blockIdx.x, gridDim.x);
    const int rhs = u / T.Nt, t = u - rhs * T.Nt;
    const Scal sc = ctl.begin(rhs, t, red_lds);
    double acc = 0.0;
    if (sc.open) {
        for (int i = threadIdx.x; i < L; i += blockDim.x) roots[i] = T.roots[i];
        const int ts = src.slice(t, T.Nt);
        for (int i = threadIdx.x; i < V; i += blockDim.x) buf[i] = src_apply(src, rhs, ts, i, T, sc);
        __syncthreads();
        const LineMap rows{1, L, 0, 1};
        const LineMap cols{L, LL, 1, L};
        fft_lines<R, false>(buf, rows, 2 * L, T.plan, roots);
        fft_lines<R, false>(buf, cols, 2 * L, T.plan, roots);
        mix_E(buf, buf + LL, LL, T.etab);
        __syncthreads();
        fft_lines<R, true>(buf, cols, 2 * L, T.plan, roots);
        fft_lines<R, true>(buf, rows, 2 * L, T.plan, roots);
        for (int i = threadIdx.x; i < V; i += blockDim.x) epi_apply(epi, rhs, t, i, buf[i], T, sc, acc);
    }
    if constexpr (Ctl::kEnd) ctl.end(acc, rhs, t, sc, red_lds);
}

// Same layout with L known at compile time (NT threads per workgroup).  The first
// row stage is fused into the source load and the last inverse row stage into the
// epilogue, so the slice makes two fewer round trips through LDS.  Every global load
// is issued ahead of its use: the source entries before anything else, E(k) and (when they
// fit the register budget) the epilogue operands once the source has been consumed, else the
// epilogue operands one stage before the epilogue; the part of the epilogue that does not
// depend on the transform (early()) runs after the forward stages, so its stores overlap the
// rest of it.
//
// HALF = true runs two workgroups per slice when there are fewer slices than compute
// units: both transform the whole source slice forward (the 2 x 2 hopping exponential
// couples the sublattices), and each mixes, transforms back and writes one sublattice.
// Three quarters of the arithmetic per workgroup, no communication between them.
// Register budget per thread for the epilogue operands: held across the whole transform
// when small (issued with the source loads), else issued one stage before the epilogue.
template <int BYTES>
struct EpiPrefetch {
    static constexpr bool early = BYTES <= 192;
    static constexpr bool late = !early && BYTES <= 400;
};

template <typename R, int L, int NT, bool HALF, class Src, class Epi, class Ctl>
__global__ void __launch_bounds__(NT)
k_fused_ct(const OpTab<R> T, const Src src, const Epi epi, const Ctl ctl) {
    constexpr CPlan P = make_cplan(L);
    static_assert(P.nst >= 1, "L = 1 takes the generic kernel");
    constexpr int LL = L * L, V = 2 * LL;
    constexpr int R0 = P.radix[0], M0 = L / R0;
    constexpr int NT0 = 2 * L * M0;                     // stage-0 tasks over both sublattices
    constexpr int NTE = HALF ? L * M0 : NT0;            // stage-0 tasks of the sublattices written
    constexpr int ROUNDS0 = (NT0 + NT - 1) / NT;
    constexpr int ROUNDSO = (NTE + NT - 1) / NT;
    constexpr int ROUNDSE = (LL + NT - 1) / NT;         // momenta per thread in the mix
    constexpr int kEpiBytes = (int)sizeof(typename Epi::Pre) * ROUNDSO * R0;
    constexpr bool kPreEarly = EpiPrefetch<kEpiBytes>::early;
    constexpr bool kPreLate = EpiPrefetch<kEpiBytes>::late;
    constexpr bool kPreEpi = kPreEarly || kPreLate;
    extern __shared__ __align__(16) unsigned char smem[];
    __shared__ double red_lds[64];
    cx<R>* buf = reinterpret_cast<cx<R>*>(smem);
    cx<R>* roots = buf + V;
    const int u = xcd_linear(blockIdx.x, gridDim.x);
    const int q = HALF ? (u >> 1) : u;
    const int h = HALF ? (u & 1) : 0;                   // sublattice written (HALF only)
    const int rhs = q / T.Nt, t = q - rhs * T.Nt;
    const int off = HALF ? h * LL : 0;                  // first site written
    const int slot = HALF ? 2 * t + h : t;
    const int tid = threadIdx.x;
    static_assert(NT >= L, "one root of unity per thread");
    // Every global load is issued before the block learns its CG scalars (the loads do not
    // depend on them), so the scalar reduction overlaps the fetch.
    //
    // FP32 (kDefer): the loads are issued in the order their data is needed and
    // unconditionally (indices clamped into range, the surplus lanes' values unused): the
    // memory counter is waited on in issue order, so a load under a branch, or one needed
    // early but issued late, would make the wave wait for every load before it.  The CG
    // partials and the roots come first; E(k) and the early epilogue operands only once the
    // source has been consumed (issued with it they would share its bandwidth and delay the
    // first stage; from there they arrive during the forward transform).
    // FP64: source, E(k) and epilogue operands together at the start, the roots when the block
    // opens; its first stage is long (the FP64 phases), and the FP32 order measured slower.
    constexpr bool kDefer = sizeof(R) == sizeof(float);
    typename Ctl::Pre cpre{};
    cx<R> root_v{};
    const int rt = tid < L ? tid : L - 1;
    if constexpr (kDefer) {
        cpre = ctl.prefetch(rhs);
        root_v = T.roots[rt];
        __builtin_amdgcn_sched_barrier(0);    // keep the issue order: the scheduler may not mix the groups
    }
    const int ts = src.slice(t, T.Nt);
    typename Src::Pre pre[ROUNDS0][R0];
#pragma unroll
    for (int rd = 0; rd < ROUNDS0; ++rd) {
        const int task = tid + rd * NT;
        if (kDefer || task < NT0) {
            const int tc = kDefer ? min(task, NT0 - 1) : task;
            const int line = tc / M0, np = tc - line * M0;
#pragma unroll
            for (int i = 0; i < R0; ++i) pre[rd][i] = src.fetch(rhs, ts, line * L + np + i * M0, T);
        }
    }
    if constexpr (kDefer) __builtin_amdgcn_sched_barrier(0);
    typename Epi::Pre ep[kPreEpi ? ROUNDSO : 1][kPreEpi ? R0 : 1];
    R ec[ROUNDSE][3];
    auto fetch_e = [&]() {
#pragma unroll
        for (int rd = 0; rd < ROUNDSE; ++rd) {
            const int p = tid + rd * NT;
            if (kDefer || p < LL) {
                const int pc = kDefer ? min(p, LL - 1) : p;
                ec[rd][0] = T.etab[4 * pc];
                ec[rd][1] = T.etab[4 * pc + 1];
                ec[rd][2] = T.etab[4 * pc + 2];
            }
        }
    };
    auto fetch_ep = [&]() {
        if constexpr (kPreEarly) {
#pragma unroll
            for (int rd = 0; rd < ROUNDSO; ++rd) {
                const int task = tid + rd * NT;
                if (kDefer || task < NTE) {
                    const int tc = kDefer ? min(task, NTE - 1) : task;
                    const int line = tc / M0, np = tc - line * M0;
#pragma unroll
                    for (int i = 0; i < R0; ++i) ep[rd][i] = epi.fetch(rhs, t, off + line * L + np + i * M0, T);
                }
            }
        }
    };
    if constexpr (!kDefer) {
        fetch_e();
        fetch_ep();
    }
    const Scal sc = kDefer ? ctl.begin(rhs, slot, red_lds, cpre) : ctl.begin(rhs, slot, red_lds);
    double acc = 0.0;
    if (sc.open) {
        if constexpr (kDefer) {
            roots[rt] = root_v;
        } else {
            for (int i = tid; i < L; i += NT) roots[i] = T.roots[i];
        }
        __syncthreads();
        // row stage 0 (natural-order input) from the prefetched entries
#pragma unroll
        for (int rd = 0; rd < ROUNDS0; ++rd) {
            const int task = tid + rd * NT;
            if (task < NT0) {
                const int line = task / M0, np = task - line * M0;
                const int base = line * L + np;
                cx<R> x[R0];
#pragma unroll
                for (int i = 0; i < R0; ++i) x[i] = src.make(pre[rd][i], sc);
                small_dft_ct<R, R0, false>(x);
                if constexpr (M0 > 1) {
#pragma unroll
                    for (int k = 1; k < R0; ++k) x[k] = cmul(x[k], roots[np * k]);
                }
#pragma unroll
                for (int i = 0; i < R0; ++i) buf[base + i * M0] = x[i];
            }
        }
        if constexpr (kDefer) {
            fetch_e();          // E(k) first: the mix needs it before the epilogue does
            fetch_ep();
        }
        __syncthreads();
        // the early epilogue after the row stages, or in FP32 after the column stages too (its
        // operands were issued later there)
        auto do_early = [&]() {
            if constexpr (kPreEarly) {
#pragma unroll
                for (int rd = 0; rd < ROUNDSO; ++rd) {
                    const int task = tid + rd * NT;
                    if (task < NTE) {
                        const int line = task / M0, np = task - line * M0;
#pragma unroll
                        for (int i = 0; i < R0; ++i)
                            epi_early<R>(epi, rhs, t, off + line * L + np + i * M0, ep[rd][i], T, sc);
                    }
                }
            }
        };
        ct_forward<R, L, 1, P.nst, false, NT>(buf, roots);
        if constexpr (!kDefer) do_early();
        ct_forward<R, L, 0, P.nst, true, NT>(buf, roots);
        if constexpr (kDefer) do_early();
        // E(k): A' = c A + sf B,  B' = conj(sf) A + c B
#pragma unroll
        for (int rd = 0; rd < ROUNDSE; ++rd) {
            const int p = tid + rd * NT;
            if (p < LL) {
                const R c = ec[rd][0], sr = ec[rd][1], si = ec[rd][2];
                const cx<R> a = buf[p], b = buf[LL + p];
                const cx<R> na = {c * a.re + sr * b.re - si * b.im, c * a.im + sr * b.im + si * b.re};
                const cx<R> nb = {c * b.re + sr * a.re + si * a.im, c * b.im + sr * a.im - si * a.re};
                if (!HALF || h == 0) buf[p] = na;
                if (!HALF || h == 1) buf[LL + p] = nb;
            }
        }
        __syncthreads();
        constexpr int NS = HALF ? 1 : 2;
        cx<R>* own = buf + off;
        ct_inverse<R, L, P.nst - 1, 0, true, NT, NS>(own, roots);
        if constexpr (kPreLate) {
#pragma unroll
            for (int rd = 0; rd < ROUNDSO; ++rd) {
                const int task = tid + rd * NT;
                if (task < NTE) {
                    const int line = task / M0, np = task - line * M0;
#pragma unroll
                    for (int i = 0; i < R0; ++i) ep[rd][i] = epi.fetch(rhs, t, off + line * L + np + i * M0, T);
                }
            }
        }
        ct_inverse<R, L, P.nst - 1, 1, false, NT, NS>(own, roots);
        // row stage 0 inverse (natural-order output) straight into the epilogue
#pragma unroll
        for (int rd = 0; rd < ROUNDSO; ++rd) {
            const int task = tid + rd * NT;
            if (task < NTE) {
                const int line = task / M0, np = task - line * M0;
                const int base = line * L + np;
                cx<R> x[R0];
#pragma unroll
                for (int k = 0; k < R0; ++k) x[k] = own[base + k * M0];
                if constexpr (M0 > 1) {
#pragma unroll
                    for (int k = 1; k < R0; ++k) x[k] = cmulc(x[k], roots[np * k]);
                }
                small_dft_ct<R, R0, true>(x);
#pragma unroll
                for (int i = 0; i < R0; ++i) {
                    if constexpr (kPreEarly) {
                        epi.store(rhs, t, off + base + i * M0, x[i], ep[rd][i], T, sc, acc);
                    } else if constexpr (kPreLate) {
                        epi_early<R>(epi, rhs, t, off + base + i * M0, ep[rd][i], T, sc);
                        epi.store(rhs, t, off + base + i * M0, x[i], ep[rd][i], T, sc, acc);
                    } else {
                        epi_apply(epi, rhs, t, off + base + i * M0, x[i], T, sc, acc);
                    }
                }
            }
        }
    } else if (sc.pending) {
        // an idle block of a paired x update whose previous step skipped x: add the pending term
        // at the sites this block writes
        if constexpr (EpiHasClosed<Epi>::value) {
#pragma unroll
            for (int rd = 0; rd < ROUNDSO; ++rd) {
                const int task = tid + rd * NT;
                if (task < NTE) {
                    const int line = task / M0, np = task - line * M0;
#pragma unroll
                    for (int i = 0; i < R0; ++i) {
                        const int k = off + line * L + np + i * M0;
                        epi.closed(rhs, t, k, epi.fetch(rhs, t, k, T), T, sc);
                    }
                }
            }
        }
    }
    if constexpr (Ctl::kEnd) ctl.end(acc, rhs, slot, sc, red_lds);
}

// ----------------------------------------------------------------------------- polynomial kernel
// E = e^{delta mu} exp(delta kappa K) applied as e^{delta mu} p(delta kappa K) with p a polynomial of
// degree DEG close to e^z on the spectrum [-x, x] of delta kappa K (x = 3 |delta kappa|; the
// host's exp_poly_ratios gives p and its error bound, and uses this kernel only where that bound
// is far below the precision's rounding).  p is evaluated in nested form,
//     y <- v + c_j K y,  j = DEG..1,   result scale * y,   c_j = delta kappa a_j / a_{j-1},
// so DEG nearest-neighbour stencil sweeps over the slice replace four L x L transforms.
//
// NSPLIT workgroups per slice split the columns n2: workgroup h writes columns
// [h L / NSPLIT, (h + 1) L / NSPLIT) and carries H = ceil(DEG/2) halo columns on each side,
// since each pair of sweeps widens a site's dependence by one column each way (A(n) reaches
// B(n - e2), B(m) reaches A(m + e2)).  RSPLIT > 1 splits the rows n1 the same way: a workgroup
// holds its group's rows and H halo rows above and below, with no wrap inside the workgroup
// (the rows beyond the halos read as 0; after DEG sweeps the values they spoil reach at most
// H - 1 rows inward, all halo rows, which are never written).  RSPLIT = 1 holds all L rows,
// periodic.  Fewer rows per lane hold fewer registers (FP64), at the cost of the halo rows.
// Lanes run along n2 (32 lanes per strip when the columns and halos fit, so a strip is half a
// wave, else 64; a site's n2 neighbours are the adjacent lanes, fetched with wave-wide DPP
// shifts, and the lanes at a strip's two edges receive another strip's values or 0, which only
// ever feed halo columns).  In FP64 (degree 9) each double crosses lanes as two 32-bit shifts
// that do not fold into the adds; there the kernel is used at L = 102 only, where the transforms
// need the three-kernel split path (at L = 51 the in-LDS transforms measured faster).  Rows n1
// (periodic, all L of them) are split into NT/32 strips of at most RMAX rows held in registers;
// the row above and below a strip cross strips through LDS once per sweep.
template <int L, int NT, int DEG, int NSPLIT, int RSPLIT>
struct PolyGeom {
    static constexpr int H = (DEG + 1) / 2;
    static constexpr int W = (L + NSPLIT - 1) / NSPLIT + 2 * H;   // widest column range with its halos
    static constexpr int LPS = W <= 32 ? 32 : 64;        // lanes (columns) per strip
    static constexpr int NSTRIP = NT / LPS;
    // rows held: all L, or the widest row group with its halos (the narrowest has one row fewer)
    static constexpr int VR = RSPLIT == 1 ? L : (L + RSPLIT - 1) / RSPLIT + 2 * H;
    static constexpr int RMAX = (VR + NSTRIP - 1) / NSTRIP;
    static_assert(W <= LPS, "column range and halos must fit one strip");
    static_assert(NT % 64 == 0, "whole waves");
    static_assert(RSPLIT == 1 || VR <= L, "a row group's halos must not wrap onto its own rows");
    static_assert(VR - 1 >= NSTRIP, "every strip holds a row");
};

// Wave-wide lane shifts (DPP): lane i receives lane i - 1 (prev) or i + 1 (next); the lane
// that has no such neighbour receives 0.  The compiler folds them into the adds that use them.
constexpr int kDppWaveShr1 = 0x138;
constexpr int kDppWaveShl1 = 0x130;
template <int CTRL>
__device__ __forceinline__ float lane_shift(float v) {
    return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), CTRL, 0xf, 0xf, false));
}
__device__ __forceinline__ cx<float> lane_prev(cx<float> v) {
    return {lane_shift<kDppWaveShr1>(v.re), lane_shift<kDppWaveShr1>(v.im)};
}
__device__ __forceinline__ cx<float> lane_next(cx<float> v) {
    return {lane_shift<kDppWaveShl1>(v.re), lane_shift<kDppWaveShl1>(v.im)};
}
// a double moves as its two 32-bit halves
template <int CTRL>
__device__ __forceinline__ double lane_shift(double v) {
    const unsigned long long b = (unsigned long long)__double_as_longlong(v);
    const unsigned lo = __builtin_amdgcn_update_dpp(0, (int)(unsigned)b, CTRL, 0xf, 0xf, false);
    const unsigned hi = __builtin_amdgcn_update_dpp(0, (int)(unsigned)(b >> 32), CTRL, 0xf, 0xf, false);
    return __longlong_as_double((long long)(((unsigned long long)hi << 32) | lo));
}
__device__ __forceinline__ cx<double> lane_prev(cx<double> v) {
    return {lane_shift<kDppWaveShr1>(v.re), lane_shift<kDppWaveShr1>(v.im)};
}
__device__ __forceinline__ cx<double> lane_next(cx<double> v) {
    return {lane_shift<kDppWaveShl1>(v.re), lane_shift<kDppWaveShl1>(v.im)};
}

// The polynomial's constants: c[j] = delta kappa a_j / a_{j-1} for sweep j = 1..10, and the final
// scale e^{delta mu} a_0.
template <typename R>
struct PolyCoef {
    R scale;
    R c[11];
};

template <typename R, int L, int NT, int DEG, int NSPLIT, int RSPLIT, class Src, class Epi, class Ctl>
__global__ void __launch_bounds__(NT)
k_exp_poly(const OpTab<R> T, const PolyCoef<R> pc, const Src src, const Epi epi, const Ctl ctl) {
    static_assert(DEG >= 1 && DEG <= 10, "c[] holds ten sweeps");
    using G = PolyGeom<L, NT, DEG, NSPLIT, RSPLIT>;
    constexpr int LL = L * L, RM = G::RMAX, NS = G::NSTRIP, PARTS = NSPLIT * RSPLIT;
    __shared__ cx<R> edgeA[2][NS][G::LPS];               // first row's A of each strip, per sweep parity
    __shared__ cx<R> edgeB[2][NS][G::LPS];               // last row's B
    __shared__ double red_lds[64];
    const int u = xcd_linear(blockIdx.x, gridDim.x);
    const int q = u / PARTS, part = u - q * PARTS;
    const int h = part % NSPLIT, g = part / NSPLIT;      // column range, row group
    const int rhs = q / T.Nt, t = q - rhs * T.Nt;
    const int slot = PARTS * t + part;
    const int tid = threadIdx.x;
    const int s = tid / G::LPS, j = tid - s * G::LPS;
    // rows held: rows v in [0, nv) are global rows vbase + v (mod L); those written are [vo0, vo0 + NR)
    const int R0 = g * L / RSPLIT, NR = (g + 1) * L / RSPLIT - R0;
    const int nv = RSPLIT == 1 ? L : NR + 2 * G::H;
    const int vbase = RSPLIT == 1 ? 0 : R0 - G::H + L;
    const int vo0 = RSPLIT == 1 ? 0 : G::H;
    const int r0 = s * nv / NS, nr = (s + 1) * nv / NS - r0;
    auto grow = [&](int v) { return RSPLIT == 1 ? v : (vbase + v) % L; };
    auto out_row = [&](int r) { return r < nr && r0 + r >= vo0 && r0 + r < vo0 + NR; };
    const int c0 = h * L / NSPLIT, ncol = (h + 1) * L / NSPLIT - c0;
    const int n2 = (c0 - G::H + j + L) % L;
    const bool out_lane = j >= G::H && j < G::H + ncol;
    // every global load before the block's CG scalars (as in k_fused_ct): partials, source
    // entries, then the epilogue operands of this lane's output sites
    typename Ctl::Pre cpre = ctl.prefetch(rhs);
    const int ts = src.slice(t, T.Nt);
    typename Src::Pre pa[RM], pb[RM];
#pragma unroll
    for (int r = 0; r < RM; ++r) {
        const int n1 = grow(r0 + min(r, nr - 1));          // rows past the strip repeat its last row
        pa[r] = src.fetch(rhs, ts, n1 * L + n2, T);
        pb[r] = src.fetch(rhs, ts, LL + n1 * L + n2, T);
    }
    // epilogue operands with the source when they fit a register budget of 64 (held across
    // the sweeps), else fetched after the sweeps
    constexpr bool kEpiEarly = sizeof(typename Epi::Pre) * 2 * RM <= 256;
    typename Epi::Pre ea[RM], eb[RM];
    // only the lanes and rows that write load them (a halo lane or a strip's missing last row
    // never uses its operands; the masked loads move no data)
    auto fetch_epi = [&]() {
#pragma unroll
        for (int r = 0; r < RM; ++r) {
            if (out_lane && out_row(r)) {
                ea[r] = epi.fetch(rhs, t, grow(r0 + r) * L + n2, T);
                eb[r] = epi.fetch(rhs, t, LL + grow(r0 + r) * L + n2, T);
            }
        }
    };
    if constexpr (kEpiEarly) fetch_epi();
    const Scal sc = ctl.begin(rhs, slot, red_lds, cpre);
    auto early_epi = [&]() {
        if (out_lane) {
#pragma unroll
            for (int r = 0; r < RM; ++r)
                if (out_row(r)) {
                    epi_early<R>(epi, rhs, t, grow(r0 + r) * L + n2, ea[r], T, sc);
                    epi_early<R>(epi, rhs, t, LL + grow(r0 + r) * L + n2, eb[r], T, sc);
                }
        }
    };
    double acc = 0.0;
    if (sc.open) {
        cx<R> va[RM], vb[RM], ya[RM], yb[RM];
#pragma unroll
        for (int r = 0; r < RM; ++r) {
            va[r] = src.make(pa[r], sc);
            vb[r] = src.make(pb[r], sc);
            ya[r] = va[r];
            yb[r] = vb[r];
        }
        if constexpr (kEpiEarly) early_epi();
        const int sp = (s + NS - 1) % NS, sn = (s + 1) % NS;
#pragma unroll
        for (int k = DEG; k >= 1; --k) {
            const int par = k & 1;
            cx<R> lastb = yb[0];
#pragma unroll
            for (int r = 1; r < RM; ++r)
                if (r < nr) lastb = yb[r];
            edgeA[par][s][j] = ya[0];
            edgeB[par][s][j] = lastb;
            __syncthreads();
            // B of row r0 - 1 (the previous strip's last), A of row r0 + nr (the next strip's
            // first); with row groups the first strip has nothing above, the last nothing below
            const cx<R> above = (RSPLIT > 1 && s == 0) ? cx<R>{0, 0} : edgeB[par][sp][j];
            const cx<R> below = (RSPLIT > 1 && s == NS - 1) ? cx<R>{0, 0} : edgeA[par][sn][j];
            const R ck = pc.c[k];
            // rows top to bottom, in place: row r's new A needs the old B of rows r and r - 1
            // (the latter carried in bup), its new B the old A of rows r and r + 1 (not yet
            // updated when row r is)
            cx<R> bup = above;
#pragma unroll
            for (int r = 0; r < RM; ++r) {
                const cx<R> adn = (r + 1 < RM && r + 1 < nr) ? ya[r + 1 < RM ? r + 1 : 0] : below;
                const cx<R> sa = yb[r] + bup + lane_prev(yb[r]);   // B(n), B(n - e1), B(n - e2)
                const cx<R> sb = ya[r] + adn + lane_next(ya[r]);   // A(m), A(m + e1), A(m + e2)
                bup = yb[r];
                ya[r] = {fmar(ck, sa.re, va[r].re), fmar(ck, sa.im, va[r].im)};
                yb[r] = {fmar(ck, sb.re, vb[r].re), fmar(ck, sb.im, vb[r].im)};
            }
        }
        if constexpr (!kEpiEarly) {
            fetch_epi();
            early_epi();
        }
        if (out_lane) {
#pragma unroll
            for (int r = 0; r < RM; ++r)
                if (out_row(r)) {
                    epi.store(rhs, t, grow(r0 + r) * L + n2, scale(pc.scale, ya[r]), ea[r], T, sc, acc);
                    epi.store(rhs, t, LL + grow(r0 + r) * L + n2, scale(pc.scale, yb[r]), eb[r], T, sc, acc);
                }
        }
    } else if (sc.pending) {
        // an idle block of a paired x update whose previous step skipped x: add the pending term
        if constexpr (EpiHasClosed<Epi>::value) {
            if constexpr (!kEpiEarly) fetch_epi();
            if (out_lane) {
#pragma unroll
                for (int r = 0; r < RM; ++r)
                    if (out_row(r)) {
                        epi.closed(rhs, t, grow(r0 + r) * L + n2, ea[r], T, sc);
                        epi.closed(rhs, t, LL + grow(r0 + r) * L + n2, eb[r], T, sc);
                    }
            }
        }
    }
    if constexpr (Ctl::kEnd) ctl.end(acc, rhs, slot, sc, red_lds);
}

// One workgroup per (right-hand side, slice) for slices larger than LDS whose single
// sublattice fits (FP32 at L = 102: 84 KB of the slice's 167 KB).  Sublattice A is
// transformed forward in LDS and its spectrum parked in registers (each thread keeps
// the momenta it will mix); then B is transformed in the same LDS, the 2 x 2 E(k) mix
// pairs each register-held A entry with the LDS-held B entry, B is transformed back
// and written, then the mixed A spectrum returns to LDS and is transformed back and
// written.  Two forward and two inverse sublattice transforms per slice, none repeated.
// The loads of B's source are issued before A's column stages, so they arrive while those run.
template <typename R, int L, int NT, class Src, class Epi, class Ctl>
__device__ __forceinline__ void fused_sub_item(const OpTab<R>& T, const Src& src, const Epi& epi, const Ctl& ctl,
                                               int u, cx<R>* buf, double* red_lds) {
    constexpr CPlan P = make_cplan(L);
    static_assert(P.nst >= 2, "needs a row stage besides the fused one");
    constexpr int LL = L * L;
    constexpr int R0 = P.radix[0], M0 = L / R0;
    constexpr int NTS = L * M0;                         // stage-0 tasks of one sublattice
    constexpr int ROUNDS = (NTS + NT - 1) / NT;
    constexpr int NP = (LL + NT - 1) / NT;              // momenta per thread in the mix
    cx<R>* roots = buf + LL;
    const int rhs = u / T.Nt, t = u - rhs * T.Nt;
    const int tid = threadIdx.x;
    static_assert(NT >= L, "one root of unity per thread");
    // loads in the order their data is needed, unconditionally (indices clamped into range):
    // the memory counter is waited on in issue order (see k_fused_ct)
    const typename Ctl::Pre cpre = ctl.prefetch(rhs);
    const int rt = tid < L ? tid : L - 1;
    const cx<R> root_v = T.roots[rt];
    __builtin_amdgcn_sched_barrier(0);    // keep the issue order (see k_fused_ct)
    const int ts = src.slice(t, T.Nt);
    typename Src::Pre pre[ROUNDS][R0];
    auto fetch_sub = [&](int s) {
#pragma unroll
        for (int rd = 0; rd < ROUNDS; ++rd) {
            const int task = min(tid + rd * NT, NTS - 1);
            const int line = task / M0, np = task - line * M0;
#pragma unroll
            for (int i = 0; i < R0; ++i) pre[rd][i] = src.fetch(rhs, ts, s * LL + line * L + np + i * M0, T);
        }
    };
    fetch_sub(0);
    __builtin_amdgcn_sched_barrier(0);
    const Scal sc = ctl.begin(rhs, t, red_lds, cpre);
    double acc = 0.0;
    if (sc.open) {
        roots[rt] = root_v;
        cx<R> ahat[NP];
#pragma unroll
        for (int s = 0; s < 2; ++s) {
            __syncthreads();
            // row stage 0 of sublattice s (natural-order input) from the fetched entries
#pragma unroll
            for (int rd = 0; rd < ROUNDS; ++rd) {
                const int task = tid + rd * NT;
                if (task < NTS) {
                    const int line = task / M0, np = task - line * M0;
                    const int base = line * L + np;
                    cx<R> x[R0];
#pragma unroll
                    for (int i = 0; i < R0; ++i) x[i] = src.make(pre[rd][i], sc);
                    small_dft_ct<R, R0, false>(x);
                    if constexpr (M0 > 1) {
#pragma unroll
                        for (int k = 1; k < R0; ++k) x[k] = cmul(x[k], roots[np * k]);
                    }
#pragma unroll
                    for (int i = 0; i < R0; ++i) buf[base + i * M0] = x[i];
                }
            }
            __syncthreads();
            ct_forward<R, L, 1, P.nst, false, NT, 1>(buf, roots);
            if (s == 0) fetch_sub(1);     // B's source arrives during A's column stages
            ct_forward<R, L, 0, P.nst, true, NT, 1>(buf, roots);
            if (s == 0) {
#pragma unroll
                for (int j = 0; j < NP; ++j) {
                    const int p = tid + j * NT;
                    if (p < LL) ahat[j] = buf[p];
                }
            }
        }
        // E(k): A' = c A + sf B (kept in registers),  B' = conj(sf) A + c B (in LDS)
#pragma unroll
        for (int j = 0; j < NP; ++j) {
            const int p = tid + j * NT;
            if (p < LL) {
                const R c = T.etab[4 * p], sr = T.etab[4 * p + 1], si = T.etab[4 * p + 2];
                const cx<R> a = ahat[j], b = buf[p];
                ahat[j] = {c * a.re + sr * b.re - si * b.im, c * a.im + sr * b.im + si * b.re};
                buf[p] = {c * b.re + sr * a.re + si * a.im, c * b.im + sr * a.im - si * a.re};
            }
        }
#pragma unroll
        for (int s = 1; s >= 0; --s) {
            if (s == 0) {
                __syncthreads();
#pragma unroll
                for (int j = 0; j < NP; ++j) {
                    const int p = tid + j * NT;
                    if (p < LL) buf[p] = ahat[j];
                }
            }
            __syncthreads();
            ct_inverse<R, L, P.nst - 1, 0, true, NT, 1>(buf, roots);
            ct_inverse<R, L, P.nst - 1, 1, false, NT, 1>(buf, roots);
            // row stage 0 inverse (natural-order output) straight into the epilogue; a few
            // rounds at a time (the ahat registers are still live)
#pragma unroll 2
            for (int rd = 0; rd < ROUNDS; ++rd) {
                const int task = tid + rd * NT;
                if (task < NTS) {
                    const int line = task / M0, np = task - line * M0;
                    const int base = line * L + np;
                    cx<R> x[R0];
#pragma unroll
                    for (int k = 0; k < R0; ++k) x[k] = buf[base + k * M0];
                    if constexpr (M0 > 1) {
#pragma unroll
                        for (int k = 1; k < R0; ++k) x[k] = cmulc(x[k], roots[np * k]);
                    }
                    small_dft_ct<R, R0, true>(x);
#pragma unroll
                    for (int i = 0; i < R0; ++i) epi_apply(epi, rhs, t, s * LL + base + i * M0, x[i], T, sc, acc);
                }
            }
        }
    }
    if constexpr (Ctl::kEnd) ctl.end(acc, rhs, t, sc, red_lds);
}

// The sublattice kernel proper: one workgroup per (right-hand side, slice).
template <typename R, int L, int NT, class Src, class Epi, class Ctl>
__global__ void __launch_bounds__(NT)
k_fused_sub(const OpTab<R> T, const Src src, const Epi epi, const Ctl ctl) {
    extern __shared__ __align__(16) unsigned char smem[];
    __shared__ double red_lds[64];
    fused_sub_item<R, L, NT>(T, src, epi, ctl, xcd_linear(blockIdx.x, gridDim.x), reinterpret_cast<cx<R>*>(smem),
                             red_lds);
}

// ----------------------------------------------------------------------------- persistent CG
// Grid-wide barrier of a cooperative launch (every workgroup co-resident).  bar[0] counts the
// arrivals, bar[1] is the generation, bar[2] the abort flag.  Every wave waits for its own
// stores, then thread 0 of each workgroup makes the workgroup's global writes visible
// device-wide (agent-scope release), arrives, and the last
// arrival opens the next generation; the others poll it.  Every wait is bounded: after `spin`
// polls a waiting workgroup sets the abort flag, and a workgroup that sees the flag stops
// waiting, so every workgroup leaves the barrier.  Returns false (in every thread) once the
// flag is set: the caller returns, the host turns the flag into an error.
__device__ __forceinline__ bool grid_barrier(unsigned* bar, long long spin) {
    __shared__ int ok;
    __builtin_amdgcn_s_waitcnt(0);       // this wave's stores have reached the L2 ...
    __syncthreads();                     // ... in every wave, before thread 0's release
    if (threadIdx.x == 0) {
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
        const unsigned g = __hip_atomic_load(&bar[1], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        const unsigned n = gridDim.x * gridDim.y * gridDim.z;
        const unsigned arrived = __hip_atomic_fetch_add(&bar[0], 1u, __ATOMIC_ACQ_REL, __HIP_MEMORY_SCOPE_AGENT);
        if (arrived == n - 1) {
            __hip_atomic_store(&bar[0], 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            __hip_atomic_store(&bar[1], g + 1u, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
        } else {
            long long polls = 0;
            while (__hip_atomic_load(&bar[1], __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_AGENT) == g) {
                if (__hip_atomic_load(&bar[2], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != 0u) break;
                if (++polls > spin) {
                    __hip_atomic_store(&bar[2], 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                    break;
                }
                __builtin_amdgcn_s_sleep(2);
            }
        }
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
        ok = __hip_atomic_load(&bar[2], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) == 0u;
    }
    __syncthreads();
    return ok != 0;
}

// Everything a persistent CG launch needs besides the operator tables.
template <typename R>
struct PersistArgs {
    double* pr;                  // ||r||^2 partials, three rotating buffers of nrhs * slots
    double* pt;                  // ||M^dag p||^2 partials
    CgScalars* sc;
    int slots, nrhs;
    long long it0;               // first iteration of this launch (selects the rotating buffers)
    int n_iter;
    cx<R>* r;
    cx<R>* p;
    cx<R>* tv;
    cx<R>* x;
    PhTable<R> tab;
    unsigned* bar;
    long long spin;
};

// The two phases of a CG iteration on one item, kept out of line: inlined into the persistent
// loop, the compiler would keep values of both phases live across it and spill.
template <typename R, int L, int NT>
__device__ __noinline__ void persist_search_item(const OpTab<R>& T, const PersistArgs<R>& a, const CtlSearch& k1,
                                                 int u, cx<R>* buf, double* red_lds) {
    fused_sub_item<R, L, NT>(T, SrcSearchNext<R>{a.r, a.p}, EpiSearchMdag<R, PhTable<R>>{a.r, a.p, a.tv, a.tab}, k1,
                             u, buf, red_lds);
}

template <typename R, int L, int NT>
__device__ __noinline__ void persist_update_item(const OpTab<R>& T, const PersistArgs<R>& a, const CtlUpdate& k2,
                                                 int u, cx<R>* buf, double* red_lds) {
    fused_sub_item<R, L, NT>(T, SrcPhasePrev<R, PhTable<R>>{a.tv, a.tab}, EpiUpdate<R>{a.tv, a.p, a.x, a.r}, k2, u,
                             buf, red_lds);
}

// n_iter CG iterations (each: t = M^dag (r + beta p), then p, x, r updated with q = M t) in one
// cooperative launch of the sublattice kernel's work: every workgroup loops over the
// (right-hand side, slice) items of a phase, and a grid barrier separates the phases.  Item k
// maps to the same slice and the same XCD as workgroup k of the two-kernel iteration, and does
// the same arithmetic, so a persistent solve equals the two-kernel one bit for bit.
template <typename R, int L, int NT>
__global__ void __launch_bounds__(NT) k_cg_persist_sub(const OpTab<R> T, const PersistArgs<R> a) {
    extern __shared__ __align__(16) unsigned char smem[];
    __shared__ double red_lds[64];
    cx<R>* buf = reinterpret_cast<cx<R>*>(smem);
    const int items = a.nrhs * T.Nt;
    const long long ns = (long long)a.nrhs * a.slots;
    for (int n = 0; n < a.n_iter; ++n) {
        const long long i = a.it0 + n;
        double* pri = a.pr + (i % 3) * ns;
        double* prm = a.pr + ((i + 2) % 3) * ns;
        double* prn = a.pr + ((i + 1) % 3) * ns;
        const CtlSearch k1{pri, prm, a.pt, a.sc, a.slots};
        for (int k = blockIdx.x; k < items; k += gridDim.x)
            persist_search_item<R, L, NT>(T, a, k1, xcd_linear(k, items), buf, red_lds);
        if (!grid_barrier(a.bar, a.spin)) return;
        const CtlUpdate k2{pri, prm, a.pt, prn, a.sc, a.slots};
        for (int k = blockIdx.x; k < items; k += gridDim.x)
            persist_update_item<R, L, NT>(T, a, k2, xcd_linear(k, items), buf, red_lds);
        if (n + 1 < a.n_iter && !grid_barrier(a.bar, a.spin)) return;
    }
}

// zero n words (the barrier state before a persistent launch; a kernel, not a memset node)
__global__ void k_zero_u32(unsigned* p, int n) {
    if ((int)threadIdx.x < n) p[threadIdx.x] = 0u;
}

// e^{i phi} as a table, evaluated in FP64 and rounded once to R
template <typename R>
__global__ void __launch_bounds__(kThreads)
k_phase_table(const double* __restrict__ phi, cx<R>* __restrict__ tab, long long n) {
    for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < n;
         i += (long long)gridDim.x * blockDim.x) {
        double s, c;
        phase_sincos(phi[i], &s, &c);
        tab[i] = {(R)c, (R)s};
    }
}

// ----------------------------------------------------------------------------- split kernels
// Slices too large for LDS: (1) row transforms of the source slice into a scratch
// vector W, (2) column transforms + E(k) + inverse column transforms of W in place,
// (3) inverse row transforms of W and the epilogue.  W is indexed by destination slice.
struct SplitGeom {
    int rb, nrb;      // rows per block, row blocks per sublattice
    int cb, ncb;      // columns per block, column blocks
};

template <typename R, class Src, class Ctl>
__global__ void __launch_bounds__(kThreads)
k_split_rows_fwd(const OpTab<R> T, const SplitGeom G, const Src src, cx<R>* __restrict__ W, const Ctl ctl) {
    extern __shared__ __align__(16) unsigned char smem[];
    __shared__ double red_lds[64];
    cx<R>* buf = reinterpret_cast<cx<R>*>(smem);
    const int L = T.L;
    cx<R>* roots = buf + G.rb * L;
    int b = blockIdx.x;
    const int rblk = b % G.nrb; b /= G.nrb;
    const int s = b % 2; b /= 2;
    const int t = b % T.Nt;
    const int rhs = b / T.Nt;
    const Scal sc = ctl.begin(rhs, -1, red_lds);
    if (!sc.open) return;
    const int r0 = rblk * G.rb;
    const int nr = min(G.rb, L - r0);
    for (int i = threadIdx.x; i < L; i += blockDim.x) roots[i] = T.roots[i];
    const int ts = src.slice(t, T.Nt);
    const int off = s * L * L + r0 * L;
    for (int i = threadIdx.x; i < nr * L; i += blockDim.x) buf[i] = src_apply(src, rhs, ts, off + i, T, sc);
    __syncthreads();
    fft_lines<R, false>(buf, LineMap{1, L, 0, 1}, nr, T.plan, roots);
    cx<R>* dst = W + rhs * T.N + (long long)t * T.V + off;
    for (int i = threadIdx.x; i < nr * L; i += blockDim.x) dst[i] = buf[i];
}

template <typename R, class Ctl>
__global__ void __launch_bounds__(kThreads)
k_split_cols(const OpTab<R> T, const SplitGeom G, cx<R>* __restrict__ W, const Ctl ctl) {
    extern __shared__ __align__(16) unsigned char smem[];
    __shared__ double red_lds[64];
    cx<R>* buf = reinterpret_cast<cx<R>*>(smem);
    const int L = T.L;
    cx<R>* roots = buf + 2 * L * G.cb;
    int b = blockIdx.x;
    const int cblk = b % G.ncb; b /= G.ncb;
    const int t = b % T.Nt;
    const int rhs = b / T.Nt;
    const Scal sc = ctl.begin(rhs, -1, red_lds);
    if (!sc.open) return;
    const int c0 = cblk * G.cb;
    const int nc = min(G.cb, L - c0);
    for (int i = threadIdx.x; i < L; i += blockDim.x) roots[i] = T.roots[i];
    cx<R>* base = W + rhs * T.N + (long long)t * T.V;
    // LDS tile [s][n1][c], c fastest
    for (int i = threadIdx.x; i < 2 * L * nc; i += blockDim.x) {
        const int c = i % nc, sn = i / nc;           // sn = s*L + n1
        buf[i] = base[(long long)sn * L + c0 + c];
    }
    __syncthreads();
    const LineMap cols{nc, L * nc, 1, nc};
    fft_lines<R, false>(buf, cols, 2 * nc, T.plan, roots);
    for (int i = threadIdx.x; i < L * nc; i += blockDim.x) {
        const int c = i % nc, n1 = i / nc;
        const int p = n1 * L + c0 + c;
        const R cc = T.etab[4 * p], sr = T.etab[4 * p + 1], si = T.etab[4 * p + 2];
        const cx<R> a = buf[i], bb = buf[L * nc + i];
        buf[i] = {cc * a.re + sr * bb.re - si * bb.im, cc * a.im + sr * bb.im + si * bb.re};
        buf[L * nc + i] = {cc * bb.re + sr * a.re + si * a.im, cc * bb.im + sr * a.im - si * a.re};
    }
    __syncthreads();
    fft_lines<R, true>(buf, cols, 2 * nc, T.plan, roots);
    for (int i = threadIdx.x; i < 2 * L * nc; i += blockDim.x) {
        const int c = i % nc, sn = i / nc;
        base[(long long)sn * L + c0 + c] = buf[i];
    }
}

template <typename R, class Epi, class Ctl>
__global__ void __launch_bounds__(kThreads)
k_split_rows_inv(const OpTab<R> T, const SplitGeom G, const cx<R>* __restrict__ W, const Epi epi,
                 const Ctl ctl) {
    extern __shared__ __align__(16) unsigned char smem[];
    __shared__ double red_lds[64];
    cx<R>* buf = reinterpret_cast<cx<R>*>(smem);
    const int L = T.L;
    cx<R>* roots = buf + G.rb * L;
    int b = blockIdx.x;
    const int slot = b % (2 * G.nrb * T.Nt);
    const int rblk = b % G.nrb; b /= G.nrb;
    const int s = b % 2; b /= 2;
    const int t = b % T.Nt;
    const int rhs = b / T.Nt;
    const Scal sc = ctl.begin(rhs, slot, red_lds);
    double acc = 0.0;
    if (sc.open) {
        const int r0 = rblk * G.rb;
        const int nr = min(G.rb, L - r0);
        for (int i = threadIdx.x; i < L; i += blockDim.x) roots[i] = T.roots[i];
        const int off = s * L * L + r0 * L;
        const cx<R>* srcp = W + rhs * T.N + (long long)t * T.V + off;
        for (int i = threadIdx.x; i < nr * L; i += blockDim.x) buf[i] = srcp[i];
        __syncthreads();
        fft_lines<R, true>(buf, LineMap{1, L, 0, 1}, nr, T.plan, roots);
        for (int i = threadIdx.x; i < nr * L; i += blockDim.x) epi_apply(epi, rhs, t, off + i, buf[i], T, sc, acc);
    }
    if constexpr (Ctl::kEnd) ctl.end(acc, rhs, slot, sc, red_lds);
}

// ----------------------------------------------------------------------------- split, compile-time L
// The three split kernels with L and the tile sizes known at compile time (both dividing L),
// so the radix plan, the index arithmetic and the DFT coefficients are constants.  The tile
// stages generalise ct_stage: line l of an LDS tile starts at (l / LG) * LGG + (l % LG) * LH
// and its elements are ES apart; rows (ES = 1) give consecutive threads consecutive
// butterflies of a line, columns give them consecutive lines.
template <typename R, int L, int Q, bool INV, int NT, int NL, int LG, int LGG, int LH, int ES>
__device__ __forceinline__ void ct_stage_tile(cx<R>* __restrict__ buf, const cx<R>* __restrict__ roots) {
    constexpr CPlan P = make_cplan(L);
    constexpr int RAD = P.radix[Q], LQ = P.len[Q], M = LQ / RAD, PER = L / RAD;
    constexpr int NTASK = NL * PER, TWS = L / LQ, ST = M * ES;
    for (int task = threadIdx.x; task < NTASK; task += NT) {
        int line, j;
        if constexpr (ES == 1) {
            line = task / PER;
            j = task - line * PER;
        } else {
            j = task / NL;
            line = task - j * NL;
        }
        const int b = j / M, np = j - b * M;
        const int lq = line / LG;
        const int base = lq * LGG + (line - lq * LG) * LH + (b * LQ + np) * ES;
        cx<R> x[RAD];
#pragma unroll
        for (int i = 0; i < RAD; ++i) x[i] = buf[base + i * ST];
        if constexpr (!INV) {
            small_dft_ct<R, RAD, false>(x);
            if constexpr (M > 1) {
#pragma unroll
                for (int k = 1; k < RAD; ++k) x[k] = cmul(x[k], roots[np * k * TWS]);
            }
        } else {
            if constexpr (M > 1) {
#pragma unroll
                for (int k = 1; k < RAD; ++k) x[k] = cmulc(x[k], roots[np * k * TWS]);
            }
            small_dft_ct<R, RAD, true>(x);
        }
#pragma unroll
        for (int i = 0; i < RAD; ++i) buf[base + i * ST] = x[i];
    }
}

template <typename R, int L, int Q, int QEND, int NT, int NL, int LG, int LGG, int LH, int ES>
__device__ __forceinline__ void ct_forward_tile(cx<R>* buf, const cx<R>* roots) {
    if constexpr (Q < QEND) {
        ct_stage_tile<R, L, Q, false, NT, NL, LG, LGG, LH, ES>(buf, roots);
        __syncthreads();
        ct_forward_tile<R, L, Q + 1, QEND, NT, NL, LG, LGG, LH, ES>(buf, roots);
    }
}

template <typename R, int L, int Q, int QLO, int NT, int NL, int LG, int LGG, int LH, int ES>
__device__ __forceinline__ void ct_inverse_tile(cx<R>* buf, const cx<R>* roots) {
    if constexpr (Q >= QLO) {
        ct_stage_tile<R, L, Q, true, NT, NL, LG, LGG, LH, ES>(buf, roots);
        __syncthreads();
        ct_inverse_tile<R, L, Q - 1, QLO, NT, NL, LG, LGG, LH, ES>(buf, roots);
    }
}

// (1) RB rows of one sublattice of the source slice, transformed, to the scratch vector W
template <typename R, int L, int RB, int NT, class Src, class Ctl>
__global__ void __launch_bounds__(NT)
k_split_rows_fwd_ct(const OpTab<R> T, const Src src, cx<R>* __restrict__ W, const Ctl ctl) {
    static_assert(L % RB == 0, "row blocks must tile the sublattice");
    constexpr int NRB = L / RB;
    constexpr CPlan P = make_cplan(L);
    extern __shared__ __align__(16) unsigned char smem[];
    __shared__ double red_lds[64];
    cx<R>* buf = reinterpret_cast<cx<R>*>(smem);
    cx<R>* roots = buf + RB * L;
    int b = blockIdx.x;
    const int rblk = b % NRB;
    b /= NRB;
    const int s = b % 2;
    b /= 2;
    const int t = b % T.Nt;
    const int rhs = b / T.Nt;
    const Scal sc = ctl.begin(rhs, -1, red_lds);
    if (!sc.open) return;
    for (int i = threadIdx.x; i < L; i += NT) roots[i] = T.roots[i];
    const int ts = src.slice(t, T.Nt);
    const int off = s * L * L + rblk * RB * L;
    for (int i = threadIdx.x; i < RB * L; i += NT) buf[i] = src_apply(src, rhs, ts, off + i, T, sc);
    __syncthreads();
    ct_forward_tile<R, L, 0, P.nst, NT, RB, 1, L, 0, 1>(buf, roots);
    cx<R>* dst = W + rhs * T.N + (long long)t * T.V + off;
    for (int i = threadIdx.x; i < RB * L; i += NT) dst[i] = buf[i];
}

// (2) CB columns of both sublattices: column transforms, E(k), inverse column transforms, in W
template <typename R, int L, int CB, int NT, class Ctl>
__global__ void __launch_bounds__(NT)
k_split_cols_ct(const OpTab<R> T, cx<R>* __restrict__ W, const Ctl ctl) {
    static_assert(L % CB == 0, "column blocks must tile the sublattice");
    constexpr int NCB = L / CB;
    constexpr CPlan P = make_cplan(L);
    extern __shared__ __align__(16) unsigned char smem[];
    __shared__ double red_lds[64];
    cx<R>* buf = reinterpret_cast<cx<R>*>(smem);
    cx<R>* roots = buf + 2 * L * CB;
    int b = blockIdx.x;
    const int cblk = b % NCB;
    b /= NCB;
    const int t = b % T.Nt;
    const int rhs = b / T.Nt;
    const Scal sc = ctl.begin(rhs, -1, red_lds);
    if (!sc.open) return;
    const int c0 = cblk * CB;
    for (int i = threadIdx.x; i < L; i += NT) roots[i] = T.roots[i];
    cx<R>* base = W + rhs * T.N + (long long)t * T.V;
    // LDS tile [s][n1][c], c fastest
    for (int i = threadIdx.x; i < 2 * L * CB; i += NT) {
        const int c = i % CB, sn = i / CB;           // sn = s*L + n1
        buf[i] = base[(long long)sn * L + c0 + c];
    }
    __syncthreads();
    ct_forward_tile<R, L, 0, P.nst, NT, 2 * CB, CB, L * CB, 1, CB>(buf, roots);
    for (int i = threadIdx.x; i < L * CB; i += NT) {
        const int c = i % CB, n1 = i / CB;
        const int p = n1 * L + c0 + c;
        const R cc = T.etab[4 * p], sr = T.etab[4 * p + 1], si = T.etab[4 * p + 2];
        const cx<R> a = buf[i], bb = buf[L * CB + i];
        buf[i] = {cc * a.re + sr * bb.re - si * bb.im, cc * a.im + sr * bb.im + si * bb.re};
        buf[L * CB + i] = {cc * bb.re + sr * a.re + si * a.im, cc * bb.im + sr * a.im - si * a.re};
    }
    __syncthreads();
    ct_inverse_tile<R, L, P.nst - 1, 0, NT, 2 * CB, CB, L * CB, 1, CB>(buf, roots);
    for (int i = threadIdx.x; i < 2 * L * CB; i += NT) {
        const int c = i % CB, sn = i / CB;
        base[(long long)sn * L + c0 + c] = buf[i];
    }
}

// (3) RB rows of W, inverse row transforms, and the epilogue
template <typename R, int L, int RB, int NT, class Epi, class Ctl>
__global__ void __launch_bounds__(NT)
k_split_rows_inv_ct(const OpTab<R> T, const cx<R>* __restrict__ W, const Epi epi, const Ctl ctl) {
    static_assert(L % RB == 0, "row blocks must tile the sublattice");
    constexpr int NRB = L / RB;
    constexpr CPlan P = make_cplan(L);
    extern __shared__ __align__(16) unsigned char smem[];
    __shared__ double red_lds[64];
    cx<R>* buf = reinterpret_cast<cx<R>*>(smem);
    cx<R>* roots = buf + RB * L;
    int b = blockIdx.x;
    const int slot = b % (2 * NRB * T.Nt);
    const int rblk = b % NRB;
    b /= NRB;
    const int s = b % 2;
    b /= 2;
    const int t = b % T.Nt;
    const int rhs = b / T.Nt;
    const Scal sc = ctl.begin(rhs, slot, red_lds);
    double acc = 0.0;
    if (sc.open) {
        for (int i = threadIdx.x; i < L; i += NT) roots[i] = T.roots[i];
        const int off = s * L * L + rblk * RB * L;
        const cx<R>* srcp = W + rhs * T.N + (long long)t * T.V + off;
        for (int i = threadIdx.x; i < RB * L; i += NT) buf[i] = srcp[i];
        __syncthreads();
        ct_inverse_tile<R, L, P.nst - 1, 0, NT, RB, 1, L, 0, 1>(buf, roots);
        for (int i = threadIdx.x; i < RB * L; i += NT) epi_apply(epi, rhs, t, off + i, buf[i], T, sc, acc);
    }
    if constexpr (Ctl::kEnd) ctl.end(acc, rhs, slot, sc, red_lds);
}

// ----------------------------------------------------------------------------- linear form
// The fermion matrix as printed in Sec. 2, eq. "ferm_op" (linear in delta*kappa) is a
// nearest-neighbour stencil in space and time: for destination (t, x)
//     M,     A site:  B_{t+1} v_{t+1,x} - e^{i phi_{t,x}}  v_{t,x} - dk sum_y v_{t,y}
//     M,     B site:  v_{t,x} - B_t e^{-i phi_{t,x}} v_{t-1,x}      - dk sum_y v_{t,y}
//     M^dag, A site:  B_t v_{t-1,x} - e^{-i phi_{t,x}} v_{t,x}      - dk sum_y v_{t,y}
//     M^dag, B site:  v_{t,x} - B_{t+1} e^{i phi_{t+1,x}} v_{t+1,x} - dk sum_y v_{t,y}
// (y over the three neighbours on the other sublattice, B_0 = -1).  Every output is one
// diagonal term, one time hop and three equal-time hops, so the kernel streams its
// vectors once from HBM; the neighbour entries are re-read from the caches.
constexpr int kLinThreads = 512;

template <typename R>
struct LinTab {
    int L, LL, V, Nt;
    int nch, chunk;              // chunks per slice, sites per chunk
    long long N;
    R dk;
};

// A linear-form source supplies the vector the operator acts on, entry by entry.
template <typename R>
struct LSrcVec {                 // v
    using Pre = cx<R>;
    const cx<R>* v;
    __device__ Pre fetch(long long k) const { return v[k]; }
    __device__ cx<R> make(const Pre& a, const Scal&) const { return a; }
};

template <typename R>
struct LSrcSearch {              // r + beta p                          (CG: the new direction)
    using Pre = PrePair<R>;
    const cx<R>* r;
    const cx<R>* p;
    __device__ Pre fetch(long long k) const { return {r[k], p[k]}; }
    __device__ cx<R> make(const Pre& a, const Scal& s) const {
        const R b = (R)s.beta;
        return {a.a.re + b * a.b.re, a.a.im + b * a.b.im};
    }
};

// A linear-form output receives the operator's value o at entry k.
template <typename R>
struct LOutStore {               // out = o
    using Pre = int;
    cx<R>* out;
    __device__ Pre fetch(long long) const { return 0; }
    __device__ void store(long long k, cx<R> o, const Pre&, const Scal&, double&) const { out[k] = o; }
};

template <typename R>
struct LOutSearch {              // CG: tv = M^dag (r + beta p); acc |tv|^2
    using Pre = int;
    cx<R>* tv;
    __device__ Pre fetch(long long) const { return 0; }
    __device__ void store(long long k, cx<R> o, const Pre&, const Scal&, double& acc) const {
        tv[k] = o;
        acc += (double)o.re * (double)o.re + (double)o.im * (double)o.im;
    }
};

template <typename R>
struct LPreUpdate {
    cx<R> p, x, r;
};
template <typename R>
struct LPreUpdateNoX {
    cx<R> p, r;
};

template <typename R, int XM = kXPlain>
struct LOutUpdate {              // CG: q = M tv; p = r + beta p; x += alpha p; r -= alpha q; acc |r|^2
    // XM: how x is updated (kXPlain, kXSkip, kXPair; see EpiUpdate)
    using Pre = std::conditional_t<XM == kXSkip, LPreUpdateNoX<R>, LPreUpdate<R>>;
    static constexpr int kXMode = XM;
    cx<R>* p;
    cx<R>* x;
    cx<R>* r;
    __device__ Pre fetch(long long k) const {
        if constexpr (XM == kXSkip) return {p[k], r[k]};
        else return {p[k], x[k], r[k]};
    }
    __device__ void store(long long k, cx<R> q, const Pre& a, const Scal& sc, double& acc) const {
        const R b = (R)sc.beta, al = (R)sc.alpha;
        const cx<R> pn = {a.r.re + b * a.p.re, a.r.im + b * a.p.im};
        const cx<R> rn = {a.r.re - al * q.re, a.r.im - al * q.im};
        p[k] = pn;
        if constexpr (XM == kXPlain) {
            x[k] = {a.x.re + al * pn.re, a.x.im + al * pn.im};
        } else if constexpr (XM == kXPair) {
            const R ap = (R)sc.alpha_prev;
            x[k] = {fmar(al, pn.re, fmar(ap, a.p.re, a.x.re)), fmar(al, pn.im, fmar(ap, a.p.im, a.x.im))};
        }
        r[k] = rn;
        acc += (double)rn.re * (double)rn.re + (double)rn.im * (double)rn.im;
    }
    // a paired step of a right-hand side that went idle after the skip: add the pending term
    __device__ void closed(long long k, const Pre& a, const Scal& sc) const {
        if constexpr (XM == kXPair) {
            const R ap = (R)sc.alpha_prev;
            x[k] = {fmar(ap, a.p.re, a.x.re), fmar(ap, a.p.im, a.x.im)};
        }
    }
};

template <typename Rlo>
struct LOutResidual {            // FP64: r_hi = chi - o (o = M M^dag x_hi); r_lo = r_hi; acc |r_hi|^2
    using Pre = cx<double>;
    const cx<double>* chi;
    cx<double>* rhi;
    cx<Rlo>* rlo;
    __device__ Pre fetch(long long k) const { return chi[k]; }
    __device__ void store(long long k, cx<double> o, const Pre& c, const Scal&, double& acc) const {
        const cx<double> rv = c - o;
        rhi[k] = rv;
        rlo[k] = {(Rlo)rv.re, (Rlo)rv.im};
        acc += rv.re * rv.re + rv.im * rv.im;
    }
};

// Where the stencil of site i reads: the three neighbours on the other sublattice
// (A(n) - B(n), B(n - e1), B(n - e2); cell n = (n1, n2), x = s L^2 + n1 L + n2).
__device__ __forceinline__ void lin_neighbours(int i, int L, int LL, int nb[3]) {
    const int s = i >= LL ? 1 : 0;
    const int n = i - s * LL;
    const int n1 = n / L, n2 = n - n1 * L;
    if (s == 0) {
        nb[0] = LL + n;
        nb[1] = LL + (n1 == 0 ? L - 1 : n1 - 1) * L + n2;
        nb[2] = LL + n1 * L + (n2 == 0 ? L - 1 : n2 - 1);
    } else {
        nb[0] = n;
        nb[1] = (n1 == L - 1 ? 0 : n1 + 1) * L + n2;
        nb[2] = n1 * L + (n2 == L - 1 ? 0 : n2 + 1);
    }
}

template <typename R, class Src, class Ph>
struct LinPre {
    typename Src::Pre own, hop, nb[3];
    typename Ph::Pre ph;
};

// One workgroup per (right-hand side, slice, chunk of sites).  The first NB sites of each
// thread have every load issued before the block learns its CG scalars (the loads do not
// depend on them), so the scalar reduction and the data fetch overlap; sites beyond
// NB * kLinThreads per chunk follow in further batches.
template <typename R, bool DAG, class Ph, class Src>
__device__ __forceinline__ void lin_fetch(const LinTab<R>& T, const Ph& ph, const Src& src, int i, long long vb,
                                          long long row, long long rowA, long long rowB, long long phB,
                                          LinPre<R, Src, Ph>& pre) {
    int nb[3];
    lin_neighbours(i, T.L, T.LL, nb);
    const bool a = i < T.LL;
    pre.own = src.fetch(vb + row + i);
    pre.hop = src.fetch(vb + (a ? rowA : rowB) + i);
#pragma unroll
    for (int m = 0; m < 3; ++m) pre.nb[m] = src.fetch(vb + row + nb[m]);
    pre.ph = ph.fetch((a ? row : phB) + i);
}

template <typename R, bool DAG, class Ph, class Src>
__device__ __forceinline__ cx<R> lin_value(const LinTab<R>& T, const Ph& ph, const Src& src, int i, R sgnA, R sgnB,
                                           const LinPre<R, Src, Ph>& pre, const Scal& sc) {
    const bool a = i < T.LL;
    const cx<R> v = src.make(pre.own, sc);
    const cx<R> h = src.make(pre.hop, sc);
    cx<R> s3 = src.make(pre.nb[0], sc);
    s3 = s3 + src.make(pre.nb[1], sc);
    s3 = s3 + src.make(pre.nb[2], sc);
    const cx<R> e = ph.value(pre.ph);
    // e^{+i phi} for M on A sites and M^dag on B sites, e^{-i phi} otherwise
    const cx<R> f = (a != DAG) ? e : cx<R>{e.re, -e.im};
    cx<R> o;
    if (a) {                                  // sgn h - f v
        const cx<R> fv = cmul(f, v);
        o = {sgnA * h.re - fv.re, sgnA * h.im - fv.im};
    } else {                                  // v - sgn f h
        const cx<R> fh = cmul(f, h);
        o = {v.re - sgnB * fh.re, v.im - sgnB * fh.im};
    }
    return {o.re - T.dk * s3.re, o.im - T.dk * s3.im};
}

template <typename R, bool DAG, int NB, class Ph, class Src, class Out, class Ctl>
__global__ void __launch_bounds__(kLinThreads)
k_lin(const LinTab<R> T, const Ph ph, const Src src, const Out out, const Ctl ctl) {
    __shared__ double red_lds[64];
    const int u = xcd_linear(blockIdx.x, gridDim.x);
    const int per_rhs = T.Nt * T.nch;
    const int rhs = u / per_rhs, slot = u - rhs * per_rhs;
    const int t = slot / T.nch, ch = slot - t * T.nch;
    const int i0 = ch * T.chunk;
    const int i1 = min(T.V, i0 + T.chunk);
    const int tp = prev_slice(t, T.Nt), tn = next_slice(t, T.Nt);
    const long long vb = rhs * T.N;
    const long long row = (long long)t * T.V;
    // A sites hop to t+1 (M) or t-1 (M^dag); B sites the other way
    const long long rowA = (long long)(DAG ? tp : tn) * T.V;
    const long long rowB = (long long)(DAG ? tn : tp) * T.V;
    const R sgnA = (DAG ? t == 0 : t == T.Nt - 1) ? (R)-1 : (R)1;
    const R sgnB = (DAG ? t == T.Nt - 1 : t == 0) ? (R)-1 : (R)1;
    const long long phB = DAG ? (long long)tn * T.V : row;   // phase slice of the B-site hop
    const int first = i0 + (int)threadIdx.x;
    LinPre<R, Src, Ph> pre[NB];
    typename Out::Pre op[NB];
#pragma unroll
    for (int j = 0; j < NB; ++j) {
        const int i = first + j * kLinThreads;
        if (i < i1) {
            lin_fetch<R, DAG>(T, ph, src, i, vb, row, rowA, rowB, phB, pre[j]);
            op[j] = out.fetch(vb + row + i);
        }
    }
    const Scal sc = ctl.begin(rhs, slot, red_lds);
    double acc = 0.0;
    if (sc.open) {
#pragma unroll
        for (int j = 0; j < NB; ++j) {
            const int i = first + j * kLinThreads;
            if (i < i1) out.store(vb + row + i, lin_value<R, DAG>(T, ph, src, i, sgnA, sgnB, pre[j], sc), op[j], sc, acc);
        }
        for (int base = first + NB * kLinThreads; base < i1; base += NB * kLinThreads) {
#pragma unroll
            for (int j = 0; j < NB; ++j) {
                const int i = base + j * kLinThreads;
                if (i < i1) {
                    lin_fetch<R, DAG>(T, ph, src, i, vb, row, rowA, rowB, phB, pre[j]);
                    op[j] = out.fetch(vb + row + i);
                }
            }
#pragma unroll
            for (int j = 0; j < NB; ++j) {
                const int i = base + j * kLinThreads;
                if (i < i1)
                    out.store(vb + row + i, lin_value<R, DAG>(T, ph, src, i, sgnA, sgnB, pre[j], sc), op[j], sc, acc);
            }
        }
    } else if (sc.pending) {
        // an idle block of a paired x update whose previous step skipped x: add the pending term
        if constexpr (EpiHasClosed<Out>::value) {
            for (int i = first; i < i1; i += kLinThreads) out.closed(vb + row + i, out.fetch(vb + row + i), sc);
        }
    }
    if constexpr (Ctl::kEnd) ctl.end(acc, rhs, slot, sc, red_lds);
}

// Force of the linear form, summed over right-hand sides, with y = M^dag x formed where
// it is needed (phi_{t,z} enters one entry of M):
//     A site:  g = -2 Im(e^{i phi_{t,z}} conj(x_{t,z}) y_{t,z})
//     B site:  g = 2 B_t Im(e^{-i phi_{t,z}} conj(x_{t,z}) y_{t-1,z})
// One thread per (t, z).
__global__ void __launch_bounds__(kThreads)
k_lin_force(const LinTab<double> T, const double* __restrict__ phi, const cx<double>* __restrict__ x,
            double* __restrict__ g, int nrhs) {
    const long long n = T.N;
    for (long long k = blockIdx.x * (long long)blockDim.x + threadIdx.x; k < n;
         k += (long long)gridDim.x * blockDim.x) {
        const int t = (int)(k / T.V), i = (int)(k - (long long)t * T.V);
        const bool a = i < T.LL;
        const int tp = prev_slice(t, T.Nt);
        int nb[3];
        lin_neighbours(i, T.L, T.LL, nb);
        double s, c;
        phase_sincos(phi[k], &s, &c);
        const double bt = t == 0 ? -1.0 : 1.0;
        // y at (ty, i): A sites y_{t} = B_t x_{t-1} - e^{-i phi_t} x_t - dk sum x_{t,nb};
        //               B sites y_{t-1} = x_{t-1} - B_t e^{i phi_t} x_t - dk sum x_{t-1,nb}
        const long long ry = (long long)(a ? t : tp) * T.V;
        double acc = 0.0;
        for (int r = 0; r < nrhs; ++r) {
            const cx<double>* xv = x + r * n;
            const cx<double> xt = xv[k], xp = xv[(long long)tp * T.V + i];
            cx<double> s3 = xv[ry + nb[0]];
            s3 = s3 + xv[ry + nb[1]];
            s3 = s3 + xv[ry + nb[2]];
            cx<double> y;
            if (a) {
                const cx<double> ex = cmulc(xt, cx<double>{c, s});     // e^{-i phi} x_t
                y = {bt * xp.re - ex.re - T.dk * s3.re, bt * xp.im - ex.im - T.dk * s3.im};
                const cx<double> z = cmul(cx<double>{c, s}, cmulc(y, xt));   // e^{i phi} conj(x) y
                acc += -2.0 * z.im;
            } else {
                const cx<double> ex = cmul(xt, cx<double>{c, s});      // e^{i phi} x_t
                y = {xp.re - bt * ex.re - T.dk * s3.re, xp.im - bt * ex.im - T.dk * s3.im};
                const cx<double> z = cmulc(cmulc(y, xt), cx<double>{c, s});  // e^{-i phi} conj(x) y
                acc += 2.0 * bt * z.im;
            }
        }
        g[k] = acc;
    }
}

// ----------------------------------------------------------------------------- elementwise kernels
// One block per (right-hand side, slice); reductions in slice order.
template <typename Rlo>
__global__ void __launch_bounds__(kThreads)
k_cg_init(const cx<double>* __restrict__ chi, cx<double>* __restrict__ xhi, cx<double>* __restrict__ rhi,
          cx<Rlo>* __restrict__ xlo, cx<Rlo>* __restrict__ rlo, cx<Rlo>* __restrict__ p, int V, int Nt,
          int zero_start, FinInit fin, RedArgs ra) {
    __shared__ double red_lds[64];
    const int t = blockIdx.x % Nt, rhs = blockIdx.x / Nt;
    const long long base = (long long)rhs * V * Nt + (long long)t * V;
    double acc = 0.0;
    for (int i = threadIdx.x; i < V; i += blockDim.x) {
        const long long k = base + i;
        const cx<double> c = chi[k];
        acc += c.re * c.re + c.im * c.im;
        xlo[k] = {(Rlo)0, (Rlo)0};
        p[k] = {(Rlo)0, (Rlo)0};
        if (zero_start) {
            xhi[k] = {0.0, 0.0};
            rhi[k] = c;
            rlo[k] = {(Rlo)c.re, (Rlo)c.im};
        }
    }
    reduce_and_finalize(acc, rhs, t, ra, fin, red_lds);
}

// x_hi += x_lo, x_lo = 0 for right-hand sides not yet done (grid-stride over N per rhs,
// gridDim.y = nrhs)
template <typename Rlo>
__global__ void __launch_bounds__(kThreads)
k_fold_solution(cx<double>* __restrict__ xhi, cx<Rlo>* __restrict__ xlo, long long N, const CgScalars* sc) {
    const int rhs = blockIdx.y;
    if (sc[rhs].done) return;
    const long long base = (long long)rhs * N;
    for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < N;
         i += (long long)gridDim.x * blockDim.x) {
        const cx<Rlo> a = xlo[base + i];
        const cx<double> h = xhi[base + i];
        xhi[base + i] = {h.re + (double)a.re, h.im + (double)a.im};
        xlo[base + i] = {(Rlo)0, (Rlo)0};
    }
}

// x = 0 for right-hand sides whose chi is zero (their exact solution)
__global__ void __launch_bounds__(kThreads)
k_zero_trivial(cx<double>* __restrict__ xhi, int V, int Nt, const CgScalars* sc) {
    const int t = blockIdx.x % Nt, rhs = blockIdx.x / Nt;
    if (sc[rhs].chichi != 0.0) return;
    const long long base = (long long)rhs * V * Nt + (long long)t * V;
    for (int i = threadIdx.x; i < V; i += blockDim.x) xhi[base + i] = {0.0, 0.0};
}

__global__ void __launch_bounds__(kThreads)
k_dot_re(const cx<double>* __restrict__ a, const cx<double>* __restrict__ b, int V, int Nt,
         FinStore fin, RedArgs ra) {
    __shared__ double red_lds[64];
    const int t = blockIdx.x % Nt, rhs = blockIdx.x / Nt;
    const long long base = (long long)rhs * V * Nt + (long long)t * V;
    double acc = 0.0;
    for (int i = threadIdx.x; i < V; i += blockDim.x) {
        const cx<double> x = a[base + i], y = b[base + i];
        acc += x.re * y.re + x.im * y.im;
    }
    reduce_and_finalize(acc, rhs, t, ra, fin, red_lds);
}

// Molecular-dynamics update of the HMC trajectory: F = phi/(delta U) + dS_f/dphi,
// pi -= eps_pi F, then phi += eps_phi pi.
__global__ void __launch_bounds__(kThreads)
k_md_update(double* __restrict__ phi, double* __restrict__ pi, const double* __restrict__ g, long long n,
            double inv_dU, double eps_pi, double eps_phi) {
    for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < n;
         i += (long long)gridDim.x * blockDim.x) {
        const double f = fma(phi[i], inv_dU, g[i]);
        const double p = fma(-eps_pi, f, pi[i]);
        pi[i] = p;
        phi[i] = fma(eps_phi, p, phi[i]);
    }
}

// Bosonic part of the HMC Hamiltonian, sum over one slice per block:
// pi^2 / 2 + phi^2 / (2 delta U).
__global__ void __launch_bounds__(kThreads)
k_boson_energy(const double* __restrict__ phi, const double* __restrict__ pi, int V, double inv_dU, FinStore fin,
               RedArgs ra) {
    __shared__ double red_lds[64];
    const int t = blockIdx.x;
    const long long base = (long long)t * V;
    double acc = 0.0;
    for (int i = threadIdx.x; i < V; i += blockDim.x) {
        const double a = phi[base + i], b = pi[base + i];
        acc += 0.5 * b * b + 0.5 * inv_dU * a * a;
    }
    reduce_and_finalize(acc, 0, t, ra, fin, red_lds);
}

__global__ void __launch_bounds__(kThreads)
k_sum_rhs(const double* __restrict__ parts, double* __restrict__ g, long long n, int nrhs) {
    for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < n;
         i += (long long)gridDim.x * blockDim.x) {
        double s = parts[i];
        for (int r = 1; r < nrhs; ++r) s += parts[r * n + i];
        g[i] = s;
    }
}

// X = 1 (V x V, column-major)
__global__ void __launch_bounds__(kThreads)
k_identity(cx<double>* __restrict__ X, int V) {
    const long long n = (long long)V * V;
    for (long long e = blockIdx.x * (long long)blockDim.x + threadIdx.x; e < n; e += (long long)gridDim.x * blockDim.x)
        X[e] = {(e / V == e % V) ? 1.0 : 0.0, 0.0};
}

// X += 1
__global__ void __launch_bounds__(kThreads)
k_add_identity(cx<double>* __restrict__ X, int V) {
    for (int j = blockIdx.x * blockDim.x + threadIdx.x; j < V; j += gridDim.x * blockDim.x)
        X[(long long)j * V + j].re += 1.0;
}

// log|det A| and arg det A of a V x V complex matrix (column-major: A[j * V + i] is row i of
// column j) by LU with partial pivoting (largest |a_ik|, ties to the lowest row) in one
// workgroup of kLuThreads; A is overwritten.  out[0] = log|det A| (-inf when a pivot column
// is zero), out[1] = arg det A reduced to (-pi, pi].  Every sum has a fixed order.
constexpr int kLuThreads = 1024;

__global__ void __launch_bounds__(kLuThreads)
k_lu_logdet(cx<double>* __restrict__ A, int V, double* __restrict__ out) {
    extern __shared__ __align__(16) unsigned char smem[];
    cx<double>* lcol = reinterpret_cast<cx<double>*>(smem);     // multipliers of column k
    cx<double>* urow = lcol + V;                               // row k right of the pivot
    __shared__ double wbest[kLuThreads / 64];
    __shared__ int widx[kLuThreads / 64];
    __shared__ int piv;
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    double lsum = 0.0, asum = 0.0;                              // thread 0's accumulators
    bool singular = false;
    for (int k = 0; k < V; ++k) {
        double best = -1.0;
        int bi = V;
        for (int i = k + tid; i < V; i += kLuThreads) {
            const cx<double> a = A[(long long)k * V + i];
            const double m = a.re * a.re + a.im * a.im;
            if (m > best) { best = m; bi = i; }
        }
#pragma unroll
        for (int off = 32; off > 0; off >>= 1) {
            const double ob = __shfl_xor(best, off, 64);
            const int oi = __shfl_xor(bi, off, 64);
            if (ob > best || (ob == best && oi < bi)) { best = ob; bi = oi; }
        }
        if (lane == 0) { wbest[wave] = best; widx[wave] = bi; }
        __syncthreads();
        if (tid == 0) {
            double b = wbest[0];
            int p = widx[0];
            for (int w = 1; w < kLuThreads / 64; ++w)
                if (wbest[w] > b || (wbest[w] == b && widx[w] < p)) { b = wbest[w]; p = widx[w]; }
            piv = (b > 0.0) ? p : -1;
        }
        __syncthreads();
        const int p = piv;
        if (p < 0) { singular = true; break; }          // uniform: every thread read the same piv
        if (p != k) {
            for (int j = tid; j < V; j += kLuThreads) {
                const long long c = (long long)j * V;
                const cx<double> t = A[c + k];
                A[c + k] = A[c + p];
                A[c + p] = t;
            }
        }
        __syncthreads();
        const cx<double> akk = A[(long long)k * V + k];
        if (tid == 0) {
            lsum += 0.5 * log(akk.re * akk.re + akk.im * akk.im);
            asum = remainder(asum + atan2(akk.im, akk.re) + (p != k ? 3.14159265358979323846 : 0.0),
                             6.28318530717958647692);
        }
        const double inv = 1.0 / (akk.re * akk.re + akk.im * akk.im);
        for (int i = k + 1 + tid; i < V; i += kLuThreads) {
            const cx<double> a = A[(long long)k * V + i];
            lcol[i] = {(a.re * akk.re + a.im * akk.im) * inv, (a.im * akk.re - a.re * akk.im) * inv};   // a / akk
        }
        for (int j = k + 1 + tid; j < V; j += kLuThreads) urow[j] = A[(long long)j * V + k];
        __syncthreads();
        const int m = V - k - 1;
        const long long tot = (long long)m * m;
        for (long long e = tid; e < tot; e += kLuThreads) {
            const int j = k + 1 + (int)(e / m), i = k + 1 + (int)(e % m);
            const cx<double> l = lcol[i], u = urow[j];
            cx<double>& a = A[(long long)j * V + i];
            a.re -= l.re * u.re - l.im * u.im;
            a.im -= l.re * u.im + l.im * u.re;
        }
        __syncthreads();
    }
    if (tid == 0) {
        out[0] = singular ? -__builtin_huge_val() : lsum;
        out[1] = singular ? 0.0 : asum;
    }
}

__global__ void __launch_bounds__(kThreads)
k_to_float(const double* __restrict__ a, float* __restrict__ b, long long n) {
    for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < n;
         i += (long long)gridDim.x * blockDim.x)
        b[i] = (float)a[i];
}

}  // namespace hub
