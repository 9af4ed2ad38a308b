// In-LDS mixed-radix transforms of the L x L torus for gfx950.
//
// The forward transform is an in-place decimation-in-frequency Cooley-Tukey
// transform: natural-order input, output in mixed-radix digit-reversed order.
// The inverse is the exact reverse sequence of stages (conjugate twiddles, then
// conjugate butterflies): digit-reversed input, natural-order output, scaled by L.
// Every butterfly reads and writes the same LDS slots, so a stage needs no second
// buffer and threads are independent within a stage.  Momentum-space work between
// the two (the 2 x 2 hopping exponential) indexes its table by transform position,
// so no permutation pass is ever made.
#pragma once

#include <hip/hip_runtime.h>

#include "hub_internal.hpp"

namespace hub {

template <typename R>
struct alignas(2 * sizeof(R)) cx {
    R re, im;
};

template <typename R>
__device__ __forceinline__ cx<R> operator+(cx<R> a, cx<R> b) { return {a.re + b.re, a.im + b.im}; }
template <typename R>
__device__ __forceinline__ cx<R> operator-(cx<R> a, cx<R> b) { return {a.re - b.re, a.im - b.im}; }
template <typename R>
__device__ __forceinline__ cx<R> scale(R s, cx<R> a) { return {s * a.re, s * a.im}; }
template <typename R>
__device__ __forceinline__ cx<R> cmul(cx<R> a, cx<R> b) {
    return {a.re * b.re - a.im * b.im, a.re * b.im + a.im * b.re};
}
// a * conj(b)
template <typename R>
__device__ __forceinline__ cx<R> cmulc(cx<R> a, cx<R> b) {
    return {a.re * b.re + a.im * b.im, a.im * b.re - a.re * b.im};
}
__device__ __forceinline__ float fmar(float a, float b, float c) { return fmaf(a, b, c); }
__device__ __forceinline__ double fmar(double a, double b, double c) { return fma(a, b, c); }

// a - i b  and  a + i b
template <typename R>
__device__ __forceinline__ cx<R> sub_i(cx<R> a, cx<R> b) { return {a.re + b.im, a.im - b.re}; }
template <typename R>
__device__ __forceinline__ cx<R> add_i(cx<R> a, cx<R> b) { return {a.re - b.im, a.im + b.re}; }

// Lines of a transform inside an LDS tile: line l starts at
// (l / g) * G + (l % g) * h and its elements are es apart.
struct LineMap {
    int g, G, h, es;
};

__device__ __forceinline__ int line_base(const LineMap& m, int l) {
    const int q = l / m.g;
    return q * m.G + (l - q * m.g) * m.h;
}

// r-point DFT in registers.  Forward: X_k = sum_j x_j e^{-2 pi i jk/r}; inverse uses
// e^{+2 pi i jk/r} (unnormalised).  cs[m] = cos(2 pi m/r), sn[m] = sin(2 pi m/r) are
// needed for odd r >= 5, which use the real-coefficient split
//   X_k, X_{r-k} = x_0 + sum_j cos(.)(x_j + x_{r-j})  -/+  i sum_j sin(.)(x_j - x_{r-j}).
template <typename R, int RAD, bool INV>
__device__ __forceinline__ void small_dft(cx<R>* x, const R* cs, const R* sn) {
    if constexpr (RAD == 2) {
        const cx<R> a = x[0], b = x[1];
        x[0] = a + b;
        x[1] = a - b;
    } else if constexpr (RAD == 3) {
        const R s3 = (R)0.86602540378443864676;   // sin(2 pi / 3)
        const cx<R> t1 = x[1] + x[2];
        const cx<R> t2 = {x[0].re - (R)0.5 * t1.re, x[0].im - (R)0.5 * t1.im};
        const cx<R> t3 = scale(s3, x[1] - x[2]);
        x[0] = x[0] + t1;
        if constexpr (!INV) {
            x[1] = sub_i(t2, t3);
            x[2] = add_i(t2, t3);
        } else {
            x[1] = add_i(t2, t3);
            x[2] = sub_i(t2, t3);
        }
    } else if constexpr (RAD == 4) {
        const cx<R> a = x[0] + x[2], b = x[0] - x[2];
        const cx<R> c = x[1] + x[3], d = x[1] - x[3];
        x[0] = a + c;
        x[2] = a - c;
        if constexpr (!INV) {
            x[1] = sub_i(b, d);
            x[3] = add_i(b, d);
        } else {
            x[1] = add_i(b, d);
            x[3] = sub_i(b, d);
        }
    } else {
        static_assert(RAD % 2 == 1, "odd radix expected");
        constexpr int H = (RAD - 1) / 2;
        cx<R> e[H + 1], o[H + 1];
        cx<R> x0 = x[0];
        cx<R> s0 = x0;
#pragma unroll
        for (int j = 1; j <= H; ++j) {
            e[j] = x[j] + x[RAD - j];
            o[j] = x[j] - x[RAD - j];
            s0 = s0 + e[j];
        }
        x[0] = s0;
#pragma unroll
        for (int k = 1; k <= H; ++k) {
            cx<R> A = x0;
            cx<R> B = {(R)0, (R)0};
#pragma unroll
            for (int j = 1; j <= H; ++j) {
                const int m = (j * k) % RAD;
                A.re += cs[m] * e[j].re;
                A.im += cs[m] * e[j].im;
                B.re += sn[m] * o[j].re;
                B.im += sn[m] * o[j].im;
            }
            if constexpr (!INV) {
                x[k] = sub_i(A, B);
                x[RAD - k] = add_i(A, B);
            } else {
                x[k] = add_i(A, B);
                x[RAD - k] = sub_i(A, B);
            }
        }
    }
}

// One radix-RAD stage over `nlines` lines of length L.  Blocks of length Lq = RAD*m.
template <typename R, int RAD, bool INV>
__device__ __forceinline__ void fft_stage(cx<R>* __restrict__ buf, const LineMap lm, int nlines,
                                          int L, int Lq, const cx<R>* __restrict__ roots) {
    const int m = Lq / RAD;
    const int per_line = L / RAD;
    const int ntask = nlines * per_line;
    const int tws = L / Lq;
    R cs[RAD], sn[RAD];
    if constexpr (RAD >= 5) {
        const int cstr = L / RAD;
#pragma unroll
        for (int j = 0; j < RAD; ++j) {
            const cx<R> w = roots[j * cstr];   // e^{-2 pi i j / RAD}
            cs[j] = w.re;
            sn[j] = -w.im;
        }
    }
    const int st = m * lm.es;
    for (int task = threadIdx.x; task < ntask; task += blockDim.x) {
        const int line = task / per_line;
        const int j = task - line * per_line;
        const int b = j / m;
        const int np = j - b * m;
        cx<R>* p = buf + line_base(lm, line) + (b * Lq + np) * lm.es;
        cx<R> x[RAD];
#pragma unroll
        for (int i = 0; i < RAD; ++i) x[i] = p[i * st];
        if constexpr (!INV) {
            small_dft<R, RAD, false>(x, cs, sn);
#pragma unroll
            for (int k = 1; k < RAD; ++k) x[k] = cmul(x[k], roots[np * k * tws]);
        } else {
#pragma unroll
            for (int k = 1; k < RAD; ++k) x[k] = cmulc(x[k], roots[np * k * tws]);
            small_dft<R, RAD, true>(x, cs, sn);
        }
#pragma unroll
        for (int i = 0; i < RAD; ++i) p[i * st] = x[i];
    }
}

template <typename R, bool INV>
__device__ __forceinline__ void fft_dispatch(int rad, cx<R>* buf, const LineMap& lm, int nlines,
                                             int L, int Lq, const cx<R>* roots) {
    switch (rad) {
        case 2: fft_stage<R, 2, INV>(buf, lm, nlines, L, Lq, roots); break;
        case 3: fft_stage<R, 3, INV>(buf, lm, nlines, L, Lq, roots); break;
        case 4: fft_stage<R, 4, INV>(buf, lm, nlines, L, Lq, roots); break;
        case 5: fft_stage<R, 5, INV>(buf, lm, nlines, L, Lq, roots); break;
        case 7: fft_stage<R, 7, INV>(buf, lm, nlines, L, Lq, roots); break;
        case 11: fft_stage<R, 11, INV>(buf, lm, nlines, L, Lq, roots); break;
        case 13: fft_stage<R, 13, INV>(buf, lm, nlines, L, Lq, roots); break;
        case 17: fft_stage<R, 17, INV>(buf, lm, nlines, L, Lq, roots); break;
        default: break;   // make_plan admits no other radix
    }
}

// Transform `nlines` lines in place.  Ends with a barrier.
template <typename R, bool INV>
__device__ __forceinline__ void fft_lines(cx<R>* buf, const LineMap lm, int nlines, const FftPlan& plan,
                                          const cx<R>* roots) {
    if constexpr (!INV) {
        for (int q = 0; q < plan.nst; ++q) {
            fft_dispatch<R, false>(plan.radix[q], buf, lm, nlines, plan.L, plan.len[q], roots);
            __syncthreads();
        }
    } else {
        for (int q = plan.nst - 1; q >= 0; --q) {
            fft_dispatch<R, true>(plan.radix[q], buf, lm, nlines, plan.L, plan.len[q], roots);
            __syncthreads();
        }
    }
}

}  // namespace hub

// ============================================================================ compile-time L
// The same transform with L known at compile time: the radix plan, every index
// division and the r-point DFT coefficients become constants.
namespace hub {

struct CPlan {
    int nst;
    int radix[kMaxStages];
    int len[kMaxStages];
};

constexpr CPlan make_cplan(int L) {
    CPlan p{};
    const int rads[] = {4, 2, 3, 5, 7, 11, 13, 17};
    int rest = L;
    for (int r : rads)
        while (rest % r == 0 && p.nst < kMaxStages) {
            p.radix[p.nst++] = r;
            rest /= r;
        }
    int len = L;
    for (int q = 0; q < p.nst; ++q) {
        p.len[q] = len;
        len /= p.radix[q];
    }
    return p;
}

// cos and sin of pi/4 * a, 0 <= a <= 1, by Taylor series (compile time only)
constexpr void ct_sincos_octant(double a, double* s, double* c) {
    const double x = 0.78539816339744830962 * a;
    const double z = x * x;
    double ts = x, tc = 1.0, ss = x, cs = 1.0;
    for (int n = 1; n < 14; ++n) {
        ts *= -z / ((2.0 * n) * (2.0 * n + 1.0));
        tc *= -z / ((2.0 * n - 1.0) * (2.0 * n));
        ss += ts;
        cs += tc;
    }
    *s = ss;
    *c = cs;
}

// cos(2 pi m / r) and sin(2 pi m / r) by octant reduction with integer arithmetic.
constexpr void ct_sincos_frac(int m, int r, double* s, double* c) {
    m %= r;
    if (m < 0) m += r;
    const int o = (8 * m) / r;
    const int rem = 8 * m - o * r;
    double sa = 0, ca = 0, sb = 0, cb = 0;
    ct_sincos_octant((double)rem / r, &sa, &ca);            // a = (pi/4) rem/r
    ct_sincos_octant((double)(r - rem) / r, &sb, &cb);      // b = pi/4 - a
    switch (o) {
        case 0: *c = ca;  *s = sa;  break;
        case 1: *c = sb;  *s = cb;  break;
        case 2: *c = -sa; *s = ca;  break;
        case 3: *c = -cb; *s = sb;  break;
        case 4: *c = -ca; *s = -sa; break;
        case 5: *c = -sb; *s = -cb; break;
        case 6: *c = sa;  *s = -ca; break;
        default: *c = cb; *s = -sb; break;
    }
}

template <int RAD>
struct DftConst {
    double c[RAD];
    double s[RAD];
    constexpr DftConst() : c(), s() {
        for (int m = 0; m < RAD; ++m) ct_sincos_frac(m, RAD, &s[m], &c[m]);
    }
};

// r-point DFT with constant coefficients (same arithmetic as small_dft).
template <typename R, int RAD, bool INV>
__device__ __forceinline__ void small_dft_ct(cx<R>* x) {
    if constexpr (RAD <= 4) {
        small_dft<R, RAD, INV>(x, nullptr, nullptr);
    } else {
        constexpr DftConst<RAD> K{};
        constexpr int H = (RAD - 1) / 2;
        cx<R> e[H + 1], o[H + 1];
        const cx<R> x0 = x[0];
        cx<R> s0 = x0;
#pragma unroll
        for (int j = 1; j <= H; ++j) {
            e[j] = x[j] + x[RAD - j];
            o[j] = x[j] - x[RAD - j];
            s0 = s0 + e[j];
        }
        x[0] = s0;
#pragma unroll
        for (int k = 1; k <= H; ++k) {
            cx<R> A = x0;
            cx<R> B = {(R)0, (R)0};
#pragma unroll
            for (int j = 1; j <= H; ++j) {
                const int m = (j * k) % RAD;
                const R cm = (R)K.c[m], sm = (R)K.s[m];
                A.re = fmar(cm, e[j].re, A.re);
                A.im = fmar(cm, e[j].im, A.im);
                B.re = fmar(sm, o[j].re, B.re);
                B.im = fmar(sm, o[j].im, B.im);
            }
            if constexpr (!INV) {
                x[k] = sub_i(A, B);
                x[RAD - k] = add_i(A, B);
            } else {
                x[k] = add_i(A, B);
                x[RAD - k] = sub_i(A, B);
            }
        }
    }
}

// One odd r-point DFT (real-coefficient split, constant coefficients) shared by a lane pair:
// half q = 0 forms the real part of every output, q = 1 the imaginary part.  Forward, with
// e_j = x_j + x_{r-j}, o_j = x_j - x_{r-j}, A_k = x_0 + sum_j cos(2 pi jk/r) e_j and
// B_k = sum_j sin(2 pi jk/r) o_j:  X_k = A_k - i B_k and X_{r-k} = A_k + i B_k, so
//     Re X_k = Re A_k + Im B_k,  Im X_k = Im A_k - Re B_k   (signs of B swap for X_{r-k}
// and for the inverse).  Lane q needs the q-th component of A and the other one of B: the
// whole butterfly's arithmetic split in two halves with nothing computed twice but the pair
// sums.  y receives the lane's component of X_0 .. X_{r-1}.
template <typename R, int RAD, bool INV>
__device__ __forceinline__ void small_dft_pair(const cx<R>* x, int q, R* y) {
    constexpr DftConst<RAD> K{};
    constexpr int H = (RAD - 1) / 2;
    // values are formed first and selected after, so that no select picks between two
    // addresses of x (which would keep x in scratch memory instead of registers)
    R e[H + 1], o[H + 1];
    const cx<R> z = x[0];
    const R x0 = q ? z.im : z.re;
    R s0 = x0;
#pragma unroll
    for (int j = 1; j <= H; ++j) {
        const cx<R> a = x[j], b = x[RAD - j];
        const R sr = a.re + b.re, si = a.im + b.im, dr = a.re - b.re, di = a.im - b.im;
        e[j] = q ? si : sr;
        o[j] = q ? dr : di;
        s0 += e[j];
    }
    y[0] = s0;
    // forward: lane 0 adds B to X_k, lane 1 subtracts it; the inverse the other way round
    const R sg = ((q == 0) != INV) ? (R)1 : (R)-1;
#pragma unroll
    for (int k = 1; k <= H; ++k) {
        R A = x0, B = (R)0;
#pragma unroll
        for (int j = 1; j <= H; ++j) {
            const int m = (j * k) % RAD;
            A = fmar((R)K.c[m], e[j], A);
            B = fmar((R)K.s[m], o[j], B);
        }
        y[k] = fmar(sg, B, A);
        y[RAD - k] = fmar(-sg, B, A);
    }
}

// Stages whose radix is odd and >= 5 with no twiddle factors (the last forward stage, the
// first inverse one) and whose butterflies fill at most half of the workgroup's lanes share
// each butterfly between a lane pair (small_dft_pair): twice the tasks at about half the
// arithmetic each, so that the stage keeps two waves on a SIMD where it kept one (a single
// wave per SIMD cannot hide the latency of its dependent FMAs).  Stages with more butterflies
// than that already keep two waves per SIMD and keep one lane per butterfly.  Sharing every
// butterfly is FP32 only: in FP64 each lane of a pair reads twice the bytes through LDS and
// it measured no faster.  The hybrid form (only the surplus butterflies shared) runs in both
// precisions: the FP64 application at L = 51 measured 1.6 % faster with it.
constexpr bool kPairOddStages = true;

// Stage Q of the row (COLS = false) or column (COLS = true) transforms of NS
// sublattice tiles [NS][L][L] in LDS (a whole slice when NS = 2).  Row tasks run along a line (consecutive threads read
// consecutive positions); column tasks run across lines (consecutive threads read
// consecutive columns), so neither direction has strided LDS access within a wave.
template <typename R, int L, int Q, bool INV, bool COLS, int NT, int NS = 2>
__device__ __forceinline__ void ct_stage(cx<R>* __restrict__ buf, const cx<R>* __restrict__ roots) {
    constexpr CPlan P = make_cplan(L);
    constexpr int RAD = P.radix[Q], LQ = P.len[Q], M = LQ / RAD, PER = L / RAD;
    constexpr int NL = NS * L, NTASK = NL * PER, TWS = L / LQ;
    constexpr int ST = COLS ? M * L : M;
    // a twiddle-free odd stage whose butterflies fill more than half of the lanes but fewer
    // than all: the first half of the workgroup takes whole butterflies, the rest are shared
    // by lane pairs on the second half, so no SIMD runs two full-butterfly waves
    if constexpr (kPairOddStages && RAD >= 5 && M == 1 && 2 * NTASK > NT &&
                  NTASK < NT && 2 * (NTASK - NT / 2) <= NT / 2) {
        constexpr int NH = NT / 2, NR = NTASK - NH;
        auto base_of = [](int task) {
            if constexpr (COLS) {
                const int b = task / NL, line = task - b * NL;
                const int s = line >= L ? 1 : 0;
                return s * L * L + (line - s * L) + b * LQ * L;
            } else {
                const int line = task / PER, b = task - line * PER;
                return line * L + b * LQ;
            }
        };
        const int tid = threadIdx.x;
        if (tid < NH) {
            const int base = base_of(tid);
            cx<R> x[RAD];
#pragma unroll
            for (int i = 0; i < RAD; ++i) x[i] = buf[base + i * ST];
            small_dft_ct<R, RAD, INV>(x);
#pragma unroll
            for (int i = 0; i < RAD; ++i) buf[base + i * ST] = x[i];
        } else if (tid < NH + 2 * NR) {
            const int t2 = tid - NH, q = t2 & 1;
            const int base = base_of(NH + (t2 >> 1));
            cx<R> x[RAD];
#pragma unroll
            for (int i = 0; i < RAD; ++i) x[i] = buf[base + i * ST];
            R y[RAD];
            small_dft_pair<R, RAD, INV>(x, q, y);
            R* comp = reinterpret_cast<R*>(buf) + q;
#pragma unroll
            for (int i = 0; i < RAD; ++i) comp[2 * (base + i * ST)] = y[i];
        }
        return;
    }
    if constexpr (kPairOddStages && sizeof(R) == sizeof(float) && RAD >= 5 && M == 1 && 2 * NTASK <= NT) {
        for (int t2 = threadIdx.x; t2 < 2 * NTASK; t2 += NT) {
            const int task = t2 >> 1, q = t2 & 1;
            int base;
            if constexpr (COLS) {
                const int b = task / NL, line = task - b * NL;
                const int s = line >= L ? 1 : 0;
                base = s * L * L + (line - s * L) + b * LQ * L;
            } else {
                const int line = task / PER, b = task - line * PER;
                base = line * L + b * LQ;
            }
            cx<R> x[RAD];
#pragma unroll
            for (int i = 0; i < RAD; ++i) x[i] = buf[base + i * ST];
            R y[RAD];
            small_dft_pair<R, RAD, INV>(x, q, y);
            R* comp = reinterpret_cast<R*>(buf) + q;
#pragma unroll
            for (int i = 0; i < RAD; ++i) comp[2 * (base + i * ST)] = y[i];
        }
        return;
    }
    for (int task = threadIdx.x; task < NTASK; task += NT) {
        int line, j;
        if constexpr (COLS) {
            j = task / NL;
            line = task - j * NL;
        } else {
            line = task / PER;
            j = task - line * PER;
        }
        const int b = j / M, np = j - b * M;
        int base;
        if constexpr (COLS) {
            const int s = line >= L ? 1 : 0;
            base = s * L * L + (line - s * L) + (b * LQ + np) * L;
        } else {
            base = line * L + b * LQ + np;
        }
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

// Forward stages Q..QEND-1 (each followed by a barrier).
template <typename R, int L, int Q, int QEND, bool COLS, int NT, int NS = 2>
__device__ __forceinline__ void ct_forward(cx<R>* buf, const cx<R>* roots) {
    if constexpr (Q < QEND) {
        ct_stage<R, L, Q, false, COLS, NT, NS>(buf, roots);
        __syncthreads();
        ct_forward<R, L, Q + 1, QEND, COLS, NT, NS>(buf, roots);
    }
}

// Inverse stages Q, Q-1, ..., QLO (each followed by a barrier).
template <typename R, int L, int Q, int QLO, bool COLS, int NT, int NS = 2>
__device__ __forceinline__ void ct_inverse(cx<R>* buf, const cx<R>* roots) {
    if constexpr (Q >= QLO) {
        ct_stage<R, L, Q, true, COLS, NT, NS>(buf, roots);
        __syncthreads();
        ct_inverse<R, L, Q - 1, QLO, COLS, NT, NS>(buf, roots);
    }
}

}  // namespace hub
