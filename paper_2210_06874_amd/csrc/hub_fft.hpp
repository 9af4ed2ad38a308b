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
__device__ __forceinline__ cx<R> mk(R a, R b) { return cx<R>{a, b}; }
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
