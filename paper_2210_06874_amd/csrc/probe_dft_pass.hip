// Measurement probe, not part of the hub C ABI: one row pass of the L-point DFT over
// every row of `ntiles` tiles [L][L] of complex64 (interleaved re, im), from HBM back to
// HBM, one workgroup per tile (a tile is one sublattice of one time slice, so L = 51 with
// 2 * N_t tiles is one pass of the per-slice transform at the precision workload).  Two forms
// of the same pass:
//   * the library's own FFT stages (the compile-time mixed-radix row transform of the
//     fused operator kernels, on the VALU); output in digit-reversed order, as there;
//   * the dense DFT as a real GEMM on the FP32 matrix cores: [Re y | Im y] = [Re x | Im x] G
//     with G = [[C, -S], [S, C]], C and S the cosine and sine of 2 pi k n / L, K = 2L padded
//     to 104 and N = 2L to 112, v_mfma_f32_16x16x4f32 tiles; output in natural order.
// The question it answers is whether the transform belongs on MFMA (the per-slice DFT is a
// dense L x L contraction): bench.py --probe-dft times both, and the matrix cores' own FP32 and
// FP64 rates beside them.
#include <hip/hip_runtime.h>

#include "hub_fft.hpp"

namespace {

using hub::cx;

template <int L, int NT>
__global__ void __launch_bounds__(NT) k_probe_fft_rows(const cx<float>* __restrict__ x, cx<float>* __restrict__ y,
                                                       const cx<float>* __restrict__ roots_g) {
    __shared__ cx<float> buf[L * L];
    __shared__ cx<float> roots[L];
    const long long base = (long long)blockIdx.x * L * L;
    for (int i = threadIdx.x; i < L; i += NT) roots[i] = roots_g[i];
    for (int i = threadIdx.x; i < L * L; i += NT) buf[i] = x[base + i];
    __syncthreads();
    constexpr hub::CPlan P = hub::make_cplan(L);
    hub::ct_forward<float, L, 0, P.nst, false, NT, 1>(buf, roots);
    for (int i = threadIdx.x; i < L * L; i += NT) y[base + i] = buf[i];
}

constexpr int kKP = 104;   // padded K: the 2L real inputs of a row
constexpr int kNP = 112;   // padded N: the 2L real outputs
typedef float v4f __attribute__((ext_vector_type(4)));

// Four waves, wave w multiplies rows [16 w, 16 w + 16) of the tile by G.  For the 16 x 16 x 4
// FP32 MFMA lane l supplies A[l % 16][l / 16] and B[l / 16][l % 16] of a K step and holds
// D[4 (l / 16) + r][l % 16], r = 0..3, of each 16 x 16 output tile.
template <int L>
__global__ void __launch_bounds__(256) k_probe_mfma_rows(const float* __restrict__ x, float* __restrict__ y,
                                                         const float* __restrict__ g) {
    static_assert(2 * L <= kKP && 2 * L <= kNP && L <= 64, "one tile row per MFMA row, four waves");
    __shared__ float xs[2 * L * L];     // the tile, interleaved complex
    __shared__ float gs[kKP * kNP];
    const long long base = (long long)blockIdx.x * 2 * L * L;
    for (int i = threadIdx.x; i < kKP * kNP / 4; i += 256)
        reinterpret_cast<float4*>(gs)[i] = reinterpret_cast<const float4*>(g)[i];
    for (int i = threadIdx.x; i < 2 * L * L; i += 256) xs[i] = x[base + i];
    __syncthreads();
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    const int row = 16 * w + (lane & 15), kq = lane >> 4;
    v4f acc[kNP / 16];
#pragma unroll
    for (int c = 0; c < kNP / 16; ++c) acc[c] = v4f{0.f, 0.f, 0.f, 0.f};
    for (int s = 0; s < kKP / 4; ++s) {
        const int k = 4 * s + kq;
        // A[row][k]: Re x[row][k] for k < L, Im x[row][k - L] for L <= k < 2L, 0 beyond
        float a = 0.f;
        if (row < L && k < 2 * L) a = xs[row * 2 * L + (k < L ? 2 * k : 2 * (k - L) + 1)];
#pragma unroll
        for (int c = 0; c < kNP / 16; ++c)
            acc[c] = __builtin_amdgcn_mfma_f32_16x16x4f32(a, gs[k * kNP + 16 * c + (lane & 15)], acc[c], 0, 0, 0);
    }
    __syncthreads();   // every wave has read its A operands: the tile's LDS takes the output
#pragma unroll
    for (int c = 0; c < kNP / 16; ++c) {
        const int n = 16 * c + (lane & 15);
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            const int orow = 16 * w + 4 * kq + r;
            if (orow < L && n < 2 * L) xs[orow * 2 * L + (n < L ? 2 * n : 2 * (n - L) + 1)] = acc[c][r];
        }
    }
    __syncthreads();
    for (int i = threadIdx.x; i < 2 * L * L; i += 256) y[base + i] = xs[i];
}

// The matrix cores' own rate: every wave issues `iters` rounds of eight independent 16 x 16 x 4
// MFMAs (FP32 or FP64) on register operands, with nothing else in the loop; the sums are stored
// so that the work stays live.
template <typename T>
__global__ void __launch_bounds__(256) k_probe_mfma_peak(T* __restrict__ out, int iters) {
    typedef T v4 __attribute__((ext_vector_type(4)));
    v4 acc[8];
#pragma unroll
    for (int k = 0; k < 8; ++k) acc[k] = v4{0, 0, 0, 0};
    const T a = (T)(threadIdx.x & 63) * (T)1e-3, b = (T)(blockIdx.x & 63) * (T)1e-3;
    for (int i = 0; i < iters; ++i) {
#pragma unroll
        for (int k = 0; k < 8; ++k) {
            if constexpr (sizeof(T) == sizeof(float))
                acc[k] = __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, acc[k], 0, 0, 0);
            else
                acc[k] = __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, acc[k], 0, 0, 0);
        }
    }
    T s = 0;
#pragma unroll
    for (int k = 0; k < 8; ++k) s += acc[k][0] + acc[k][1] + acc[k][2] + acc[k][3];
    out[(long long)blockIdx.x * 256 + threadIdx.x] = s;
}

}  // namespace

extern "C" {

// The FP32 (fp64 = 0) or FP64 (fp64 = 1) MFMA rate: nblocks workgroups of four waves, each wave
// issuing iters * 8 MFMAs of 16 x 16 x 4 (2048 flops each).  out: device, nblocks * 256 floats
// (or doubles).  Returns 0, or the HIP error of the launch.
int probe_mfma_peak(void* out, int nblocks, int iters, int fp64, void* stream) {
    if (nblocks <= 0 || iters <= 0) return 0;
    if (fp64)
        hipLaunchKernelGGL(k_probe_mfma_peak<double>, dim3(nblocks), dim3(256), 0, (hipStream_t)stream,
                           static_cast<double*>(out), iters);
    else
        hipLaunchKernelGGL(k_probe_mfma_peak<float>, dim3(nblocks), dim3(256), 0, (hipStream_t)stream,
                           static_cast<float*>(out), iters);
    return (int)hipGetLastError();
}


// Row pass of the 51-point DFT by the library's FFT stages.  x, y: device, ntiles * 51 * 51
// complex64 each (distinct buffers); roots: device, 51 complex64, roots[m] = e^{-2 pi i m / 51};
// stream: a hipStream_t.  Returns 0, or the HIP error of the launch.
int probe_dft_rows_fft51(const float* x, float* y, const float* roots, int ntiles, void* stream) {
    if (ntiles <= 0) return 0;
    hipLaunchKernelGGL((k_probe_fft_rows<51, 512>), dim3(ntiles), dim3(512), 0, (hipStream_t)stream,
                       reinterpret_cast<const cx<float>*>(x), reinterpret_cast<cx<float>*>(y),
                       reinterpret_cast<const cx<float>*>(roots));
    return (int)hipGetLastError();
}

// Row pass of the 51-point DFT as FP32 MFMA GEMMs.  x, y as above; g: device, 104 x 112 floats,
// row k, column n: the real DFT matrix [[C, -S], [S, C]] (C, S = cos, sin of 2 pi k n / 51),
// zero in the padding.  Returns 0, or the HIP error of the launch.
int probe_dft_rows_mfma51(const float* x, float* y, const float* g, int ntiles, void* stream) {
    if (ntiles <= 0) return 0;
    hipLaunchKernelGGL((k_probe_mfma_rows<51>), dim3(ntiles), dim3(256), 0, (hipStream_t)stream, x, y, g);
    return (int)hipGetLastError();
}

}  // extern "C"
