// Ram-Lak ramp filter as a GEMM on the gfx950 matrix cores.
//
// The filtered projection Q = P * H of arXiv 2109.02174 (section "Computed
// tomography") with the Ram-Lak kernel is, for all rows at once,
//     Q[R][D] = P[R][D] x T,   T[m][n] = tap(n - m) = dt h(n - m),
// a dense contraction over the D input bins (linear convolution: the kernel
// spans every |n - m| <= D-1, so nothing is truncated).  T is symmetric and
// Toeplitz, so no T matrix exists in memory: each workgroup loads the slice of
// the 1D tap table its output columns need into LDS and feeds the B operand
// from there.
//
// Workgroup: 256 lanes = 4 waves in a 2 x 2 arrangement, 64 x 64 outputs, each
// wave one 32 x 32 MFMA accumulator block (FP32 accumulate).
//   FP32:       v_mfma_f32_32x32x2_f32, K-step 32 staged through LDS.
//   BF16/FP16:  v_mfma_f32_32x32x16_{bf16,f16}; A is rounded to 16 bits (RNE)
//               as it is staged; the tap table is kept as eight copies shifted by
//               one element so every 8-tap B fragment is one aligned 16-byte read.
#include <hip/hip_bf16.h>
#include <hip/hip_fp16.h>

#include "fbp_internal.hpp"

namespace fbp {

namespace {

typedef float v16f __attribute__((ext_vector_type(16)));
typedef __bf16 v8bf __attribute__((ext_vector_type(8)));
typedef _Float16 v8h __attribute__((ext_vector_type(8)));
typedef unsigned short v8u16 __attribute__((ext_vector_type(8)));

constexpr int kBK32 = 32;   // K-step of the FP32 path
constexpr int kBK16 = 64;   // K-step of the 16-bit paths
constexpr int kAStride32 = kBK32 + 1;   // LDS row stride (floats), odd: no bank conflicts
constexpr int kAStride16 = kBK16 + 8;   // LDS row stride (16-bit), 16-byte aligned rows

__device__ __forceinline__ unsigned short to_bf16_rne(float x) {
    unsigned int u = __float_as_uint(x);
    u += 0x7FFFu + ((u >> 16) & 1u);
    return (unsigned short)(u >> 16);
}

__device__ __forceinline__ unsigned short to_f16_rne(float x) {
    _Float16 h = (_Float16)x;
    return __builtin_bit_cast(unsigned short, h);
}

// Output element (m, n) of accumulator register i of a 32x32 MFMA block for lane l:
// n = l % 32, m = 8 (i / 4) + 4 (l / 32) + i % 4.
__device__ __forceinline__ void store_block(const v16f& acc, float* __restrict__ q, int R, int D,
                                            int m0, int n0, float s) {
    const int l = threadIdx.x & 63;
    const int n = n0 + (l & 31);
    if (n >= D) return;
#pragma unroll
    for (int i = 0; i < 16; ++i) {
        const int m = m0 + 8 * (i >> 2) + 4 * (l >> 5) + (i & 3);
        if (m < R) q[(size_t)m * D + n] = acc[i] * s;
    }
}

// ---------------------------------------------------------------- FP32 operands

__device__ __forceinline__ void gemm_tile_f32(const GemmJob& job, int mt, int nt, float* smem) {
    float* As = smem;                                  // [64][kAStride32]
    float* Bt = smem + kGemmBM * kAStride32;           // taps d = n0 - Dp + 1 + x
    const int t = threadIdx.x;
    const int w = t >> 6, l = t & 63;
    const int wm = w >> 1, wn = w & 1;
    const int m0 = mt * kGemmBM, n0 = nt * kGemmBN;
    const int R = job.R, D = job.D, Dp = job.Dp;
    const float* __restrict__ taps = static_cast<const float*>(job.taps);
    const float* __restrict__ P = job.p;

    __syncthreads();  // LDS reuse across tiles of a persistent workgroup
    // taps for d in [n0 - Dp + 1, n0 + 63]: table index d + Dp in [n0 + 1, n0 + Dp + 63]
    const int n_taps = Dp + kGemmBN - 1;
    for (int x = t; x < n_taps; x += kBpThreads) Bt[x] = taps[n0 + 1 + x];

    v16f acc = {};
    const int col_l = wn * 32 + (l & 31);              // output column within the tile
    const int row_l = wm * 32 + (l & 31);              // A row within the tile
    for (int k0 = 0; k0 < D; k0 += kBK32) {
        __syncthreads();
        for (int e = t; e < kGemmBM * kBK32; e += kBpThreads) {
            const int row = e / kBK32, col = e % kBK32;
            const int m = m0 + row, k = k0 + col;
            As[row * kAStride32 + col] = (m < R && k < D) ? P[(size_t)m * D + k] : 0.0f;
        }
        __syncthreads();
#pragma unroll
        for (int ks = 0; ks < kBK32; ks += 2) {
            const int kk = ks + (l >> 5);
            const float a = As[row_l * kAStride32 + kk];
            // tap(n - k) with n = n0 + col_l, k = k0 + kk: Bt index n - k - (n0 - Dp + 1)
            const float b = Bt[col_l + Dp - 1 - (k0 + kk)];
            acc = __builtin_amdgcn_mfma_f32_32x32x2f32(a, b, acc, 0, 0, 0);
        }
    }
    store_block(acc, job.q, R, D, m0 + wm * 32, n0 + wn * 32, job.out_scale);
}

// ---------------------------------------------------------------- 16-bit operands

template <int PREC>
__device__ __forceinline__ void gemm_tile_16(const GemmJob& job, int mt, int nt, unsigned short* smem) {
    // LDS: A [64][kAStride16] 16-bit, then 8 shifted copies of the tap slice.
    unsigned short* As = smem;
    unsigned short* Tc = smem + kGemmBM * kAStride16;
    const int t = threadIdx.x;
    const int w = t >> 6, l = t & 63;
    const int wm = w >> 1, wn = w & 1;
    const int m0 = mt * kGemmBM, n0 = nt * kGemmBN;
    const int R = job.R, D = job.D, Dp = job.Dp;
    const unsigned short* __restrict__ taps = static_cast<const unsigned short*>(job.taps);
    const float* __restrict__ P = job.p;

    // B fragment of lane l at K-step base kb: taps at d = k - n for
    // k = kb + 8 (l / 32) + i, i = 0..7, n = n0 + wn*32 + l%32 (tap(n-k) = tap(k-n)).
    // d ranges over [-(n0 + 63), Dp - 1 - n0 + 8]; slice origin d_lo = -(n0 + 64).
    const int d_lo = -(n0 + kGemmBN);
    const int span = Dp + kGemmBN + 16;                // covers d_lo .. Dp - n0 + 15
    const int cstride = (span + 7 + 7) & ~7;           // per-copy length, multiple of 8

    __syncthreads();
    for (int x = t; x < 8 * cstride; x += kBpThreads) {
        const int c = x / cstride, y = x - c * cstride;
        const int d = d_lo + y + c;                    // copy c holds slice[y + c]
        const int idx = d + Dp;
        Tc[x] = (idx >= 0 && idx < 2 * Dp) ? taps[idx] : (unsigned short)0;
    }

    v16f acc = {};
    const int row_l = wm * 32 + (l & 31);
    const int n_l = n0 + wn * 32 + (l & 31);
    const int kq = 8 * (l >> 5);
    for (int k0 = 0; k0 < D; k0 += kBK16) {
        __syncthreads();
        // stage A: 64 rows x 64 k, four consecutive k per lane-step
        for (int e = t; e < kGemmBM * (kBK16 / 4); e += kBpThreads) {
            const int row = e / (kBK16 / 4), c4 = (e % (kBK16 / 4)) * 4;
            const int m = m0 + row;
            unsigned short h[4];
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                const int k = k0 + c4 + i;
                const float v = (m < R && k < D) ? P[(size_t)m * D + k] : 0.0f;
                h[i] = (PREC == kBF16) ? to_bf16_rne(v) : to_f16_rne(v);
            }
            unsigned int* dst = reinterpret_cast<unsigned int*>(As + row * kAStride16 + c4);
            dst[0] = (unsigned int)h[0] | ((unsigned int)h[1] << 16);
            dst[1] = (unsigned int)h[2] | ((unsigned int)h[3] << 16);
        }
        __syncthreads();
#pragma unroll
        for (int ks = 0; ks < kBK16; ks += 16) {
            const v8u16 av = *reinterpret_cast<const v8u16*>(As + row_l * kAStride16 + ks + kq);
            const int y = (k0 + ks + kq) - n_l - d_lo;     // slice index of the first tap
            const int c = y & 7;
            const v8u16 bv = *reinterpret_cast<const v8u16*>(Tc + c * cstride + (y - c));
            if constexpr (PREC == kBF16) {
                acc = __builtin_amdgcn_mfma_f32_32x32x16_bf16(__builtin_bit_cast(v8bf, av),
                                                              __builtin_bit_cast(v8bf, bv), acc, 0, 0, 0);
            } else {
                acc = __builtin_amdgcn_mfma_f32_32x32x16_f16(__builtin_bit_cast(v8h, av),
                                                             __builtin_bit_cast(v8h, bv), acc, 0, 0, 0);
            }
        }
    }
    store_block(acc, job.q, R, D, m0 + wm * 32, n0 + wn * 32, job.out_scale);
}

template <int PREC>
__device__ __forceinline__ void gemm_tile(const GemmJob& job, int mt, int nt, void* smem) {
    if constexpr (PREC == kFP32)
        gemm_tile_f32(job, mt, nt, static_cast<float*>(smem));
    else
        gemm_tile_16<PREC>(job, mt, nt, static_cast<unsigned short*>(smem));
}

template <int PREC>
__global__ __launch_bounds__(kBpThreads) void gemm_grid_kernel(GemmJob job) {
    extern __shared__ float4 smem4[];
    const int tiles_m = (job.R + kGemmBM - 1) / kGemmBM;
    // blockIdx.x: output tile index, row tiles fastest so neighbours share tap slices
    const int b = blockIdx.x;
    const int nt = b / tiles_m, mt = b - nt * tiles_m;
    gemm_tile<PREC>(job, mt, nt, smem4);
}

template <int PREC>
__global__ __launch_bounds__(kBpThreads) void gemm_list_kernel(const GemmListArgs* __restrict__ args) {
    extern __shared__ float4 smem4[];
    const GemmListArgs a = *args;
    const int n_jobs = a.counts[0];
    if (n_jobs <= 0) return;
    const int total = a.tile_prefix[n_jobs];
    for (int it = blockIdx.x; it < total; it += gridDim.x) {
        int lo = 0, hi = n_jobs - 1;
        while (lo < hi) {
            const int mid = (lo + hi + 1) >> 1;
            if (a.tile_prefix[mid] <= it) lo = mid; else hi = mid - 1;
        }
        const GemmJob job = a.jobs[lo];
        const int tt = it - a.tile_prefix[lo];
        const int tiles_m = (job.R + kGemmBM - 1) / kGemmBM;
        const int nt = tt / tiles_m, mt = tt - nt * tiles_m;
        gemm_tile<PREC>(job, mt, nt, smem4);
    }
}

template <int PREC>
int occ(int lds) {
    int n = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, gemm_list_kernel<PREC>, kBpThreads, lds) !=
        hipSuccess)
        return 1;
    return n > 0 ? n : 1;
}

}  // namespace

int gemm_lds_bytes(int prec, int Dp) {
    if (prec == kFP32) return (kGemmBM * kAStride32 + Dp + kGemmBN) * 4;
    const int span = Dp + kGemmBN + 16;
    const int cstride = (span + 7 + 7) & ~7;
    return (kGemmBM * kAStride16 + 8 * cstride) * 2;
}

hipError_t launch_gemm_grid(int prec, const GemmJob& job, hipStream_t stream) {
    const int tiles_m = (job.R + kGemmBM - 1) / kGemmBM;
    const unsigned grid = (unsigned)(tiles_m * job.tiles_n);
    const size_t lds = (size_t)gemm_lds_bytes(prec, job.Dp);
    switch (prec) {
        case kFP32: hipLaunchKernelGGL(gemm_grid_kernel<kFP32>, dim3(grid), dim3(kBpThreads), lds, stream, job); break;
        case kBF16: hipLaunchKernelGGL(gemm_grid_kernel<kBF16>, dim3(grid), dim3(kBpThreads), lds, stream, job); break;
        case kFP16: hipLaunchKernelGGL(gemm_grid_kernel<kFP16>, dim3(grid), dim3(kBpThreads), lds, stream, job); break;
        default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

hipError_t launch_gemm_list(int prec, const GemmListArgs* a, int grid, size_t lds, hipStream_t stream) {
    switch (prec) {
        case kFP32: hipLaunchKernelGGL(gemm_list_kernel<kFP32>, dim3(grid), dim3(kBpThreads), lds, stream, a); break;
        case kBF16: hipLaunchKernelGGL(gemm_list_kernel<kBF16>, dim3(grid), dim3(kBpThreads), lds, stream, a); break;
        case kFP16: hipLaunchKernelGGL(gemm_list_kernel<kFP16>, dim3(grid), dim3(kBpThreads), lds, stream, a); break;
        default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

int gemm_occupancy(int prec, size_t lds_bytes) {
    const int lds = (int)lds_bytes;
    switch (prec) {
        case kFP32: return occ<kFP32>(lds);
        case kBF16: return occ<kBF16>(lds);
        case kFP16: return occ<kFP16>(lds);
        default: return 1;
    }
}

}  // namespace fbp
