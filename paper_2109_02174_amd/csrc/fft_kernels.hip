// FFT filter path for gfx950: the ramp filter of every projection row as a
// circular convolution of the zero-padded row, computed with one complex FFT per
// pair of rows in LDS.
//
// The filter (the convolution Q = P * H, arXiv 2109.02174, section "Computed
// tomography") is linear with taps t(d) = dt h(d) for |d| <= D-1.  With the row
// zero-padded to L >= 2D - 1 points, the circular convolution with the taps
// wrapped modulo L equals the linear one on the D output bins (no output sees a
// wrapped tap).  The taps are even in d, so their L-point DFT H is real and even;
// two real rows a, b packed as z = a + i b therefore give
//     IFFT(FFT(z) H) = (a * t) + i (b * t)
// and the two filtered rows are the real and imaginary parts.  One workgroup per
// row pair: load (zero padding), forward FFT, multiply by H (which also carries
// 1/L and the output scale), inverse FFT, store the first D points.
//
// The FFT is a Stockham autosort FFT in LDS (natural order in and out, one
// buffer: every pass reads all of its inputs into registers before a barrier
// and writes all of its outputs after it): up to L = 2^11 one radix-2 pass when
// log2 L is odd, then radix-4 passes; longer transforms use radix-8 passes (an
// 8-point DFT as two 4-point DFTs of the sums and twiddled differences) after one
// radix-2 or radix-4 pass, e.g. 5 passes instead of 7 at L = 2^13.  Twiddles come
// from a table e^{-2 pi i m / L} made in
// FP64 on the host; up to L = 4096 its first quarter is copied to LDS and the
// rest follows from W^(m + jL/4) = (-i)^j W^m.
#include "fbp_internal.hpp"

namespace fbp {

namespace {

// threads per workgroup: one radix-4 butterfly per thread and pass (64 to 1024)
constexpr int fft_threads(int log2L) {
    return log2L <= 8 ? 64 : (log2L >= 12 ? 1024 : (1 << (log2L - 2)));
}

__device__ __forceinline__ float2 cmul(float2 a, float2 b) {
    return make_float2(fmaf(a.x, b.x, -a.y * b.y), fmaf(a.x, b.y, a.y * b.x));
}

template <int LOG2L>
__global__ __launch_bounds__(fft_threads(LOG2L)) void fft_filter_kernel(FftJob job) {
    constexpr int kFftThreads = fft_threads(LOG2L);
    constexpr int L = 1 << LOG2L;
    constexpr int Q4 = L / 4;                                   // radix-4 butterflies per pass
    constexpr int NB4 = Q4 >= kFftThreads ? Q4 / kFftThreads : 1;
    constexpr int H2 = L / 2;                                   // radix-2 butterflies
    constexpr int NB2 = H2 >= kFftThreads ? H2 / kFftThreads : 1;
    constexpr int Q8 = L / 8;                                   // radix-8 butterflies per pass
    constexpr int NB8 = Q8 >= kFftThreads ? Q8 / kFftThreads : 1;
    // twiddles from an LDS copy of the first quarter of the table (L <= 4096):
    // W^(m + jL/4) = (-i)^j W^m
    constexpr bool kLdsTw = LOG2L >= 2 && LOG2L <= 12;
    constexpr int QT = kLdsTw ? L / 4 : 1;
    __shared__ float2 buf[L];
    __shared__ float2 qtw[QT];
    const int t = threadIdx.x;
    const int D = job.D;
    const int ra = 2 * blockIdx.x, rb = ra + 1;
    const bool has_b = rb < job.R;
    const float* __restrict__ pa = job.p + (size_t)ra * D;
    const float* __restrict__ pb = job.p + (size_t)(has_b ? rb : ra) * D;
    const float2* __restrict__ tw = job.tw;

    for (int n = t; n < L; n += kFftThreads) {                  // column weights (if any) applied on load
        const float w = (job.colw && n < D) ? job.colw[n] : 1.0f;
        const float a = n < D ? pa[n] * w : 0.0f;
        const float b = (has_b && n < D) ? pb[n] * w : 0.0f;
        buf[n] = make_float2(a, b);
    }
    if constexpr (kLdsTw) {
        for (int m = t; m < QT; m += kFftThreads) qtw[m] = tw[m];
    }
    __syncthreads();
    auto twiddle = [&](int m) -> float2 {                       // W^m, m < L
        if constexpr (kLdsTw) {
            const float2 w = qtw[m & (QT - 1)];
            switch (m >> (LOG2L - 2)) {
                case 0: return w;
                case 1: return make_float2(w.y, -w.x);
                case 2: return make_float2(-w.x, -w.y);
                default: return make_float2(-w.y, w.x);
            }
        } else {
            return tw[m];
        }
    };
    auto add = [](float2 a, float2 b) { return make_float2(a.x + b.x, a.y + b.y); };
    auto sub = [](float2 a, float2 b) { return make_float2(a.x - b.x, a.y - b.y); };
    // 4-point DFT (forward: e^{-2 pi i r s / 4}; inverse: its conjugate)
    auto dft4 = [&](float2 x0, float2 x1, float2 x2, float2 x3, bool inverse, float2* y, int ys) {
        const float2 t0 = add(x0, x2), t1 = sub(x0, x2), t2 = add(x1, x3), d = sub(x1, x3);
        const float2 t3 = inverse ? make_float2(-d.y, d.x) : make_float2(d.y, -d.x);
        y[0] = add(t0, t2);
        y[ys] = add(t1, t3);
        y[2 * ys] = sub(t0, t2);
        y[3 * ys] = sub(t1, t3);
    };

    // pass schedule: up to L = 2^11 one radix-2 pass when log2 L is odd, then radix-4
    // passes; from 2^12 on one radix-2 (log2 L = 1 mod 3) or radix-4 (= 2 mod 3)
    // pass, then radix-8 passes (fewer barriers; below 2^12 half the threads of a
    // radix-8 pass would idle and it measured slower)
    constexpr bool R8 = LOG2L >= 12;
    constexpr bool kFirst2 = R8 ? (LOG2L % 3 == 1) : ((LOG2L & 1) != 0);
    constexpr int kN4 = R8 ? (LOG2L % 3 == 2 ? 1 : 0) : LOG2L / 2;

    auto fft = [&](bool inverse) {
        int Ns = 1;
        if constexpr (kFirst2) {                                // one radix-2 pass (k = 0: no twiddle)
            float2 v[NB2][2];
#pragma unroll
            for (int q = 0; q < NB2; ++q) {
                const int j = t + q * kFftThreads;
                if (j < H2) {
                    v[q][0] = buf[j];
                    v[q][1] = buf[j + H2];
                }
            }
            __syncthreads();
#pragma unroll
            for (int q = 0; q < NB2; ++q) {
                const int j = t + q * kFftThreads;
                if (j < H2) {
                    buf[2 * j] = make_float2(v[q][0].x + v[q][1].x, v[q][0].y + v[q][1].y);
                    buf[2 * j + 1] = make_float2(v[q][0].x - v[q][1].x, v[q][0].y - v[q][1].y);
                }
            }
            __syncthreads();
            Ns = 2;
        }
        for (int p4 = 0; p4 < kN4; ++p4, Ns *= 4) {             // radix 4
            float2 v[NB4][4];
#pragma unroll
            for (int q = 0; q < NB4; ++q) {
                const int j = t + q * kFftThreads;
                if (j < Q4) {
#pragma unroll
                    for (int r = 0; r < 4; ++r) v[q][r] = buf[j + r * Q4];
                }
            }
            __syncthreads();
#pragma unroll
            for (int q = 0; q < NB4; ++q) {
                const int j = t + q * kFftThreads;
                if (j < Q4) {
                    const int k = j & (Ns - 1);
                    const int step = k * (L / (4 * Ns));        // twiddle W^(r k L / (4 Ns)), index < 3L/4
                    if (step != 0) {
#pragma unroll
                        for (int r = 1; r < 4; ++r) {
                            float2 w = twiddle(r * step);
                            if (inverse) w.y = -w.y;
                            v[q][r] = cmul(v[q][r], w);
                        }
                    }
                    float2 y[4];
                    dft4(v[q][0], v[q][1], v[q][2], v[q][3], inverse, y, 1);
                    const int o = (j - k) * 4 + k;
#pragma unroll
                    for (int r = 0; r < 4; ++r) buf[o + r * Ns] = y[r];
                }
            }
            __syncthreads();
        }
        if constexpr (!R8) return;
        for (; R8 && Ns < L; Ns *= 8) {                         // radix 8
            float2 v[NB8][8];
#pragma unroll
            for (int q = 0; q < NB8; ++q) {
                const int j = t + q * kFftThreads;
                if (j < Q8) {
#pragma unroll
                    for (int r = 0; r < 8; ++r) v[q][r] = buf[j + r * Q8];
                }
            }
            __syncthreads();
#pragma unroll
            for (int q = 0; q < NB8; ++q) {
                const int j = t + q * kFftThreads;
                if (j < Q8) {
                    const int k = j & (Ns - 1);
                    const int step = k * (L / (8 * Ns));        // twiddle W^(r k L / (8 Ns)), index < 7L/8
                    if (step != 0) {
#pragma unroll
                        for (int r = 1; r < 8; ++r) {
                            float2 w = twiddle(r * step);
                            if (inverse) w.y = -w.y;
                            v[q][r] = cmul(v[q][r], w);
                        }
                    }
                    // 8-point DFT: two 4-point DFTs of the sums and of the differences
                    // times e^{-+2 pi i r / 8} (even and odd outputs)
                    constexpr float c = 0.70710678118654752f;
                    const float2 a0 = add(v[q][0], v[q][4]), a1 = add(v[q][1], v[q][5]);
                    const float2 a2 = add(v[q][2], v[q][6]), a3 = add(v[q][3], v[q][7]);
                    const float2 b0 = sub(v[q][0], v[q][4]), d1 = sub(v[q][1], v[q][5]);
                    const float2 d2 = sub(v[q][2], v[q][6]), d3 = sub(v[q][3], v[q][7]);
                    const float2 b1 = inverse ? make_float2(c * (d1.x - d1.y), c * (d1.x + d1.y))
                                              : make_float2(c * (d1.x + d1.y), c * (d1.y - d1.x));
                    const float2 b2 = inverse ? make_float2(-d2.y, d2.x) : make_float2(d2.y, -d2.x);
                    const float2 b3 = inverse ? make_float2(-c * (d3.x + d3.y), c * (d3.x - d3.y))
                                              : make_float2(c * (d3.y - d3.x), -c * (d3.x + d3.y));
                    float2 y[8];
                    dft4(a0, a1, a2, a3, inverse, y, 2);
                    dft4(b0, b1, b2, b3, inverse, y + 1, 2);
                    const int o = (j - k) * 8 + k;
#pragma unroll
                    for (int r = 0; r < 8; ++r) buf[o + r * Ns] = y[r];
                }
            }
            __syncthreads();
        }
    };

    fft(false);
    for (int n = t; n < L; n += kFftThreads) {
        const float h = job.H[n];
        const float2 z = buf[n];
        buf[n] = make_float2(z.x * h, z.y * h);
    }
    __syncthreads();
    fft(true);

    float* __restrict__ qa = job.q + (size_t)ra * D;
    float* __restrict__ qb = job.q + (size_t)rb * D;
    for (int n = t; n < D; n += kFftThreads) {
        const float2 z = buf[n];
        qa[n] = z.x;
        if (has_b) qb[n] = z.y;
    }
}

template <int LOG2L>
hipError_t launch_fft_l(const FftJob& job, unsigned blocks, hipStream_t stream) {
    return launch_kernel(fft_filter_kernel<LOG2L>, dim3(blocks), dim3(fft_threads(LOG2L)), 0, stream, job);
}

}  // namespace

int fft_length_log2(int D) {
    int lg = 0;
    while ((1 << lg) < 2 * D - 1) ++lg;
    return lg;
}

hipError_t launch_fft_filter(const FftJob& job, hipStream_t stream) {
    if (job.R <= 0) return hipSuccess;
    if (job.log2L < 0 || job.log2L > kFftMaxLog2 || (1 << job.log2L) < 2 * job.D - 1) return hipErrorInvalidValue;
    const unsigned blocks = (unsigned)((job.R + 1) / 2);
    switch (job.log2L) {
        case 0: return launch_fft_l<0>(job, blocks, stream);
        case 1: return launch_fft_l<1>(job, blocks, stream);
        case 2: return launch_fft_l<2>(job, blocks, stream);
        case 3: return launch_fft_l<3>(job, blocks, stream);
        case 4: return launch_fft_l<4>(job, blocks, stream);
        case 5: return launch_fft_l<5>(job, blocks, stream);
        case 6: return launch_fft_l<6>(job, blocks, stream);
        case 7: return launch_fft_l<7>(job, blocks, stream);
        case 8: return launch_fft_l<8>(job, blocks, stream);
        case 9: return launch_fft_l<9>(job, blocks, stream);
        case 10: return launch_fft_l<10>(job, blocks, stream);
        case 11: return launch_fft_l<11>(job, blocks, stream);
        case 12: return launch_fft_l<12>(job, blocks, stream);
        case 13: return launch_fft_l<13>(job, blocks, stream);
        default: return hipErrorInvalidValue;
    }
}

}  // namespace fbp
