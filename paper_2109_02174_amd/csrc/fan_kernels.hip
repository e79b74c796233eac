// Fan-beam kernels for gfx950: cosine pre-weighting of the views and the
// distance-weighted backprojection (flat detector through the rotation centre).
//
// Geometry (the second geometry of the filtered-backprojection method of arXiv
// 2109.02174, section "Computed tomography"; fan-beam weights of Kak & Slaney
// 1988, ch. 3): view k has its source at R (cos b_k, sin b_k); bin j sits at
// s_j = (j - (D-1)/2) ds on the detector line through the centre along
// (-sin b_k, cos b_k).  A pixel X = (x, y) is at depth L = R - (x cos b + y sin b)
// and is seen at s = R (X . e) / L.  The reconstruction is
//     views * R / sqrt(R^2 + s^2)  ->  filter with half the kernel  ->
//     img(X) = (2 pi / K) sum_k (R/L)^2 Q~_k(s / ds + (D-1)/2)
// (linear interpolation, zero beyond the detector).
//
// The backprojector keeps the parallel-beam design: a workgroup owns a 16 x 16
// pixel tile (one pixel per lane), stages for a block of views the window of
// bins the tile can see as (A_i, dQ_i) pairs in LDS, and sums the views in a
// fixed order; each pixel is written once, no atomics.  Per (tile, view) the
// window origin and the coefficients of the pixel -> (bin, weight) map are made
// in FP64 by one lane; per pixel the map is two FP32 linear forms and one
// reciprocal: rho = R/L = 1 / (d0 + d1 dx + d2 dy), u = (n0 + n1 dx + n2 dy) rho
// (u local to the window), weight rho^2.
#include "fbp_internal.hpp"

#include <algorithm>

namespace fbp {

namespace {

constexpr int kFanThreads = kFanTile * kFanTile;

__global__ __launch_bounds__(256) void preweight_kernel(const float* __restrict__ in, float* __restrict__ out,
                                                        const float* __restrict__ w, int64_t n, int D) {
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < n; e += stride)
        out[e] = in[e] * w[e % D];
}

__global__ __launch_bounds__(kFanThreads) void fan_bp_kernel(FanJob job) {
    extern __shared__ __align__(16) char smem[];
    const int KB = job.KB, WL = job.WL, N = job.N, K = job.K, D = job.D;
    float* coef = reinterpret_cast<float*>(smem);                      // [KB][8]
    int* org = reinterpret_cast<int*>(coef + 8 * KB);                  // [KB] window origins
    float2* win = reinterpret_cast<float2*>(org + ((KB + 3) & ~3));    // [KB][WL] (A_i, dQ_i)
    const int tiles = job.tiles_x * job.tiles_x;
    const int s = blockIdx.x / tiles;
    const int tile = blockIdx.x - s * tiles;
    const int c0 = (tile % job.tiles_x) * kFanTile, r0 = (tile / job.tiles_x) * kFanTile;
    const int dx = threadIdx.x & (kFanTile - 1), dy = threadIdx.x / kFanTile;
    const bool inside = c0 + dx < N && r0 + dy < N;
    const int cw = min(kFanTile, N - c0), rh = min(kFanTile, N - r0);   // pixels of the tile in the image
    const float fdx = (float)dx, fdy = (float)dy;
    const float* __restrict__ qs = job.q + (size_t)s * K * D;
    float acc = 0.0f;
    for (int k0 = 0; k0 < K; k0 += KB) {
        const int nk = min(KB, K - k0);
        __syncthreads();                                               // previous block's reads done
        if ((int)threadIdx.x < nk) {
            // FP64: window origin and map coefficients of this tile for view k0 + t
            const int k = k0 + threadIdx.x;
            const double c = job.cs[2 * k], sn = job.cs[2 * k + 1];
            const double R = job.R, ds = job.ds, cd = job.centre_det;
            const double xt = (double)c0 - job.half_pix, yt = (double)r0 - job.half_pix;
            const double Lt = R - (c * xt + sn * yt);                  // depth of the tile origin
            const double Nt = R * (-sn * xt + c * yt);                 // R (X . e) at the tile origin
            double umin = INFINITY;
            for (int q = 0; q < 4; ++q) {                              // extremes sit at the corners
                const double ex = (q & 1) ? (double)(cw - 1) : 0.0, ey = (q & 2) ? (double)(rh - 1) : 0.0;
                const double u = (Nt + R * (-sn * ex + c * ey)) / ((Lt - c * ex - sn * ey) * ds) + cd;
                umin = fmin(umin, u);
            }
            const double i0 = floor(umin);
            const double G = (i0 - cd) * ds;
            const double a0 = Nt - G * Lt, a1 = -R * sn + G * c, a2 = R * c + G * sn;
            const double inv = 1.0 / (ds * R);
            float* cf = coef + 8 * threadIdx.x;
            cf[0] = (float)(a0 * inv);
            cf[1] = (float)(a1 * inv);
            cf[2] = (float)(a2 * inv);
            cf[3] = 0.0f;
            cf[4] = (float)(Lt / R);
            cf[5] = (float)(-c / R);
            cf[6] = (float)(-sn / R);
            cf[7] = 0.0f;
            org[threadIdx.x] = (int)i0;
        }
        __syncthreads();
        // windows: value at local u in [i, i+1) is A_i + u dQ_i, zero beyond the detector
        for (int e = threadIdx.x; e < nk * WL; e += kFanThreads) {
            const int kk = e / WL, i = e - kk * WL;
            const int bin = org[kk] + i;
            const float* __restrict__ q = qs + (size_t)(k0 + kk) * D;
            const float a = (bin >= 0 && bin < D) ? q[bin] : 0.0f;
            const float b = (bin + 1 >= 0 && bin + 1 < D) ? q[bin + 1] : 0.0f;
            const float dq = b - a;
            win[e] = make_float2(fmaf(-(float)i, dq, a), dq);
        }
        __syncthreads();
        if (inside) {
            for (int kk = 0; kk < nk; ++kk) {
                const float4 nf = *reinterpret_cast<const float4*>(coef + 8 * kk);
                const float4 df = *reinterpret_cast<const float4*>(coef + 8 * kk + 4);
                const float den = fmaf(df.z, fdy, fmaf(df.y, fdx, df.x));
                const float num = fmaf(nf.z, fdy, fmaf(nf.y, fdx, nf.x));
                const float rho = __builtin_amdgcn_rcpf(den);          // R / L
                const float u = num * rho;
                const int i = min(max((int)u, 0), WL - 1);
                const float2 p = win[kk * WL + i];
                acc = fmaf(rho * rho, fmaf(u, p.y, p.x), acc);
            }
        }
    }
    if (inside) job.img[(size_t)s * N * N + (size_t)(r0 + dy) * N + (c0 + dx)] = acc * job.scale;
}

}  // namespace

size_t fan_lds_bytes(int KB, int WL) {
    return sizeof(float) * 8 * (size_t)KB + sizeof(int) * (size_t)((KB + 3) & ~3) +
           sizeof(float) * 2 * (size_t)KB * (size_t)WL;
}

hipError_t launch_preweight(const float* in, float* out, const float* w, int64_t rows, int D, hipStream_t stream) {
    const int64_t n = rows * (int64_t)D;
    if (n <= 0) return hipSuccess;
    const int64_t blocks = std::min<int64_t>((n + 255) / 256, 65536);
    return launch_kernel(preweight_kernel, dim3((unsigned)blocks), dim3(256), 0, stream, in, out, w, n, D);
}

hipError_t launch_fan_bp(const FanJob& job, int n_slices, hipStream_t stream) {
    if (n_slices <= 0) return hipSuccess;
    if (job.KB < 1 || job.WL < 2) return hipErrorInvalidValue;
    const int64_t blocks = (int64_t)job.tiles_x * job.tiles_x * n_slices;
    if (blocks > INT32_MAX) return hipErrorInvalidValue;
    const size_t lds = fan_lds_bytes(job.KB, job.WL);
    if (lds > kFanLdsBudget) return hipErrorInvalidValue;
    return launch_kernel(fan_bp_kernel, dim3((unsigned)blocks), dim3(kFanThreads), lds, stream, job);
}

}  // namespace fbp
