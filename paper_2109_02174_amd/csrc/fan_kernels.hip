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
constexpr int kRawF32 = 0x00020000;     // buffer resource word 3: 32-bit data, raw (stride 0)
constexpr int kPastEnd = 0x7FFFFFF0;    // byte offset beyond any view block: reads as 0

__global__ __launch_bounds__(256) void preweight_kernel(const float* __restrict__ in, float* __restrict__ out,
                                                        const float* __restrict__ w, int64_t n, int D) {
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < n; e += stride)
        out[e] = in[e] * w[e % D];
}

// M slices per workgroup (a stack of one geometry): the map of a pixel and view
// (rho, u, window index) is made once and applied to the M slices' windows, so a
// slice's arithmetic and summation order are those of M = 1 (bitwise equal).
template <int M>
__global__ __launch_bounds__(kFanThreads) void fan_bp_kernel(FanJob job) {
    extern __shared__ __align__(16) char smem[];
    const int KB = job.KB, WL = job.WL, N = job.N, K = job.K, D = job.D;
    float* coef = reinterpret_cast<float*>(smem);                      // [KB][8]
    int* org = reinterpret_cast<int*>(coef + 8 * KB);                  // [KB] window origins
    // (A_i, dQ_i) pairs: M = 1 [KB][WL]; M > 1 [KB][M/2 planes][WL] float4 holding
    // slices 2h, 2h+1, so lanes at consecutive bins read 16-byte strides
    float2* win = reinterpret_cast<float2*>(org + ((KB + 3) & ~3));
    const int tiles = job.tiles_x * job.tiles_x;
    const int g = blockIdx.x / tiles;                                  // group of M slices, or view part
    const int tile = blockIdx.x - g * tiles;
    const int c0 = (tile % job.tiles_x) * kFanTile, r0 = (tile / job.tiles_x) * kFanTile;
    const int dx = threadIdx.x & (kFanTile - 1), dy = threadIdx.x / kFanTile;
    const bool inside = c0 + dx < N && r0 + dy < N;
    const int cw = min(kFanTile, N - c0), rh = min(kFanTile, N - r0);   // pixels of the tile in the image
    const float fdx = (float)dx, fdy = (float)dy;
    const size_t qstride = (size_t)K * D;
    // split > 1 (one slice, M = 1): this workgroup sums the views of part g only
    const int kpart = (K + job.split - 1) / job.split;
    const int kbeg = job.split > 1 ? g * kpart : 0;
    const int kend = job.split > 1 ? min(K, kbeg + kpart) : K;
    const float* __restrict__ qs = job.q + (job.split > 1 ? (size_t)0 : (size_t)g * M * qstride);
    const float inv_wl = 1.0f / (float)WL;
    float acc[M];
#pragma unroll
    for (int m = 0; m < M; ++m) acc[m] = 0.0f;
    for (int k0 = kbeg; k0 < kend; k0 += KB) {
        const int nk = min(KB, kend - k0);
        __syncthreads();                                               // previous block's reads done
        if ((int)threadIdx.x < nk) {
            // FP64: window origin and map coefficients of this tile for view k0 + t.
            // The window starts half_span bins below the bin of the tile's centre
            // (the centre of its pixels inside the image): no pixel of the tile is
            // farther than that from it.
            const int k = k0 + threadIdx.x;
            const double c = job.cs[2 * k], sn = job.cs[2 * k + 1];
            const double R = job.R, ds = job.ds, cd = job.centre_det;
            const double xt = (double)c0 - job.half_pix, yt = (double)r0 - job.half_pix;
            const double Lt = R - (c * xt + sn * yt);                  // depth of the tile origin
            const double Nt = R * (-sn * xt + c * yt);                 // R (X . e) at the tile origin
            const double ex = 0.5 * (double)(cw - 1), ey = 0.5 * (double)(rh - 1);
            const double uc = (Nt + R * (-sn * ex + c * ey)) / ((Lt - c * ex - sn * ey) * ds) + cd;
            const double i0 = floor(uc - job.half_span);
            const double G = (i0 - cd) * ds;
            const double a0 = Nt - G * Lt, a1 = -R * sn + G * c, a2 = R * c + G * sn;
            const double inv = job.inv_dsR, ir = job.inv_R;
            float* cf = coef + 8 * threadIdx.x;
            cf[0] = (float)(a0 * inv);
            cf[1] = (float)(a1 * inv);
            cf[2] = (float)(a2 * inv);
            cf[3] = 0.0f;
            cf[4] = (float)(Lt * ir);
            cf[5] = (float)(-c * ir);
            cf[6] = (float)(-sn * ir);
            cf[7] = 0.0f;
            org[threadIdx.x] = (int)i0;
        }
        __syncthreads();
        // windows: value at local u in [i, i+1) is A_i + u dQ_i, zero beyond the detector;
        // e -> (view, bin) by a float reciprocal (exact: e < KB WL <= 6144, margin 0.5/WL);
        // branch-free buffer loads: offsets of bins off the detector are past the end
#pragma unroll
        for (int m = 0; m < M; ++m) {
            const __amdgpu_buffer_rsrc_t rows = __builtin_amdgcn_make_buffer_rsrc(
                const_cast<float*>(qs + m * qstride + (size_t)k0 * D), (short)0, nk * D * 4, kRawF32);
#pragma unroll 2
            for (int e = threadIdx.x; e < nk * WL; e += kFanThreads) {
                const int kk = (int)(((float)e + 0.5f) * inv_wl), i = e - __mul24(kk, WL);
                const int bin = org[kk] + i;
                const int o = (__mul24(kk, D) + bin) * 4;
                const int oa = (unsigned)bin < (unsigned)D ? o : kPastEnd;
                const int ob = (unsigned)(bin + 1) < (unsigned)D ? o + 4 : kPastEnd;
                const float a = __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(rows, oa, 0, 0));
                const float b = __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(rows, ob, 0, 0));
                const float dq = b - a;
                const int at = M == 1 ? e : ((kk * (M / 2) + m / 2) * WL + i) * 2 + (m & 1);
                win[at] = make_float2(fmaf(-(float)i, dq, a), dq);
            }
        }
        __syncthreads();
        if (inside) {
            const float umax = (float)(WL - 1);
            // one view: the pixel's map, then the M slices' pairs at its window index
            auto map = [&](int kk, float& u, float& w) {
                const float4 nf = *reinterpret_cast<const float4*>(coef + 8 * kk);
                const float4 df = *reinterpret_cast<const float4*>(coef + 8 * kk + 4);
                const float den = fmaf(df.z, fdy, fmaf(df.y, fdx, df.x));
                const float num = fmaf(nf.z, fdy, fmaf(nf.y, fdx, nf.x));
                const float rho = __builtin_amdgcn_rcpf(den);          // R / L
                u = num * rho;
                w = rho * rho;
                const int i = (int)__builtin_amdgcn_fmed3f(u, 0.0f, umax);   // in the window whatever u holds
                return M == 1 ? win + (size_t)kk * WL + i                // pair, or first plane of the M slices
                              : win + ((size_t)kk * (M / 2) * WL + i) * 2;
            };
            auto fetch = [&](const float2* pw, float2 (&p)[M]) {
                if constexpr (M == 1) {
                    p[0] = pw[0];
                } else {
#pragma unroll
                    for (int h = 0; h < M / 2; ++h) {                  // 16-byte reads, two slices each
                        const float4 v = reinterpret_cast<const float4*>(pw)[h * WL];
                        p[2 * h] = make_float2(v.x, v.y);
                        p[2 * h + 1] = make_float2(v.z, v.w);
                    }
                }
            };
            int kk = 0;
            // four views per round: all maps, then all reads, then the sums in view order
            for (; kk + 4 <= nk; kk += 4) {
                float u[4], w[4];
                const float2* pw[4];
                float2 p[4][M];
#pragma unroll
                for (int q = 0; q < 4; ++q) pw[q] = map(kk + q, u[q], w[q]);
#pragma unroll
                for (int q = 0; q < 4; ++q) fetch(pw[q], p[q]);
#pragma unroll
                for (int q = 0; q < 4; ++q) {
#pragma unroll
                    for (int m = 0; m < M; ++m) acc[m] = fmaf(w[q], fmaf(u[q], p[q][m].y, p[q][m].x), acc[m]);
                }
            }
            for (; kk < nk; ++kk) {
                float u, w;
                float2 p[M];
                fetch(map(kk, u, w), p);
#pragma unroll
                for (int m = 0; m < M; ++m) acc[m] = fmaf(w, fmaf(u, p[m].y, p[m].x), acc[m]);
            }
        }
    }
    if (inside) {
        if (job.split > 1) {                                           // partial sum of part g
            job.part[(size_t)g * N * N + (size_t)(r0 + dy) * N + (c0 + dx)] = acc[0];
        } else {
#pragma unroll
            for (int m = 0; m < M; ++m)
                job.img[((size_t)g * M + m) * N * N + (size_t)(r0 + dy) * N + (c0 + dx)] = acc[m] * job.scale;
        }
    }
}

// Quarter-turn views (K = 4 K4, b_{k + i K4} = b_k + i pi/2): turning a pixel by
// +pi/2 about the centre, (x, y) -> (-y, x), and its view by +pi/2 leaves the
// depth L and the detector coordinate s unchanged.  A workgroup owns a 16 x 16
// tile of the base region (rows [0, N/2), columns [0, (N+1)/2): the top-left
// quadrant, or for odd N a pinwheel piece whose four turns cover every pixel but
// the centre) and its three turned copies R_j (j = 1..3).  Per
// base view k < K4 a lane makes its pixel's maps at the four views k + m K4
// (m = 0..3) and applies map m to R_j X at view k + ((m + j) mod 4) K4 for every
// j: sixteen updates per four maps.  The four windows of map m (one per j, all
// at map m's origin) are interleaved two pairs per float4 plane, so 2M reads at
// the map's window index fetch the pairs of the four turned pixels (times M
// slices).  Each output pixel sums its views in a fixed order (base views
// ascending, then m).  Odd N: the centre pixel has depth R and detector
// coordinate (D-1)/2 on every view (weight 1); the workgroup of the first tile
// sums it from the filtered rows after its tile (lanes over views, then a fixed
// butterfly).
template <int M>
__global__ __launch_bounds__(kFanThreads) void fan_rot_kernel(FanJob job) {
    extern __shared__ __align__(16) char smem[];
    const int KB = job.KB, WL = job.WL, N = job.N, K = job.K, D = job.D;
    const int K4 = K / 4, H = N / 2, Wc = (N + 1) / 2;   // base region: H rows, Wc columns
    float* coef = reinterpret_cast<float*>(smem);                      // [KB][4 maps][8]
    int* org = reinterpret_cast<int*>(coef + 32 * KB);                 // [KB][4 maps] window origins
    // [KB][4 maps][2M planes][WL] float4: plane h holds pairs 2h, 2h+1 of the
    // (turn j, slice) list j M + slice, so lanes at consecutive bins read 16-byte strides
    float4* win = reinterpret_cast<float4*>(org + 4 * KB);
    const int tiles = job.tiles_x * ((H + kFanTile - 1) / kFanTile);   // base-region tiles
    const int g = blockIdx.x / tiles;                                  // group of M slices, or view part
    const int tile = blockIdx.x - g * tiles;
    const int c0 = (tile % job.tiles_x) * kFanTile, r0 = (tile / job.tiles_x) * kFanTile;
    const int dx = threadIdx.x & (kFanTile - 1), dy = threadIdx.x / kFanTile;
    const bool inside = c0 + dx < Wc && r0 + dy < H;
    const int cw = min(kFanTile, Wc - c0), rh = min(kFanTile, H - r0);  // pixels of the tile in the base region
    const float fdx = (float)dx, fdy = (float)dy;
    const size_t qstride = (size_t)K * D;
    // split > 1 (one slice, M = 1): this workgroup sums the base views of part g only
    const int kpart = (K4 + job.split - 1) / job.split;
    const int kbeg = job.split > 1 ? g * kpart : 0;
    const int kend = job.split > 1 ? min(K4, kbeg + kpart) : K4;
    const float* __restrict__ qs = job.q + (job.split > 1 ? (size_t)0 : (size_t)g * M * qstride);
    const float inv_wl = 1.0f / (float)WL;
    float acc[4][M];
#pragma unroll
    for (int j = 0; j < 4; ++j)
#pragma unroll
        for (int m = 0; m < M; ++m) acc[j][m] = 0.0f;
    for (int k0 = kbeg; k0 < kend; k0 += KB) {
        const int nk = min(KB, kend - k0);
        __syncthreads();                                               // previous block's reads done
        if ((int)threadIdx.x < 4 * nk) {
            // FP64: window origin and map of this tile at view k0 + kk + m K4, as in
            // the one-view kernel
            const int k = k0 + ((int)threadIdx.x >> 2) + ((int)threadIdx.x & 3) * K4;
            const double c = job.cs[2 * k], sn = job.cs[2 * k + 1];
            const double R = job.R, ds = job.ds, cd = job.centre_det;
            const double xt = (double)c0 - job.half_pix, yt = (double)r0 - job.half_pix;
            const double Lt = R - (c * xt + sn * yt);
            const double Nt = R * (-sn * xt + c * yt);
            const double ex = 0.5 * (double)(cw - 1), ey = 0.5 * (double)(rh - 1);
            const double uc = (Nt + R * (-sn * ex + c * ey)) / ((Lt - c * ex - sn * ey) * ds) + cd;
            const double i0 = floor(uc - job.half_span);
            const double G = (i0 - cd) * ds;
            const double a0 = Nt - G * Lt, a1 = -R * sn + G * c, a2 = R * c + G * sn;
            const double inv = job.inv_dsR, ir = job.inv_R;
            float* cf = coef + 8 * threadIdx.x;
            cf[0] = (float)(a0 * inv);
            cf[1] = (float)(a1 * inv);
            cf[2] = (float)(a2 * inv);
            cf[3] = 0.0f;
            cf[4] = (float)(Lt * ir);
            cf[5] = (float)(-c * ir);
            cf[6] = (float)(-sn * ir);
            cf[7] = 0.0f;
            org[threadIdx.x] = (int)i0;
        }
        __syncthreads();
        // windows: (map km = kk 4 + m, bin index i) holds, for the four turns j, the
        // pairs of bin org + i of view k0 + kk + ((m + j) mod 4) K4 (times M slices)
        // in the 2M planes of map km; (km, i) from a float reciprocal (exact: km WL + i < 4 KB WL,
        // which the LDS budget keeps below 2^11; margin 0.5/WL).  Branch-free buffer
        // loads over each slice's K D values (offsets of bins off the detector are
        // past the end), 8 M in flight per lane.
        {
            __amdgpu_buffer_rsrc_t rows[M];
#pragma unroll
            for (int mm = 0; mm < M; ++mm)
                rows[mm] = __builtin_amdgcn_make_buffer_rsrc(const_cast<float*>(qs + mm * qstride), (short)0,
                                                             (int)(qstride * 4), kRawF32);
            for (int e4 = threadIdx.x; e4 < 4 * nk * WL; e4 += kFanThreads) {
                const int km = (int)(((float)e4 + 0.5f) * inv_wl);
                const int i = e4 - __mul24(km, WL);
                const int bin = org[km] + i;
                const bool va = (unsigned)bin < (unsigned)D, vb = (unsigned)(bin + 1) < (unsigned)D;
                const int m = km & 3, kb = k0 + (km >> 2);
                const float fi = (float)i;
                float2 pr[4][M];
#pragma unroll
                for (int j = 0; j < 4; ++j) {
                    const int o = (__mul24(kb + __mul24((m + j) & 3, K4), D) + bin) * 4;   // below kPastEnd
                    const int oa = va ? o : kPastEnd, ob = vb ? o + 4 : kPastEnd;
#pragma unroll
                    for (int mm = 0; mm < M; ++mm) {
                        const float a = __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(rows[mm], oa, 0, 0));
                        const float b = __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(rows[mm], ob, 0, 0));
                        const float dq = b - a;
                        pr[j][mm] = make_float2(fmaf(-fi, dq, a), dq);
                    }
                }
                float4* dst = win + (size_t)km * 2 * M * WL + i;
#pragma unroll
                for (int h = 0; h < 2 * M; ++h) {
                    const float2 x = pr[(2 * h) / M][(2 * h) % M], y = pr[(2 * h + 1) / M][(2 * h + 1) % M];
                    dst[h * WL] = make_float4(x.x, x.y, y.x, y.y);
                }
            }
        }
        __syncthreads();
        if (inside) {
            const float umax = (float)(WL - 1);
            for (int kk = 0; kk < nk; ++kk) {
                float u[4], w[4];
                const float4* pw[4];
#pragma unroll
                for (int m = 0; m < 4; ++m) {                          // the four maps first
                    const float4 nf = *reinterpret_cast<const float4*>(coef + 8 * (4 * kk + m));
                    const float4 df = *reinterpret_cast<const float4*>(coef + 8 * (4 * kk + m) + 4);
                    const float den = fmaf(df.z, fdy, fmaf(df.y, fdx, df.x));
                    const float num = fmaf(nf.z, fdy, fmaf(nf.y, fdx, nf.x));
                    const float rho = __builtin_amdgcn_rcpf(den);      // R / L
                    u[m] = num * rho;
                    w[m] = rho * rho;
                    const int i = (int)__builtin_amdgcn_fmed3f(u[m], 0.0f, umax);   // in the window whatever u holds
                    pw[m] = win + (size_t)(4 * kk + m) * 2 * M * WL + i;
                }
#pragma unroll
                for (int m = 0; m < 4; ++m) {
                    float4 v[2 * M];                                   // (A, dQ) of the 4 turns x M slices
#pragma unroll
                    for (int h = 0; h < 2 * M; ++h) v[h] = pw[m][h * WL];
#pragma unroll
                    for (int j = 0; j < 4; ++j) {
#pragma unroll
                        for (int mm = 0; mm < M; ++mm) {
                            const int f = j * M + mm;                  // pair f: float4 f / 2, half f % 2
                            const float A = (f & 1) ? v[f >> 1].z : v[f >> 1].x;
                            const float dQ = (f & 1) ? v[f >> 1].w : v[f >> 1].y;
                            acc[j][mm] = fmaf(w[m], fmaf(u[m], dQ, A), acc[j][mm]);
                        }
                    }
                }
            }
        }
    }
    if (inside) {
        const int c = c0 + dx, r = r0 + dy;
        // R_j (c, r): j = 1 (-y, x), j = 2 (-x, -y), j = 3 (y, -x) about the centre
        const int cj[4] = {c, N - 1 - r, N - 1 - c, r};
        const int rj[4] = {r, c, N - 1 - r, N - 1 - c};
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            const size_t pix = (size_t)rj[j] * N + cj[j];
            if (job.split > 1) {
                job.part[(size_t)g * N * N + pix] = acc[j][0];
            } else {
#pragma unroll
                for (int mm = 0; mm < M; ++mm) job.img[((size_t)g * M + mm) * N * N + pix] = acc[j][mm] * job.scale;
            }
        }
    }
    if ((N & 1) && tile == 0 && threadIdx.x < 64) {
        const int lane = threadIdx.x, jc = (D - 1) >> 1, nv = 4 * (kend - kbeg);
        const bool between = (D & 1) == 0;            // (D-1)/2 midway between bins jc and jc + 1
        const size_t pix = (size_t)(N >> 1) * N + (N >> 1);
#pragma unroll
        for (int mm = 0; mm < M; ++mm) {
            const float* __restrict__ qm = qs + mm * qstride;
            float csum = 0.0f;
            for (int t = lane; t < nv; t += 64) {     // view kbeg + t / 4 + (t % 4) K4
                const float* __restrict__ row = qm + (size_t)(kbeg + (t >> 2) + (t & 3) * K4) * D;
                csum += between ? 0.5f * (row[jc] + row[jc + 1]) : row[jc];
            }
#pragma unroll
            for (int o = 32; o > 0; o >>= 1) csum += __shfl_xor(csum, o);
            if (lane == 0) {
                if (job.split > 1) job.part[(size_t)g * N * N + pix] = csum;
                else job.img[((size_t)g * M + mm) * N * N + pix] = csum * job.scale;
            }
        }
    }
}

}  // namespace

size_t fan_lds_bytes(int KB, int WL, int M) {
    return sizeof(float) * 8 * (size_t)KB + sizeof(int) * (size_t)((KB + 3) & ~3) +
           sizeof(float) * 2 * (size_t)M * (size_t)KB * (size_t)WL;
}

bool fan_rot_addressable(int K, int D, int WL) {
    // every byte offset the staging forms, (view D + bin) 4 with bin < D + WL,
    // stays below the past-the-end offset
    return ((int64_t)K * D + WL + 1) * 4 < (int64_t)kPastEnd;
}

size_t fan_rot_lds_bytes(int KB, int WL, int M) {
    return sizeof(float) * 32 * (size_t)KB + sizeof(int) * 4 * (size_t)KB +
           sizeof(float) * 2 * 16 * (size_t)M * (size_t)KB * (size_t)WL;
}

// Quarter-turn form (N >= 2, K = 4 K4 with the views in quarter turns, K D 4 bytes
// addressable by a buffer resource): groups of M slices, the rest one slice per
// workgroup; a single slice may split its base views over job.split parts.
hipError_t launch_fan_rot(const FanJob& job, int n_slices, int M, int KBm, hipStream_t stream) {
    if (n_slices <= 0) return hipSuccess;
    if (job.N < 2 || (job.K & 3) || job.K < 4 || job.KB < 1 || 4 * job.KB > kFanThreads || job.WL < 2 ||
        (M != 1 && M != 2 && M != 4) || (M > 1 && (KBm < 1 || 4 * KBm > kFanThreads)) ||
        !fan_rot_addressable(job.K, job.D, job.WL) || job.tiles_x != ((job.N + 1) / 2 + kFanTile - 1) / kFanTile)
        return hipErrorInvalidValue;
    const int64_t tiles = (int64_t)job.tiles_x * ((job.N / 2 + kFanTile - 1) / kFanTile);
    const int grouped = (M > 1) ? n_slices - n_slices % M : 0;
    if (grouped > 0) {
        FanJob j = job;
        j.KB = KBm;
        j.split = 1;
        const size_t lds = fan_rot_lds_bytes(KBm, job.WL, M);
        const int64_t blocks = tiles * (grouped / M);
        if (blocks > INT32_MAX || lds > kFanLdsBudget) return hipErrorInvalidValue;
        const hipError_t e = (M == 2)
            ? launch_kernel(fan_rot_kernel<2>, dim3((unsigned)blocks), dim3(kFanThreads), lds, stream, j)
            : launch_kernel(fan_rot_kernel<4>, dim3((unsigned)blocks), dim3(kFanThreads), lds, stream, j);
        if (e != hipSuccess) return e;
    }
    const int rest = n_slices - grouped;
    if (rest == 0) return hipSuccess;
    const size_t lds = fan_rot_lds_bytes(job.KB, job.WL, 1);
    if (lds > kFanLdsBudget) return hipErrorInvalidValue;
    if (job.split > 1) {                                               // one slice, base views split over parts
        if (n_slices != 1 || M != 1 || !job.part || job.split > job.K / 4) return hipErrorInvalidValue;
        const int64_t blocks = tiles * job.split;
        if (blocks > INT32_MAX) return hipErrorInvalidValue;
        return launch_kernel(fan_rot_kernel<1>, dim3((unsigned)blocks), dim3(kFanThreads), lds, stream, job);
    }
    FanJob j = job;
    j.q = job.q + (size_t)grouped * job.K * job.D;
    j.img = job.img + (size_t)grouped * job.N * job.N;
    const int64_t blocks = tiles * rest;
    if (blocks > INT32_MAX) return hipErrorInvalidValue;
    return launch_kernel(fan_rot_kernel<1>, dim3((unsigned)blocks), dim3(kFanThreads), lds, stream, j);
}

hipError_t launch_preweight(const float* in, float* out, const float* w, int64_t rows, int D, hipStream_t stream) {
    const int64_t n = rows * (int64_t)D;
    if (n <= 0) return hipSuccess;
    const int64_t blocks = std::min<int64_t>((n + 255) / 256, 65536);
    return launch_kernel(preweight_kernel, dim3((unsigned)blocks), dim3(256), 0, stream, in, out, w, n, D);
}

// n_slices of one geometry: groups of M through the M-slice kernel (KB views per
// block for it), the rest one slice per workgroup.
hipError_t launch_fan_bp(const FanJob& job, int n_slices, int M, int KBm, hipStream_t stream) {
    if (n_slices <= 0) return hipSuccess;
    if (job.KB < 1 || job.WL < 2 || (M != 1 && M != 2 && M != 4) || (M > 1 && KBm < 1)) return hipErrorInvalidValue;
    const int64_t tiles = (int64_t)job.tiles_x * job.tiles_x;
    const int grouped = (M > 1) ? n_slices - n_slices % M : 0;
    if (grouped > 0) {
        FanJob j = job;
        j.KB = KBm;
        const size_t lds = fan_lds_bytes(KBm, job.WL, M);
        const int64_t blocks = tiles * (grouped / M);
        if (blocks > INT32_MAX || lds > kFanLdsBudget) return hipErrorInvalidValue;
        const hipError_t e = (M == 2)
            ? launch_kernel(fan_bp_kernel<2>, dim3((unsigned)blocks), dim3(kFanThreads), lds, stream, j)
            : launch_kernel(fan_bp_kernel<4>, dim3((unsigned)blocks), dim3(kFanThreads), lds, stream, j);
        if (e != hipSuccess) return e;
    }
    const int rest = n_slices - grouped;
    if (rest == 0) return hipSuccess;
    if (job.split > 1) {                                               // one slice, views split over parts
        if (n_slices != 1 || M != 1 || !job.part || job.split > job.K) return hipErrorInvalidValue;
        const size_t lds = fan_lds_bytes(job.KB, job.WL, 1);
        const int64_t blocks = tiles * job.split;
        if (blocks > INT32_MAX || lds > kFanLdsBudget) return hipErrorInvalidValue;
        return launch_kernel(fan_bp_kernel<1>, dim3((unsigned)blocks), dim3(kFanThreads), lds, stream, job);
    }
    FanJob j = job;
    j.q = job.q + (size_t)grouped * job.K * job.D;
    j.img = job.img + (size_t)grouped * job.N * job.N;
    const size_t lds = fan_lds_bytes(job.KB, job.WL, 1);
    const int64_t blocks = tiles * rest;
    if (blocks > INT32_MAX || lds > kFanLdsBudget) return hipErrorInvalidValue;
    return launch_kernel(fan_bp_kernel<1>, dim3((unsigned)blocks), dim3(kFanThreads), lds, stream, j);
}

}  // namespace fbp
