// Cone-beam (FDK) backprojection for gfx950: circular source orbit, flat
// detector through the rotation axis.
//
// The 3D extension (Feldkamp, Davis & Kress 1984; Kak & Slaney 1988, ch. 3) of
// the filtered backprojection of arXiv 2109.02174 (section "Computed
// tomography", Eq. 2).  View k has its source at (R cos b_k, R sin b_k, 0);
// detector column i sits at s_i = (i - (Du-1)/2) du along (-sin b, cos b, 0) and
// row j at z_j = (j - (Dv-1)/2) dv along z.  A voxel X = (x, y, z) at depth
// L = R - (x cos b + y sin b) is seen at s = R (x, y) . e / L, z' = R z / L, and
//     vol(X) = (2 pi / K) sum_k (R/L)^2 Q~_k(s/du + (Du-1)/2, z'/dv + (Dv-1)/2)
// with bilinear interpolation, zero beyond the detector.  (The pre-weighting and
// row filter run through the pre-weight kernel and the filter GEMM.)
//
// A workgroup owns a 16 x 16 column tile of the volume and a block of 32 slices
// in z (one column per lane, 32 voxels each).  Per block of views it stages, for
// each view, the detector window the tile's voxels can see (columns from the
// in-plane map, rows from the z extent times the magnification range) as raw
// values in LDS.  The in-plane map is that of the fan beam (per (tile, view) an
// FP64 origin and six FP32 coefficients; per column rho = R/L, the column
// coordinate u and the weight rho^2); along z the row coordinate is
// v = z rho / dv + const, one FMA per voxel, and the four detector values come
// from two two-dword LDS reads.  Views are summed in a fixed order, each voxel is
// written once, no atomics.
#include "fbp_internal.hpp"

#include <algorithm>

namespace fbp {

namespace {

constexpr int kConeThreads = kConeTile * kConeTile;

// STAGED: the detector windows go through LDS (they fit: the host checked);
// otherwise (strong magnification) the four values come from global memory with
// detector bounds checks, in the same arithmetic order.
template <bool STAGED>
__global__ __launch_bounds__(kConeThreads) void cone_bp_kernel(ConeJob job) {
    extern __shared__ __align__(16) char smem[];
    const int KB = job.KB, WL = job.WL, WV = job.WV, N = job.N, K = job.K, Du = job.Du, Dv = job.Dv;
    const int CW = WL + 1, RW = WV + 1;                 // staged columns and rows per view (+1: bilinear)
    float* coef = reinterpret_cast<float*>(smem);      // [KB][8]: n0 n1 n2 cvj d0 d1 d2 -
    int* org = reinterpret_cast<int*>(coef + 8 * KB);  // [KB][2]: column and row origins
    float* win = reinterpret_cast<float*>(org + 2 * KB);   // [KB][RW][CW]
    const int tiles = job.tiles_x * job.tiles_x;
    const int zb = blockIdx.x / tiles;
    const int tile = blockIdx.x - zb * tiles;
    const int c0 = (tile % job.tiles_x) * kConeTile, r0 = (tile / job.tiles_x) * kConeTile;
    const int z0 = zb * kConeZB;
    const int zn = min(kConeZB, job.Nz - z0);
    const int dx = threadIdx.x & (kConeTile - 1), dy = threadIdx.x / kConeTile;
    const bool inside = c0 + dx < N && r0 + dy < N;
    const int cw = min(kConeTile, N - c0), rh = min(kConeTile, N - r0);
    const float fdx = (float)dx, fdy = (float)dy;
    const double zlo = (double)z0 - job.half_z, zhi = zlo + (double)(zn - 1);
    const float zlo_dv = (float)(zlo / job.dv), inv_dv = (float)(1.0 / job.dv);
    float acc[kConeZB];
#pragma unroll
    for (int q = 0; q < kConeZB; ++q) acc[q] = 0.0f;
    const int per_view = RW * CW;
    const float inv_cw = 1.0f / (float)CW, inv_pv = 1.0f / (float)per_view;
    for (int k0 = 0; k0 < K; k0 += KB) {
        const int nk = min(KB, K - k0);
        __syncthreads();                                // previous block's reads done
        if ((int)threadIdx.x < nk) {
            // FP64, per view: column window and in-plane map (as the fan beam), row
            // window from the z extent times the range of R/L over the tile
            const int k = k0 + threadIdx.x;
            const double c = job.cs[2 * k], sn = job.cs[2 * k + 1];
            const double R = job.R, du = job.du;
            const double xt = (double)c0 - job.half_pix, yt = (double)r0 - job.half_pix;
            const double Lt = R - (c * xt + sn * yt);
            const double Nt = R * (-sn * xt + c * yt);
            const double ex = 0.5 * (double)(cw - 1), ey = 0.5 * (double)(rh - 1);
            const double uc = (Nt + R * (-sn * ex + c * ey)) / ((Lt - c * ex - sn * ey) * du) + job.cu;
            const double i0 = floor(uc - job.half_span);
            const double G = (i0 - job.cu) * du;
            const double a0 = Nt - G * Lt, a1 = -R * sn + G * c, a2 = R * c + G * sn;
            double Lmin = INFINITY, Lmax = -INFINITY;
            for (int q = 0; q < 4; ++q) {               // L is linear: extremes at the corners
                const double L = Lt - c * ((q & 1) ? (double)(cw - 1) : 0.0) - sn * ((q & 2) ? (double)(rh - 1) : 0.0);
                Lmin = fmin(Lmin, L);
                Lmax = fmax(Lmax, L);
            }
            const double rlo = R / Lmax, rhi = R / Lmin;
            const double vmin = fmin(fmin(zlo * rlo, zlo * rhi), fmin(zhi * rlo, zhi * rhi)) / job.dv + job.cv;
            const double j0 = floor(vmin);
            float* cf = coef + 8 * threadIdx.x;
            cf[0] = (float)(a0 * job.inv_duR);
            cf[1] = (float)(a1 * job.inv_duR);
            cf[2] = (float)(a2 * job.inv_duR);
            cf[3] = (float)(job.cv - j0);
            cf[4] = (float)(Lt * job.inv_R);
            cf[5] = (float)(-c * job.inv_R);
            cf[6] = (float)(-sn * job.inv_R);
            cf[7] = 0.0f;
            org[2 * threadIdx.x] = (int)i0;
            org[2 * threadIdx.x + 1] = (int)j0;
        }
        __syncthreads();
        // stage the windows (zero off the detector); e -> (view, row, column) by
        // float reciprocals (exact: e < KB RW CW <= 2^20 and the margins 0.5/CW, 0.5/per_view)
        for (int e = threadIdx.x; STAGED && e < nk * per_view; e += kConeThreads) {
            const int kk = (int)(((float)e + 0.5f) * inv_pv);
            const int rem = e - kk * per_view;
            const int rr = (int)(((float)rem + 0.5f) * inv_cw);
            const int cc = rem - rr * CW;
            const int col = org[2 * kk] + cc, row = org[2 * kk + 1] + rr;
            float val = 0.0f;
            if ((unsigned)col < (unsigned)Du && (unsigned)row < (unsigned)Dv)
                val = job.q[((size_t)(k0 + kk) * Dv + row) * Du + col];
            win[e] = val;
        }
        __syncthreads();
        if (inside) {
            const float umax = (float)(WL - 1), vmax = (float)(WV - 1);
            for (int kk = 0; kk < nk; ++kk) {
                const float4 nf = *reinterpret_cast<const float4*>(coef + 8 * kk);
                const float4 df = *reinterpret_cast<const float4*>(coef + 8 * kk + 4);
                const float den = fmaf(df.z, fdy, fmaf(df.y, fdx, df.x));
                const float num = fmaf(nf.z, fdy, fmaf(nf.y, fdx, nf.x));
                const float rho = __builtin_amdgcn_rcpf(den);          // R / L
                const float u = __builtin_amdgcn_fmed3f(num * rho, 0.0f, umax);
                const float w = rho * rho;
                const int iu = (int)u;
                const float fu = u - (float)iu;
                const float a = rho * inv_dv;                          // rows per slice
                const float v0 = fmaf(zlo_dv, rho, nf.w);              // window row of the block's first slice
                if constexpr (STAGED) {
                    const float* __restrict__ base = win + kk * per_view + iu;
#pragma unroll
                    for (int q = 0; q < kConeZB; ++q) {
                        const float v = __builtin_amdgcn_fmed3f(fmaf((float)q, a, v0), 0.0f, vmax);
                        const int iv = (int)v;
                        const float fv = v - (float)iv;
                        const float* __restrict__ p = base + iv * CW;
                        const float r0v = fmaf(fu, p[1] - p[0], p[0]);
                        const float r1v = fmaf(fu, p[CW + 1] - p[CW], p[CW]);
                        acc[q] = fmaf(w, fmaf(fv, r1v - r0v, r0v), acc[q]);
                    }
                } else {
                    const float* __restrict__ qv = job.q + (size_t)(k0 + kk) * Dv * Du;
                    const int col = org[2 * kk] + iu;
                    const int row0 = org[2 * kk + 1];
                    auto at = [&](int cc, int rr) {
                        return ((unsigned)cc < (unsigned)Du && (unsigned)rr < (unsigned)Dv) ? qv[(size_t)rr * Du + cc]
                                                                                        : 0.0f;
                    };
#pragma unroll 4
                    for (int q = 0; q < kConeZB; ++q) {
                        const float v = __builtin_amdgcn_fmed3f(fmaf((float)q, a, v0), 0.0f, vmax);
                        const int iv = (int)v;
                        const float fv = v - (float)iv;
                        const int row = row0 + iv;
                        const float p00 = at(col, row), p01 = at(col + 1, row);
                        const float p10 = at(col, row + 1), p11 = at(col + 1, row + 1);
                        const float r0v = fmaf(fu, p01 - p00, p00);
                        const float r1v = fmaf(fu, p11 - p10, p10);
                        acc[q] = fmaf(w, fmaf(fv, r1v - r0v, r0v), acc[q]);
                    }
                }
            }
        }
    }
    if (inside) {
#pragma unroll
        for (int q = 0; q < kConeZB; ++q)
            if (q < zn)
                job.vol[((size_t)(z0 + q) * N + (r0 + dy)) * N + (c0 + dx)] = acc[q] * job.scale;
    }
}

}  // namespace

size_t cone_lds_bytes(int KB, int WL, int WV, bool staged) {
    return sizeof(float) * 8 * (size_t)KB + sizeof(int) * 2 * (size_t)KB +
           (staged ? sizeof(float) * (size_t)KB * (size_t)(WV + 1) * (size_t)(WL + 1) : 0);
}

hipError_t launch_cone_bp(const ConeJob& job, bool staged, hipStream_t stream) {
    if (job.KB < 1 || job.KB > kConeThreads || job.WL < 2 || job.WV < 2) return hipErrorInvalidValue;
    const size_t lds = cone_lds_bytes(job.KB, job.WL, job.WV, staged);
    if (lds > kConeLdsBudget || (staged && (size_t)job.KB * (job.WV + 1) * (job.WL + 1) > ((size_t)1 << 20)))
        return hipErrorInvalidValue;
    const int64_t blocks = (int64_t)job.tiles_x * job.tiles_x * ((job.Nz + kConeZB - 1) / kConeZB);
    if (blocks > INT32_MAX) return hipErrorInvalidValue;
    return staged ? launch_kernel(cone_bp_kernel<true>, dim3((unsigned)blocks), dim3(kConeThreads), lds, stream, job)
                  : launch_kernel(cone_bp_kernel<false>, dim3((unsigned)blocks), dim3(kConeThreads), lds, stream, job);
}

}  // namespace fbp
