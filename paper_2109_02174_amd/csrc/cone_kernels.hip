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
// each view, exactly the detector window the block's voxels can see (found in
// FP64 from the tile's corners and the block's z extent) as raw values in LDS,
// windows packed back to back.  The in-plane map is that of the fan beam (per
// (tile, view) an FP64 origin and six FP32 coefficients; per column rho = R/L,
// the column coordinate u and the weight rho^2); along z the row coordinate is
// v = z rho / dv + const, one FMA per voxel, and the four detector values come
// from two two-dword LDS reads at one address.  Views are summed in a fixed
// order, each voxel is written once, no atomics.
#include "fbp_internal.hpp"

#include <algorithm>
#include <type_traits>

namespace fbp {

namespace {

constexpr int kConeThreads = kConeTile * kConeTile;
constexpr int kConeCoef = 12;                           // per-view floats in LDS

// Copies units of G consecutive detector columns (G = 4: one 16-byte load and
// LDS store; the window origins, Du, the pitch and the view base are then
// multiples of four floats, so a unit lies wholly on or off the detector) of the
// windows of views kq .. kq+3 into LDS, one unit per lane and view in flight.
template <int G>
__device__ __forceinline__ void cone_stage(const ConeJob& job, const int* org, float* win, int kq, int nk, int k0,
                                           int pitch) {
    using V = typename std::conditional<G == 4, float4, float>::type;
    int i0[4], j0[4], ng[4], nr[4], units[4], off[4];
    float inv_ng[4];
    int most = 0;
#pragma unroll
    for (int u = 0; u < 4; ++u) {
        const int kk = min(kq + u, nk - 1);
        const int4 o = *reinterpret_cast<const int4*>(org + 8 * kk);
        i0[u] = o.x;
        j0[u] = o.y;
        ng[u] = o.z / G;
        nr[u] = o.w;
        off[u] = org[8 * kk + 4];
        units[u] = kq + u < nk ? ng[u] * nr[u] : 0;
        inv_ng[u] = 1.0f / (float)ng[u];
        most = max(most, units[u]);
    }
    for (int e = threadIdx.x; e < most; e += kConeThreads) {
        V val[4];
        int at[4];
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            // unit e is (row e / ng, group e % ng); the quotient from a float
            // reciprocal is exact: e < 2^16, and (e + 1/2) / ng is at least
            // 1 / (2 ng) away from an integer
            const int rr = (int)(((float)e + 0.5f) * inv_ng[u]);
            const int cc = G * (e - __mul24(rr, ng[u]));
            const int row = j0[u] + rr, col = i0[u] + cc;
            at[u] = e < units[u] ? off[u] + __mul24(rr, pitch) + cc : -1;
            const float* __restrict__ src = job.q + (size_t)(k0 + kq + u) * job.Dv * job.Du;
            const unsigned gb = (unsigned)(__mul24(row, job.Du) + col) * 4u;   // < 2^28
            if (e < units[u] && (unsigned)row < (unsigned)job.Dv && (unsigned)col < (unsigned)job.Du)
                val[u] = *reinterpret_cast<const V*>(reinterpret_cast<const char*>(src) + gb);
            else
                val[u] = V{};
        }
#pragma unroll
        for (int u = 0; u < 4; ++u)
            if (at[u] >= 0) *reinterpret_cast<V*>(win + at[u]) = val[u];
    }
}

// STAGED: each view's detector window goes through LDS with a row pitch of P
// floats (P = 0: the pitch is job.pitch; a fixed P lets the two rows of a bilinear
// sample come from one LDS address with constant offsets).  Windows are packed
// back to back by their actual row count, so a block takes as many of the next
// KB views as fit job.cap floats (at least one: the host checks that the largest
// possible window fits).  Otherwise the four values come from global memory with
// detector bounds checks.  Both read the same per-view window and share the
// arithmetic.
template <bool STAGED, int P>
__global__ __launch_bounds__(kConeThreads) void cone_bp_kernel(ConeJob job) {
    extern __shared__ __align__(16) char smem[];
    const int KB = job.KB, N = job.N, K = job.K, Du = job.Du, Dv = job.Dv;
    const int pitch = P > 0 ? P : job.pitch;
    const int RW = job.WV + 1;                         // rows of the largest window
    const int A = job.vec4 ? 4 : 1;                    // column alignment of the windows
    // per view: n0 n1 n2 cvj | d0 d1 d2 umax | vmax - - - (floats); column
    // origin, row origin, columns, rows, LDS offset, - - - (ints); then the
    // number of views in the block
    float* coef = reinterpret_cast<float*>(smem);
    int* org = reinterpret_cast<int*>(coef + kConeCoef * KB);
    int* nk_lds = org + 8 * KB;
    float* win = reinterpret_cast<float*>(nk_lds + 4);
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
    for (int k0 = 0; k0 < K;) {
        const int nmax = min(KB, K - k0);
        __syncthreads();                                // previous block's reads done
        if (threadIdx.x < 64) {                         // wave 0: one view per lane (KB <= 64)
            int size = 0;
            if ((int)threadIdx.x < nmax) {
                // FP64, per view: the in-plane map (as the fan beam) and the window
                // of detector cells the tile's voxels can reach.  u = N/L and
                // rho = R/L are linear-fractional in (x, y), so over the tile their
                // extremes sit at the corners; v = z rho / dv + cv is then extreme
                // at a corner of (z, rho).  One cell of margin on each side covers
                // FP32 rounding, and the clamps below keep every read inside the
                // window regardless.
                const int k = k0 + threadIdx.x;
                const double c = job.cs[2 * k], sn = job.cs[2 * k + 1];
                const double R = job.R, du = job.du;
                const double xt = (double)c0 - job.half_pix, yt = (double)r0 - job.half_pix;
                const double Lt = R - (c * xt + sn * yt);
                const double Nt = R * (-sn * xt + c * yt);
                double Lmin = INFINITY, Lmax = -INFINITY, umin = INFINITY, umax = -INFINITY;
                for (int q = 0; q < 4; ++q) {
                    const double ex = (q & 1) ? (double)(cw - 1) : 0.0, ey = (q & 2) ? (double)(rh - 1) : 0.0;
                    const double L = Lt - c * ex - sn * ey;
                    const double u = (Nt + R * (-sn * ex + c * ey)) / (L * du);
                    Lmin = fmin(Lmin, L);
                    Lmax = fmax(Lmax, L);
                    umin = fmin(umin, u);
                    umax = fmax(umax, u);
                }
                const double rlo = R / Lmax, rhi = R / Lmin;
                const double vmin = fmin(fmin(zlo * rlo, zlo * rhi), fmin(zhi * rlo, zhi * rhi)) / job.dv;
                const double vmax = fmax(fmax(zlo * rlo, zlo * rhi), fmax(zhi * rlo, zhi * rhi)) / job.dv;
                // column origin rounded down to the alignment, width up to it
                const int i0 = (int)floor(umin + job.cu) - 1;
                const int i0a = i0 - (((i0 % A) + A) % A);
                const int j0 = (int)floor(vmin + job.cv) - 1;
                const int ncw = (int)floor(umax + job.cu) + 3 - i0a;
                const int nc = min(pitch, (ncw + A - 1) / A * A);
                const int nr = min(RW, (int)floor(vmax + job.cv) + 4 - j0);   // one more row: see the clamp
                const double G = ((double)i0a - job.cu) * du;
                const double a0 = Nt - G * Lt, a1 = -R * sn + G * c, a2 = R * c + G * sn;
                float* cf = coef + kConeCoef * threadIdx.x;
                cf[0] = (float)(a0 * job.inv_duR);
                cf[1] = (float)(a1 * job.inv_duR);
                cf[2] = (float)(a2 * job.inv_duR);
                cf[3] = (float)(job.cv - (double)j0);
                cf[4] = (float)(Lt * job.inv_R);
                cf[5] = (float)(-c * job.inv_R);
                cf[6] = (float)(-sn * job.inv_R);
                cf[7] = (float)(nc - 2);
                cf[8] = (float)(nr - 2);
                int* og = org + 8 * threadIdx.x;
                og[0] = i0a;
                og[1] = j0;
                og[2] = nc;
                og[3] = nr;
                size = nr * pitch;
            }
            if constexpr (STAGED) {
                // pack the windows: LDS offsets from a prefix sum over the lanes; the
                // block takes the views whose windows end within cap (a prefix of them)
                int incl = size;
#pragma unroll
                for (int d = 1; d < 64; d <<= 1) {
                    const int y = __shfl_up(incl, d, 64);
                    if ((int)threadIdx.x >= d) incl += y;
                }
                if ((int)threadIdx.x < nmax) org[8 * threadIdx.x + 4] = incl - size;
                const unsigned long long fit = __ballot((int)threadIdx.x < nmax && incl <= job.cap);
                if (threadIdx.x == 0) nk_lds[0] = __popcll(fit);
            }
        }
        __syncthreads();
        int nk = nmax;
        if constexpr (STAGED) {
            nk = nk_lds[0];
            for (int kq = 0; kq < nk; kq += 4) {
                if (job.vec4)
                    cone_stage<4>(job, org, win, kq, nk, k0, pitch);
                else
                    cone_stage<1>(job, org, win, kq, nk, k0, pitch);
            }
            __syncthreads();
        }
        if (inside) {
            for (int kk = 0; kk < nk; ++kk) {
                const float4 nf = *reinterpret_cast<const float4*>(coef + kConeCoef * kk);
                const float4 df = *reinterpret_cast<const float4*>(coef + kConeCoef * kk + 4);
                const float vmax = coef[kConeCoef * kk + 8];
                const float den = fmaf(df.z, fdy, fmaf(df.y, fdx, df.x));
                const float num = fmaf(nf.z, fdy, fmaf(nf.y, fdx, nf.x));
                const float rho = __builtin_amdgcn_rcpf(den);          // R / L
                const float u = __builtin_amdgcn_fmed3f(num * rho, 0.0f, df.w);
                const float w = rho * rho;
                const int iu = (int)u;
                const float fu = u - (float)iu;
                const float wb = w * fu, wa = w - wb;                  // column weights
                const float a = rho * inv_dv;                          // rows per slice
                const float v0 = fmaf(zlo_dv, rho, nf.w);              // window row of the block's first slice
                if constexpr (STAGED) {
                    // byte offset of the sample's window column in LDS, kept in one
                    // register so each sample's address is one 24-bit multiply-add
                    unsigned boff = (unsigned)((const char*)(win + org[8 * kk + 4] + iu) - smem);
                    asm volatile("" : "+v"(boff));
                    auto sample = [&](int q, float v) {
                        const int iv = (int)v;
                        const float fv = __builtin_amdgcn_fractf(v);   // v >= 0: v - floor(v)
                        const float* __restrict__ p =
                            reinterpret_cast<const float*>(smem + __umul24((unsigned)iv, (unsigned)(4 * pitch)) + boff);
                        const float c0v = fmaf(fv, p[pitch] - p[0], p[0]);
                        const float c1v = fmaf(fv, p[pitch + 1] - p[1], p[1]);
                        acc[q] = fmaf(wb, c1v, fmaf(wa, c0v, acc[q]));
                    };
                    // v is monotone in q (a > 0, and FP32 rounding keeps the order), so
                    // when the first and last slices' rows lie in the window every
                    // slice's does and the clamp can be left out
                    if (v0 >= 0.0f && fmaf((float)(kConeZB - 1), a, v0) <= vmax) {
#pragma unroll
                        for (int q = 0; q < kConeZB; ++q) sample(q, fmaf((float)q, a, v0));
                    } else {
#pragma unroll
                        for (int q = 0; q < kConeZB; ++q)
                            sample(q, __builtin_amdgcn_fmed3f(fmaf((float)q, a, v0), 0.0f, vmax));
                    }
                } else {
                    const float* __restrict__ qv = job.q + (size_t)(k0 + kk) * Dv * Du;
                    const int col = org[8 * kk] + iu;
                    const int row0 = org[8 * kk + 1];
                    auto at = [&](int cc, int rr) {
                        return ((unsigned)cc < (unsigned)Du && (unsigned)rr < (unsigned)Dv) ? qv[rr * Du + cc] : 0.0f;
                    };
#pragma unroll 4
                    for (int q = 0; q < kConeZB; ++q) {
                        const float v = __builtin_amdgcn_fmed3f(fmaf((float)q, a, v0), 0.0f, vmax);
                        const int iv = (int)v;
                        const float fv = __builtin_amdgcn_fractf(v);
                        const int row = row0 + iv;
                        const float p00 = at(col, row), p01 = at(col + 1, row);
                        const float p10 = at(col, row + 1), p11 = at(col + 1, row + 1);
                        const float c0v = fmaf(fv, p10 - p00, p00);
                        const float c1v = fmaf(fv, p11 - p01, p01);
                        acc[q] = fmaf(wb, c1v, fmaf(wa, c0v, acc[q]));
                    }
                }
            }
        }
        k0 += nk;
    }
    if (inside) {
#pragma unroll
        for (int q = 0; q < kConeZB; ++q)
            if (q < zn)
                job.vol[((size_t)(z0 + q) * N + (r0 + dy)) * N + (c0 + dx)] = acc[q] * job.scale;
    }
}

// fixed row pitches (floats) of the staged windows; the second row of a bilinear
// sample sits at an LDS offset of P + 1 <= 255 dwords
constexpr int kConePitches[] = {16, 24, 32, 40, 48, 64, 80, 96, 128, 160, 192, 248};

template <int I>
hipError_t launch_pitch(int pitch, const ConeJob& job, dim3 grid, size_t lds, hipStream_t stream) {
    if constexpr (I < (int)(sizeof(kConePitches) / sizeof(int))) {
        if (pitch == kConePitches[I])
            return launch_kernel(cone_bp_kernel<true, kConePitches[I]>, grid, dim3(kConeThreads), lds, stream, job);
        return launch_pitch<I + 1>(pitch, job, grid, lds, stream);
    } else {
        return launch_kernel(cone_bp_kernel<true, 0>, grid, dim3(kConeThreads), lds, stream, job);
    }
}

}  // namespace

int cone_pitch(int WL) {
    for (int p : kConePitches)
        if (p >= WL + 1) return p;
    return (WL + 4) / 4 * 4;
}

size_t cone_lds_bytes(int KB, int cap, bool staged) {
    return sizeof(float) * kConeCoef * (size_t)KB + sizeof(int) * 8 * (size_t)KB + sizeof(int) * 4 +
           (staged ? sizeof(float) * (size_t)cap : 0);
}

hipError_t launch_cone_bp(const ConeJob& job, bool staged, hipStream_t stream) {
    if (job.KB < 1 || job.KB > 64 || job.WL < 2 || job.WV < 2 || job.pitch < job.WL + 1)
        return hipErrorInvalidValue;
    if (job.vec4 && (job.Du % 4 != 0 || job.pitch % 4 != 0 || job.pitch < job.WL + 7 ||
                     reinterpret_cast<uintptr_t>(job.q) % 16 != 0))
        return hipErrorInvalidValue;
    if (staged && (int64_t)(job.WV + 1) * job.pitch > job.cap) return hipErrorInvalidValue;   // one window must fit
    const size_t lds = cone_lds_bytes(job.KB, job.cap, staged);
    if (lds > kConeLdsBudget) return hipErrorInvalidValue;
    const int64_t blocks = (int64_t)job.tiles_x * job.tiles_x * ((job.Nz + kConeZB - 1) / kConeZB);
    if (blocks > INT32_MAX) return hipErrorInvalidValue;
    const dim3 grid((unsigned)blocks);
    return staged ? launch_pitch<0>(job.pitch, job, grid, lds, stream)
                  : launch_kernel(cone_bp_kernel<false, 0>, grid, dim3(kConeThreads), lds, stream, job);
}

}  // namespace fbp
