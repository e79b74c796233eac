// Pixel-driven, gather-only backprojection for gfx950.
//
// Computes Eq. 2 of arXiv 2109.02174 (section "Computed tomography") with the
// pi/K weight and linear interpolation:
//     img[r][c] = (pi/K) sum_k Q~_k(u_k),  u_k = (x_c cos th_k + y_r sin th_k)/dt + (D-1)/2.
//
// Design:
//  * A workgroup owns a TW x TH tile of the upper half image AND the tile's point
//    reflection through the centre.  The reflected pixel (-x, -y) sits at
//    u' = (D-1) - u, so it reads the reversed filtered row at the SAME local
//    coordinate: one coordinate, one truncation and one LDS address serve two pixels.
//  * Angles are streamed in blocks of KB.  Per (tile, angle) the window origin is
//    computed once in FP64; lanes then work in FP32 coordinates local to that
//    window.  The window starts one bin below the tile's smallest coordinate, so
//    every local coordinate is >= 1 - (rounding) > 0 and truncation toward zero is
//    floor: one v_cvt_i32_f32 gives the bin.
//  * The staged window holds, per bin j and for both directions, the pair
//    (A_j, dL_j) with dL_j = L[j+1] - L[j] and A_j = L[j] - j dL_j, so the
//    interpolated value at local coordinate u in [j, j+1) is A_j + u dL_j: one
//    FMA, no fraction.  One ds_read_b128 returns both directions.
//  * The workgroup has S groups of 256 lanes over the same pixels; group g takes
//    the g-th contiguous quarter (for S = 4) of every staged block, and the S
//    partial sums are added in fixed order at the end.  This gives a single 512^2
//    slice enough waves per CU.  Per-angle constants come from LDS (not scalar
//    loads, which would force full LDS drains inside the loop).
//  * The next block's filtered rows are loaded into registers while the current
//    block is computed, so the global-load latency hides behind the LDS work.
//    The loads are buffer loads whose range check supplies the zeros beyond the
//    detector ends, so staging has no compares or branches.
//  * Each pixel is written once by one lane; no atomics.  The summation order
//    depends only on the tile shape, which is fixed per geometry, so repeated and
//    batched calls are bitwise identical.
#include "fbp_internal.hpp"

namespace fbp {

namespace {

__device__ __forceinline__ float ld_zero(const float* __restrict__ row, int g, int D) {
    return (g >= 0 && g < D) ? row[g] : 0.0f;
}

// XCD-aware remap: hardware places block b on XCD b % 8; give each XCD a contiguous
// range of logical tiles so the tiles sharing filtered rows share an L2.
__device__ __forceinline__ int xcd_logical(int b, int G) {
    const int x = b & 7;
    const int slot = b >> 3;
    const int per = G >> 3;
    const int extra = G & 7;
    return x * per + min(x, extra) + slot;
}

// Word 3 of a raw (stride 0) buffer resource: 32-bit data format, no swizzle; reads
// at byte offsets >= num_records return 0.
constexpr int kBufferWord3 = 0x00020000;

// LDS layout: prm[2][kMaxKB] float4 {b, cos/dt, sin/dt, i0 bits} per angle of the
// current and next block, then the window (float4 [KB][WL]), which the final
// cross-group reduction reuses.
constexpr int kPrmBytes = kBpPrmBytes;

template <int TW, int P, int S>
struct Shape {
    static constexpr int NT = kGroupThreads * S;
    static constexpr int TH = (kGroupThreads / TW) * P;
    static constexpr int RED_BYTES = (S - 1) * kGroupThreads * 2 * P * 4;
};

template <int TW, int P, int S>
__device__ __forceinline__ void bp_tile(const BpJob& job, const float* __restrict__ q,
                                        float* __restrict__ img, int c0, int r0, char* smem) {
    using Sh = Shape<TW, P, S>;
    constexpr int NT = Sh::NT;
    constexpr int TH = Sh::TH;
    float4* prm = reinterpret_cast<float4*>(smem);                      // [2][kMaxKB]
    float4* win = reinterpret_cast<float4*>(smem + kPrmBytes);

    const int t = threadIdx.x;
    const int grp = __builtin_amdgcn_readfirstlane(t >> 8);   // wave-uniform angle group
    const int tl = t & (kGroupThreads - 1);
    const int lx = tl % TW;
    const int ly0 = (tl / TW) * P;
    const int N = job.N, K = job.K, D = job.D, WL = job.WL, KB = job.KB;
    const double x0 = (double)c0 - job.half_pix;
    const double y0 = (double)r0 - job.half_pix;
    const float flx = (float)lx;
    const float fly = (float)ly0;

    // Staging: one wave fills one segment of 63 window bins of one angle per pass.
    // Lane j loads bin i0 + 63 seg + j of the forward row and the mirrored bin of the
    // reversed row with single-dword buffer loads; a per-row buffer resource of D
    // floats returns 0 outside the detector, which is the zero extension of the
    // filtered row.  The value at bin + 1 comes from the next lane (ds_bpermute), so
    // 64 lanes produce 63 (A, dL) pairs per direction.
    constexpr int W = NT / 64;                  // waves per workgroup
    const int wave = __builtin_amdgcn_readfirstlane(t >> 6);
    const int lane = t & 63;
    const int seg_shift = job.seg_shift;        // log2(segments per angle)
    const int nxt = ((lane + 1) & 63) << 2;     // ds_bpermute source: lane + 1
    const int d4 = (D - 1) * 4;

    float accf[P], accr[P];
#pragma unroll
    for (int i = 0; i < P; ++i) {
        accf[i] = 0.0f;
        accr[i] = 0.0f;
    }

    // window origin (FP64) of the angles of the block starting at kb, into buffer buf
    auto params = [&](int kb, int buf) {
        const int nb = min(KB, K - kb);
        if (t < nb) {
            const double cd = job.cs[2 * (kb + t)];
            const double sd = job.cs[2 * (kb + t) + 1];
            const double uo = x0 * cd + y0 * sd + job.centre_det;
            const double umin = uo + fmin(0.0, (double)(TW - 1) * cd) + fmin(0.0, (double)(TH - 1) * sd);
            const int i0 = (int)floor(umin) - 1;
            prm[buf * kMaxKB + t] = make_float4((float)(uo - (double)i0), (float)cd, (float)sd,
                                                __int_as_float(i0));
        }
    };
    float pf[kStageE], pr[kStageE];
    auto load = [&](int kb, int buf) {
        const int nslot = min(KB, K - kb) << seg_shift;
#pragma unroll
        for (int e = 0; e < kStageE; ++e) {
            const int slot = wave + e * W;                       // wave-uniform
            if (slot < nslot) {
                const int a = slot >> seg_shift;
                const int seg = slot & ((1 << seg_shift) - 1);
                const __amdgpu_buffer_rsrc_t row = __builtin_amdgcn_make_buffer_rsrc(
                    const_cast<float*>(q + (size_t)(kb + a) * (size_t)D), (short)0, D * 4, kBufferWord3);
                const int g4 = (__float_as_int(prm[buf * kMaxKB + a].w) + 63 * seg + lane) * 4;
                pf[e] = __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(row, g4, 0, 0));
                pr[e] = __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(row, d4 - g4, 0, 0));
            }
        }
    };
    auto store = [&](int kb) {
        const int nslot = min(KB, K - kb) << seg_shift;
#pragma unroll
        for (int e = 0; e < kStageE; ++e) {
            const int slot = wave + e * W;
            if (slot < nslot) {
                const int a = slot >> seg_shift;
                const int j = 63 * (slot & ((1 << seg_shift) - 1)) + lane;
                const float f1 = __builtin_bit_cast(float, __builtin_amdgcn_ds_bpermute(nxt, __builtin_bit_cast(int, pf[e])));
                const float r1 = __builtin_bit_cast(float, __builtin_amdgcn_ds_bpermute(nxt, __builtin_bit_cast(int, pr[e])));
                if (lane < 63 && j < WL) {
                    const float df = f1 - pf[e];
                    const float db = r1 - pr[e];
                    const float jj = (float)j;
                    win[a * WL + j] = make_float4(fmaf(-jj, df, pf[e]), df, fmaf(-jj, db, pr[e]), db);
                }
            }
        }
    };

    __syncthreads();   // LDS of a previous tile (persistent workgroups) fully consumed
    params(0, 0);
    __syncthreads();
    load(0, 0);
    int buf = 0;
    for (int k0 = 0; k0 < K; k0 += KB, buf ^= 1) {
        const int nb = min(KB, K - k0);
        store(k0);
        if (k0 + KB < K) params(k0 + KB, buf ^ 1);
        __syncthreads();
        if (k0 + KB < K) load(k0 + KB, buf ^ 1);
        // group grp takes the contiguous angles [a_lo, a_hi) of this block
        const int per = (nb + S - 1) / S;
        const int a_lo = min(nb, grp * per);
        const int a_hi = min(nb, a_lo + per);
        const float4* __restrict__ pa = prm + buf * kMaxKB;
#pragma unroll 4
        for (int a = a_lo; a < a_hi; ++a) {
            const float4 p = pa[a];
            const float u0 = fmaf(flx, p.y, fmaf(fly, p.z, p.x));
            const float4* __restrict__ w = win + a * WL;
#pragma unroll
            for (int i = 0; i < P; ++i) {
                const float u = (i == 0) ? u0 : fmaf((float)i, p.z, u0);
                const int j = (int)u;   // u > 0: truncation is floor
                const float4 v = w[j];
                accf[i] += fmaf(u, v.y, v.x);
                accr[i] += fmaf(u, v.w, v.z);
            }
        }
        __syncthreads();
    }

    if constexpr (S > 1) {
        float* red = reinterpret_cast<float*>(win);   // [S-1][256][2P]
        if (grp > 0) {
#pragma unroll
            for (int i = 0; i < P; ++i) {
                red[((grp - 1) * kGroupThreads + tl) * 2 * P + 2 * i] = accf[i];
                red[((grp - 1) * kGroupThreads + tl) * 2 * P + 2 * i + 1] = accr[i];
            }
        }
        __syncthreads();
        if (grp > 0) return;
#pragma unroll
        for (int gg = 1; gg < S; ++gg) {
#pragma unroll
            for (int i = 0; i < P; ++i) {
                accf[i] += red[((gg - 1) * kGroupThreads + tl) * 2 * P + 2 * i];
                accr[i] += red[((gg - 1) * kGroupThreads + tl) * 2 * P + 2 * i + 1];
            }
        }
    }

    // Each pixel of the upper half (and the middle row's left half for odd N) is
    // "primary"; its lane writes it and its reflection.
    const float scale = job.scale;
    const int half_rows = (N + 1) >> 1;
    const int c = c0 + lx;
#pragma unroll
    for (int i = 0; i < P; ++i) {
        const int r = r0 + ly0 + i;
        if (c < N && r < half_rows) {
            const bool mid = (2 * r == N - 1);
            if (!mid || 2 * c <= N - 1) {
                img[(size_t)r * N + c] = accf[i] * scale;
                if (!(mid && 2 * c == N - 1))
                    img[(size_t)(N - 1 - r) * N + (N - 1 - c)] = accr[i] * scale;
            }
        }
    }
}

template <int TW, int P, int S>
__global__ __launch_bounds__(kGroupThreads * S, 2 * S) void bp_grid_kernel(BpJob job, size_t q_stride,
                                                                    size_t img_stride, int tiles_per_slice) {
    extern __shared__ float4 smem4[];
    char* smem = reinterpret_cast<char*>(smem4);
    constexpr int TH = Shape<TW, P, S>::TH;
    const int lb = xcd_logical(blockIdx.x, gridDim.x);
    const int s = lb / tiles_per_slice;
    const int tt = lb - s * tiles_per_slice;
    const int ty = tt / job.tiles_x;
    const int tx = tt - ty * job.tiles_x;
    bp_tile<TW, P, S>(job, job.q + (size_t)s * q_stride, job.img + (size_t)s * img_stride, tx * TW,
                      ty * TH, smem);
}

template <int TW, int P, int S>
__global__ __launch_bounds__(kGroupThreads * S, 2 * S) void bp_list_kernel(const BpListArgs* __restrict__ args) {
    extern __shared__ float4 smem4[];
    char* smem = reinterpret_cast<char*>(smem4);
    const BpListArgs a = load_const(args);
    constexpr int TH = Shape<TW, P, S>::TH;
    const auto* __restrict__ prefix = as_const(a.tile_prefix);
    const int n_sel = *as_const(a.counts);
    if (n_sel <= 0) return;
    const int total = prefix[n_sel];
    const int G = gridDim.x;
    for (int it = xcd_logical(blockIdx.x, G); it < total; it += G) {
        // largest s with tile_prefix[s] <= it (uniform: scalar loads and branches)
        int lo = 0, hi = n_sel - 1;
        while (lo < hi) {
            const int mid = (lo + hi + 1) >> 1;
            if (prefix[mid] <= it) lo = mid; else hi = mid - 1;
        }
        const BpJob job = load_const(a.jobs + as_const(a.job_index)[lo]);
        const int tt = it - prefix[lo];
        const int ty = tt / job.tiles_x;
        const int tx = tt - ty * job.tiles_x;
        bp_tile<TW, P, S>(job, job.q, job.img, tx * TW, ty * TH, smem);
    }
}

constexpr TileShape kShapes[kNumTileConfigs] = {
    {32, 2, 16, 4, "32x16 tile, 2 px/lane, 4 angle groups"},
    {16, 2, 32, 4, "16x32 tile, 2 px/lane, 4 angle groups"},
    {32, 4, 32, 2, "32x32 tile, 4 px/lane, 2 angle groups"},
    {32, 1, 8, 4, "32x8 tile, 1 px/lane, 4 angle groups"},
    {32, 4, 32, 1, "32x32 tile, 4 px/lane, 1 angle group"},
    {16, 2, 32, 2, "16x32 tile, 2 px/lane, 2 angle groups"},
    {32, 2, 16, 1, "32x16 tile, 2 px/lane, 1 angle group"},
    {16, 1, 16, 4, "16x16 tile, 1 px/lane, 4 angle groups"},
    {16, 4, 64, 4, "16x64 tile, 4 px/lane, 4 angle groups"},
};

template <int TW, int P, int S>
hipError_t grid_launch(const BpJob& job, int n_slices, size_t q_stride, size_t img_stride,
                       int tiles_per_slice, size_t lds, hipStream_t stream) {
    const unsigned grid = (unsigned)n_slices * (unsigned)tiles_per_slice;
    hipLaunchKernelGGL((bp_grid_kernel<TW, P, S>), dim3(grid), dim3(kGroupThreads * S), lds, stream,
                       job, q_stride, img_stride, tiles_per_slice);
    return hipGetLastError();
}

template <int TW, int P, int S>
hipError_t list_launch(const BpListArgs* a, int grid, size_t lds, hipStream_t stream) {
    hipLaunchKernelGGL((bp_list_kernel<TW, P, S>), dim3(grid), dim3(kGroupThreads * S), lds, stream, a);
    return hipGetLastError();
}

template <int TW, int P, int S>
int occupancy(size_t lds) {
    int n = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, bp_list_kernel<TW, P, S>, kGroupThreads * S,
                                                     lds) != hipSuccess)
        return 1;
    return n > 0 ? n : 1;
}

template <int TW, int P, int S>
constexpr int red_bytes() { return Shape<TW, P, S>::RED_BYTES; }

#define FBP_FOR_EACH_SHAPE(X) \
    X(0, 32, 2, 4)            \
    X(1, 16, 2, 4)            \
    X(2, 32, 4, 2)            \
    X(3, 32, 1, 4)            \
    X(4, 32, 4, 1)            \
    X(5, 16, 2, 2)            \
    X(6, 32, 2, 1)            \
    X(7, 16, 1, 4)            \
    X(8, 16, 4, 4)

}  // namespace

const TileShape& tile_shape(int cfg) { return kShapes[cfg]; }

int bp_lds_bytes(int cfg, int WL, int KB) {
    int red = 0;
    switch (cfg) {
#define X(id, tw, p, s) case id: red = red_bytes<tw, p, s>(); break;
        FBP_FOR_EACH_SHAPE(X)
#undef X
        default: break;
    }
    const int win = WL * KB * 16;
    return kPrmBytes + (win > red ? win : red);
}

hipError_t launch_bp_grid(int cfg, const BpJob& job, int n_slices, size_t q_stride,
                          size_t img_stride, int tiles_per_slice, hipStream_t stream) {
    const size_t lds = (size_t)bp_lds_bytes(cfg, job.WL, job.KB);
    switch (cfg) {
#define X(id, tw, p, s) \
        case id: return grid_launch<tw, p, s>(job, n_slices, q_stride, img_stride, tiles_per_slice, lds, stream);
        FBP_FOR_EACH_SHAPE(X)
#undef X
        default: return hipErrorInvalidValue;
    }
}

hipError_t launch_bp_list(int cfg, const BpListArgs* a, int grid, size_t lds, hipStream_t stream) {
    switch (cfg) {
#define X(id, tw, p, s) case id: return list_launch<tw, p, s>(a, grid, lds, stream);
        FBP_FOR_EACH_SHAPE(X)
#undef X
        default: return hipErrorInvalidValue;
    }
}

int bp_occupancy(int cfg, size_t lds) {
    switch (cfg) {
#define X(id, tw, p, s) case id: return occupancy<tw, p, s>(lds);
        FBP_FOR_EACH_SHAPE(X)
#undef X
        default: return 1;
    }
}

}  // namespace fbp
