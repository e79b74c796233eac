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
//    the angles k = g (mod S), and the S partial sums are added in fixed order at
//    the end.  This gives a single 512^2 slice enough waves per CU.  Per-angle
//    constants come from LDS (not scalar loads, which would force full LDS drains
//    inside the loop).
//  * For stacks of slices with one geometry, a workgroup can take M = 4 slices of
//    the same tile: the coordinate, its truncation and the LDS address are shared
//    by 2 M pixels, and the window bins of the M slices sit side by side.  Each
//    slice's arithmetic, and the order of its sums, is that of the one-slice
//    kernel of the same tile shape, so the results are bitwise identical.
//  * The next block's filtered rows are loaded into registers while the current
//    block is computed, so the global-load latency hides behind the LDS work.
//    The loads are buffer loads whose range check supplies the zeros beyond the
//    detector ends, so staging has no compares or branches.
//  * Each pixel is written once by one lane; no atomics.  The summation order
//    depends only on the tile shape, which is fixed per geometry, so repeated and
//    batched calls are bitwise identical.
#include <algorithm>

#include "fbp_internal.hpp"

namespace fbp {

namespace {

__device__ __forceinline__ float ld_zero(const float* __restrict__ row, int g, int D) {
    return (g >= 0 && g < D) ? row[g] : 0.0f;
}

// Word 3 of a raw (stride 0) buffer resource: 32-bit data format, no swizzle; reads
// at byte offsets >= num_records return 0.
constexpr int kBufferWord3 = 0x00020000;

// LDS layout: prm[2][kMaxKB] float4 {b, cos/dt, sin/dt, i0 bits} per angle of the
// current and next block, then the window (float4 [KB][WL]), which the final
// cross-group reduction reuses.
constexpr int kPrmBytes = kBpPrmBytes;

template <int TW, int P, int S, bool ROT = false>
struct Shape {
    static constexpr int NT = kGroupThreads * S;
    static constexpr int TH = (kGroupThreads / TW) * P;
    static constexpr int NACC = ROT ? 4 : 2;                      // accumulators per pixel row
    static constexpr int RED_BYTES = (S - 1) * kGroupThreads * NACC * P * 4;
    static constexpr int XPOSE_BYTES = ROT ? 2 * TH * (TW + 1) * 4 : 0;
};

// LDS of the rotation-symmetric shapes: prm float4 {bU, bV, cos/dt, sin/dt} and
// pri int2 {iU0, iV0} for the angle pairs of the current and next block, then the
// windows.
constexpr int kRotPrmBytes = kBpRotPrmBytes;

// The M slices a workgroup backprojects together.  They share the geometry, so one
// coordinate, one truncation and one LDS address serve 2 M pixels.  Entries at
// m >= n repeat slice 0's pointers; their rows are read as zeros and never stored.
template <int M>
struct SliceSet {
    const float* q[M];
    float* img[M];
    int n;   // valid slices, 1 <= n <= M
};

// Window bins of the M slices of one angle are interleaved with a stride of ST
// float4s; an odd stride keeps lanes at consecutive bins on distinct LDS banks.
template <int M>
constexpr int bin_stride() { return (M == 1) ? 1 : (M | 1); }

template <int M>
constexpr int log2_slices() { return M == 1 ? 0 : (M == 2 ? 1 : 2); }

// With job.split = R > 1 the workgroup backprojects only the angles part, part + R,
// part + 2R, ... and stores their unscaled sum (ss.img then points at the part's
// plane of the partial-sum buffer).
template <int TW, int P, int S, int M>
__device__ __forceinline__ void bp_tile(const BpJob& job, const SliceSet<M>& ss, int c0, int r0,
                                        char* smem, int part) {
    static_assert(M == 1 || M == 2 || M == 4, "slices per workgroup");
    using Sh = Shape<TW, P, S>;
    constexpr int NT = Sh::NT;
    constexpr int TH = Sh::TH;
    constexpr int E = stage_elems(S);
    constexpr int ST = bin_stride<M>();
    constexpr int LM = log2_slices<M>();
    constexpr int UB = (8 / (P * M) < 1) ? 1 : (8 / (P * M) > 4 ? 4 : 8 / (P * M));
    float4* prm = reinterpret_cast<float4*>(smem);                      // [2][kMaxKB]
    float4* win = reinterpret_cast<float4*>(smem + kPrmBytes);          // [KB][WL][ST]

    const int t = threadIdx.x;
    const int grp = __builtin_amdgcn_readfirstlane(t >> 8);   // wave-uniform angle group
    const int tl = t & (kGroupThreads - 1);
    const int lx = tl % TW;
    const int ly0 = (tl / TW) * P;
    const int N = job.N, D = job.D, WL = job.WL, KB = job.KB;
    const int split = job.split;
    const int K = (job.K - part + split - 1) / split;   // angles of this workgroup
    const double x0 = (double)c0 - job.half_pix;
    const double y0 = (double)r0 - job.half_pix;
    const float flx = (float)lx;
    const float fly = (float)ly0;

    // Staging: one wave fills one segment of 63 window bins of one (angle, slice)
    // per pass.  Lane j loads bin i0 + 63 seg + j of the forward row and the
    // mirrored bin of the reversed row with single-dword buffer loads; a per-row
    // buffer resource of D floats returns 0 outside the detector, which is the zero
    // extension of the filtered row.  The value at bin + 1 comes from the next lane
    // (ds_bpermute), so 64 lanes produce 63 (A, dL) pairs per direction.
    constexpr int W = NT / 64;                  // waves per workgroup
    const int wave = __builtin_amdgcn_readfirstlane(t >> 6);
    const int lane = t & 63;
    const int seg_shift = job.seg_shift;        // log2(segments per angle)
    const int nxt = ((lane + 1) & 63) << 2;     // ds_bpermute source: lane + 1
    const int d4 = (D - 1) * 4;

    float accf[M][P], accr[M][P];
#pragma unroll
    for (int m = 0; m < M; ++m) {
#pragma unroll
        for (int i = 0; i < P; ++i) {
            accf[m][i] = 0.0f;
            accr[m][i] = 0.0f;
        }
    }

    // window origin (FP64) of the angles of the block starting at kb, into buffer buf
    auto params = [&](int kb, int buf) {
        const int nb = min(KB, K - kb);
        if (t < nb) {
            const int k = part + (kb + t) * split;
            const double cd = job.cs[2 * k];
            const double sd = job.cs[2 * k + 1];
            const double uo = x0 * cd + y0 * sd + job.centre_det;
            const double umin = uo + fmin(0.0, (double)(TW - 1) * cd) + fmin(0.0, (double)(TH - 1) * sd);
            const int i0 = (int)floor(umin) - 1;
            prm[buf * kMaxKB + t] = make_float4((float)(uo - (double)i0), (float)cd, (float)sd,
                                                __int_as_float(i0));
        }
    };
    // angle weights (non-uniform angle lists): staged values are scaled by w_k/(pi/K)
    const float* __restrict__ wscale = job.wscale;
    float pf[E], pr[E];
    auto load = [&](int kb, int buf) {
        const int nslot = min(KB, K - kb) << (LM + seg_shift);
#pragma unroll
        for (int e = 0; e < E; ++e) {
            const int slot = wave + e * W;                       // wave-uniform
            if (slot < nslot) {
                const int a = slot >> (LM + seg_shift);
                const int m = (slot >> seg_shift) & (M - 1);
                const int seg = slot & ((1 << seg_shift) - 1);
                const float* qm = ss.q[0];
#pragma unroll
                for (int mm = 1; mm < M; ++mm)
                    if (m == mm) qm = ss.q[mm];
                const int nrec = (m < ss.n) ? D * 4 : 0;
                const int k = part + (kb + a) * split;
                const __amdgpu_buffer_rsrc_t row = __builtin_amdgcn_make_buffer_rsrc(
                    const_cast<float*>(qm + (size_t)k * (size_t)D), (short)0, nrec, kBufferWord3);
                const int g4 = (__float_as_int(prm[buf * kMaxKB + a].w) + 63 * seg + lane) * 4;
                pf[e] = __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(row, g4, 0, 0));
                pr[e] = __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(row, d4 - g4, 0, 0));
            }
        }
    };
    auto store = [&](int kb) {
        const int nslot = min(KB, K - kb) << (LM + seg_shift);
#pragma unroll
        for (int e = 0; e < E; ++e) {
            const int slot = wave + e * W;
            if (slot < nslot) {
                const int a = slot >> (LM + seg_shift);
                const int m = (slot >> seg_shift) & (M - 1);
                const int j = 63 * (slot & ((1 << seg_shift) - 1)) + lane;
                if (wscale) {   // uniform: the factor is a scalar load
                    const float c = wscale[part + (kb + a) * split];
                    pf[e] *= c;
                    pr[e] *= c;
                }
                const float f1 = __builtin_bit_cast(float, __builtin_amdgcn_ds_bpermute(nxt, __builtin_bit_cast(int, pf[e])));
                const float r1 = __builtin_bit_cast(float, __builtin_amdgcn_ds_bpermute(nxt, __builtin_bit_cast(int, pr[e])));
                if (lane < 63 && j < WL) {
                    const float df = f1 - pf[e];
                    const float db = r1 - pr[e];
                    const float jj = (float)j;
                    win[(a * WL + j) * ST + m] = make_float4(fmaf(-jj, df, pf[e]), df, fmaf(-jj, db, pr[e]), db);
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
        // group grp takes the angles k = grp (mod S): the assignment and the order of
        // each group's sum depend on neither the block length nor M
        const float4* __restrict__ pa = prm + buf * kMaxKB;
        int a = (grp - k0 % S + S) % S;
        // UB angles per step: every window read of the step is issued before the
        // first is consumed, so each wave keeps P M UB (up to 8) LDS reads in flight
        for (; a + (UB - 1) * S < nb; a += UB * S) {
            float4 p[UB];
#pragma unroll
            for (int b = 0; b < UB; ++b) p[b] = pa[a + b * S];
            float u[UB][P];
            float4 v[UB][P][M];
#pragma unroll
            for (int b = 0; b < UB; ++b) {
                const float u0 = fmaf(flx, p[b].y, fmaf(fly, p[b].z, p[b].x));
                const float4* __restrict__ w = win + (a + b * S) * WL * ST;
#pragma unroll
                for (int i = 0; i < P; ++i) {
                    u[b][i] = (i == 0) ? u0 : fmaf((float)i, p[b].z, u0);
                    const float4* __restrict__ wj = w + (int)u[b][i] * ST;   // u > 0: truncation is floor
#pragma unroll
                    for (int m = 0; m < M; ++m) v[b][i][m] = wj[m];
                }
            }
#pragma unroll
            for (int b = 0; b < UB; ++b)
#pragma unroll
                for (int i = 0; i < P; ++i)
#pragma unroll
                    for (int m = 0; m < M; ++m) {
                        accf[m][i] += fmaf(u[b][i], v[b][i][m].y, v[b][i][m].x);
                        accr[m][i] += fmaf(u[b][i], v[b][i][m].w, v[b][i][m].z);
                    }
        }
        for (; a < nb; a += S) {
            const float4 p = pa[a];
            const float u0 = fmaf(flx, p.y, fmaf(fly, p.z, p.x));
            const float4* __restrict__ w = win + a * WL * ST;
#pragma unroll
            for (int i = 0; i < P; ++i) {
                const float u = (i == 0) ? u0 : fmaf((float)i, p.z, u0);
                const float4* __restrict__ wj = w + (int)u * ST;
#pragma unroll
                for (int m = 0; m < M; ++m) {
                    const float4 v = wj[m];
                    accf[m][i] += fmaf(u, v.y, v.x);
                    accr[m][i] += fmaf(u, v.w, v.z);
                }
            }
        }
        __syncthreads();
    }

    if constexpr (S > 1) {
        constexpr int NV = 2 * P * M;                 // partial sums per lane
        float* red = reinterpret_cast<float*>(win);   // [S-1][NV][256]
        if (grp > 0) {
            float* r = red + (grp - 1) * NV * kGroupThreads + tl;
#pragma unroll
            for (int m = 0; m < M; ++m) {
#pragma unroll
                for (int i = 0; i < P; ++i) {
                    r[(2 * (m * P + i)) * kGroupThreads] = accf[m][i];
                    r[(2 * (m * P + i) + 1) * kGroupThreads] = accr[m][i];
                }
            }
        }
        __syncthreads();
        if (grp > 0) return;
#pragma unroll
        for (int gg = 1; gg < S; ++gg) {
            const float* r = red + (gg - 1) * NV * kGroupThreads + tl;
#pragma unroll
            for (int m = 0; m < M; ++m) {
#pragma unroll
                for (int i = 0; i < P; ++i) {
                    accf[m][i] += r[(2 * (m * P + i)) * kGroupThreads];
                    accr[m][i] += r[(2 * (m * P + i) + 1) * kGroupThreads];
                }
            }
        }
    }

    // Each pixel of the upper half (and the middle row's left half for odd N) is
    // "primary"; its lane writes it and its reflection.
    const float scale = (split > 1) ? 1.0f : job.scale;
    const int half_rows = (N + 1) >> 1;
    const int c = c0 + lx;
#pragma unroll
    for (int i = 0; i < P; ++i) {
        const int r = r0 + ly0 + i;
        if (c < N && r < half_rows) {
            const bool mid = (2 * r == N - 1);
            if (!mid || 2 * c <= N - 1) {
                const bool refl = !(mid && 2 * c == N - 1);
#pragma unroll
                for (int m = 0; m < M; ++m) {
                    if (m < ss.n) {
                        ss.img[m][(size_t)r * N + c] = accf[m][i] * scale;
                        if (refl) ss.img[m][(size_t)(N - 1 - r) * N + (N - 1 - c)] = accr[m][i] * scale;
                    }
                }
            }
        }
    }
}


// Rotation-symmetric variant for angle lists closed under +pi/2 (theta_{k+K/2} =
// theta_k + pi/2) and even N.  The workgroup owns a tile T of the top-left image
// quadrant and its three 90-degree rotations.  Rotating a pixel by +90 degrees
// and its angle by +pi/2 leaves the ray coordinate unchanged, so for an angle
// pair (theta, theta + pi/2) the four rotated copies of a pixel need only two
// local coordinates, U = u_theta(p) and V = u_theta(R p):
//     p     : theta fwd at U,   theta+pi/2 rev at V
//     R^2 p : theta rev at U,   theta+pi/2 fwd at V
//     R p   : theta fwd at V,   theta+pi/2 fwd at U
//     R^3 p : theta rev at V,   theta+pi/2 rev at U
// (R(x, y) = (-y, x); "rev" is the reversed filtered row, as for the point
// reflection).  Each window bin holds both angles' forward and reversed (A, dL)
// pairs in two float4 planes (theta, theta + pi/2), so lanes at consecutive bins
// read 16-byte-strided addresses without bank conflicts: 8 updates per 2
// coordinates, 2 truncations, 4 ds_read_b128.
// The eight updates of one angle pair (theta, theta + pi/2) for a pixel and its
// three rotations, from the coordinates U, V and the window bins read at them;
// the theta term first, then theta + pi/2, for every pixel.
__device__ __forceinline__ void rot_accumulate(float u, float v, const float4& qu0, const float4& qu1,
                                               const float4& qv0, const float4& qv1, float& acc0, float& acc1,
                                               float& acc2, float& acc3) {
    acc0 += fmaf(u, qu0.y, qu0.x);
    acc0 += fmaf(v, qv1.w, qv1.z);
    acc2 += fmaf(u, qu0.w, qu0.z);
    acc2 += fmaf(v, qv1.y, qv1.x);
    acc1 += fmaf(v, qv0.y, qv0.x);
    acc1 += fmaf(u, qu1.y, qu1.x);
    acc3 += fmaf(v, qv0.w, qv0.z);
    acc3 += fmaf(u, qu1.w, qu1.z);
}

// With job.split = R > 1 the workgroup takes only the angle pairs part, part + R,
// ... and stores their unscaled sums (img then points at the part's plane).
template <int TW, int P, int S>
__device__ __forceinline__ void bp_tile_rot4(const BpJob& job, const float* __restrict__ q,
                                             float* __restrict__ img, int c0, int r0, char* smem, int part) {
    using Sh = Shape<TW, P, S, true>;
    constexpr int NT = Sh::NT;
    constexpr int TH = Sh::TH;
    constexpr int UB = (4 / P < 1) ? 1 : 4 / P;
    float4* prm = reinterpret_cast<float4*>(smem);                        // [2][kMaxKB]
    int2* pri = reinterpret_cast<int2*>(smem + 2 * kMaxKB * 16);          // [2][kMaxKB]
    float4* win = reinterpret_cast<float4*>(smem + kRotPrmBytes);         // [KB][2][2][WL]

    const int t = threadIdx.x;
    const int grp = __builtin_amdgcn_readfirstlane(t >> 8);
    const int tl = t & (kGroupThreads - 1);
    const int lx = tl % TW;
    const int ly0 = (tl / TW) * P;
    const int N = job.N, D = job.D, WL = job.WL, KB = job.KB;
    const int KH = job.K >> 1;                 // angle pairs (k, k + K/2)
    const int split = job.split;
    const int K2 = (KH - part + split - 1) / split;   // pairs of this workgroup
    const double x0 = (double)c0 - job.half_pix;
    const double y0 = (double)r0 - job.half_pix;
    const float flx = (float)lx;
    const float fly = (float)ly0;
    const float nfly = -fly;

    constexpr int W = NT / 64;
    const int wave = __builtin_amdgcn_readfirstlane(t >> 6);
    const int lane = t & 63;
    const int seg_shift = job.seg_shift;
    const int nxt = ((lane + 1) & 63) << 2;
    const int d4 = (D - 1) * 4;

    float acc0[P], acc1[P], acc2[P], acc3[P];   // p, R p, R^2 p, R^3 p
#pragma unroll
    for (int i = 0; i < P; ++i) {
        acc0[i] = 0.0f;
        acc1[i] = 0.0f;
        acc2[i] = 0.0f;
        acc3[i] = 0.0f;
    }

    auto params = [&](int kb, int buf) {
        const int nb = min(KB, K2 - kb);
        if (t < nb) {
            const int k = part + (kb + t) * split;
            const double cd = job.cs[2 * k];
            const double sd = job.cs[2 * k + 1];
            const double uo = x0 * cd + y0 * sd + job.centre_det;
            const double umin = uo + fmin(0.0, (double)(TW - 1) * cd) + fmin(0.0, (double)(TH - 1) * sd);
            const double vo = x0 * sd - y0 * cd + job.centre_det;
            const double vmin = vo + fmin(0.0, (double)(TW - 1) * sd) + fmin(0.0, -(double)(TH - 1) * cd);
            const int iu = (int)floor(umin) - 1;
            const int iv = (int)floor(vmin) - 1;
            prm[buf * kMaxKB + t] = make_float4((float)(uo - (double)iu), (float)(vo - (double)iv),
                                                (float)cd, (float)sd);
            pri[buf * kMaxKB + t] = make_int2(iu, iv);
        }
    };
    // staging slot = (pair a, window w in {U, V}, 63-bin segment): 4 single-dword
    // buffer loads per lane (forward and reversed row of both angles)
    const float* __restrict__ wscale = job.wscale;   // angle weights / (pi/K), or null
    float pf[kStageE][4];
    auto load = [&](int kb, int buf) {
        const int nslot = min(KB, K2 - kb) << (seg_shift + 1);
#pragma unroll
        for (int e = 0; e < kStageE; ++e) {
            const int slot = wave + e * W;
            if (slot < nslot) {
                const int a = slot >> (seg_shift + 1);
                const int w = (slot >> seg_shift) & 1;
                const int seg = slot & ((1 << seg_shift) - 1);
                const int k = part + (kb + a) * split;
                const __amdgpu_buffer_rsrc_t ra = __builtin_amdgcn_make_buffer_rsrc(
                    const_cast<float*>(q + (size_t)k * (size_t)D), (short)0, D * 4, kBufferWord3);
                const __amdgpu_buffer_rsrc_t rb = __builtin_amdgcn_make_buffer_rsrc(
                    const_cast<float*>(q + (size_t)(k + KH) * (size_t)D), (short)0, D * 4, kBufferWord3);
                const int2 io = pri[buf * kMaxKB + a];
                const int g4 = ((w ? io.y : io.x) + 63 * seg + lane) * 4;
                pf[e][0] = __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(ra, g4, 0, 0));
                pf[e][1] = __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(ra, d4 - g4, 0, 0));
                pf[e][2] = __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(rb, g4, 0, 0));
                pf[e][3] = __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(rb, d4 - g4, 0, 0));
            }
        }
    };
    auto store = [&](int kb) {
        const int nslot = min(KB, K2 - kb) << (seg_shift + 1);
#pragma unroll
        for (int e = 0; e < kStageE; ++e) {
            const int slot = wave + e * W;
            if (slot < nslot) {
                const int a = slot >> (seg_shift + 1);
                const int w = (slot >> seg_shift) & 1;
                const int j = 63 * (slot & ((1 << seg_shift) - 1)) + lane;
                if (wscale) {   // uniform: the factors are scalar loads
                    const int k = part + (kb + a) * split;
                    const float ca = wscale[k], cb = wscale[k + KH];
                    pf[e][0] *= ca;
                    pf[e][1] *= ca;
                    pf[e][2] *= cb;
                    pf[e][3] *= cb;
                }
                float nx[4];
#pragma unroll
                for (int c = 0; c < 4; ++c)
                    nx[c] = __builtin_bit_cast(float, __builtin_amdgcn_ds_bpermute(nxt, __builtin_bit_cast(int, pf[e][c])));
                if (lane < 63 && j < WL) {
                    const float jj = (float)j;
                    float d[4];
#pragma unroll
                    for (int c = 0; c < 4; ++c) d[c] = nx[c] - pf[e][c];
                    float4* dst = win + (a * 2 + w) * 2 * WL + j;
                    dst[0] = make_float4(fmaf(-jj, d[0], pf[e][0]), d[0], fmaf(-jj, d[1], pf[e][1]), d[1]);
                    dst[WL] = make_float4(fmaf(-jj, d[2], pf[e][2]), d[2], fmaf(-jj, d[3], pf[e][3]), d[3]);
                }
            }
        }
    };

    __syncthreads();
    params(0, 0);
    __syncthreads();
    load(0, 0);
    int buf = 0;
    for (int k0 = 0; k0 < K2; k0 += KB, buf ^= 1) {
        const int nb = min(KB, K2 - k0);
        store(k0);
        if (k0 + KB < K2) params(k0 + KB, buf ^ 1);
        __syncthreads();
        if (k0 + KB < K2) load(k0 + KB, buf ^ 1);
        const int per = (nb + S - 1) / S;
        const int a_lo = min(nb, grp * per);
        const int a_hi = min(nb, a_lo + per);
        const float4* __restrict__ pa = prm + buf * kMaxKB;
        // UB angle pairs per step, every window read issued before the first is used
        int a = a_lo;
        for (; a + UB <= a_hi; a += UB) {
            float4 p[UB];
#pragma unroll
            for (int b = 0; b < UB; ++b) p[b] = pa[a + b];    // bU, bV, cos, sin
            float u[UB][P], v[UB][P];
            float4 qu0[UB][P], qu1[UB][P], qv0[UB][P], qv1[UB][P];
#pragma unroll
            for (int b = 0; b < UB; ++b) {
                const float u0 = fmaf(flx, p[b].z, fmaf(fly, p[b].w, p[b].x));
                const float v0 = fmaf(flx, p[b].w, fmaf(nfly, p[b].z, p[b].y));
                const float4* __restrict__ wu = win + (a + b) * 4 * WL;
                const float4* __restrict__ wv = wu + 2 * WL;
#pragma unroll
                for (int i = 0; i < P; ++i) {
                    u[b][i] = (i == 0) ? u0 : fmaf((float)i, p[b].w, u0);
                    v[b][i] = (i == 0) ? v0 : fmaf(-(float)i, p[b].z, v0);
                    const int ju = (int)u[b][i];   // both > 0: truncation is floor
                    const int jv = (int)v[b][i];
                    qu0[b][i] = wu[ju];
                    qu1[b][i] = wu[WL + ju];
                    qv0[b][i] = wv[jv];
                    qv1[b][i] = wv[WL + jv];
                }
            }
#pragma unroll
            for (int b = 0; b < UB; ++b)
#pragma unroll
                for (int i = 0; i < P; ++i)
                    rot_accumulate(u[b][i], v[b][i], qu0[b][i], qu1[b][i], qv0[b][i], qv1[b][i], acc0[i],
                                   acc1[i], acc2[i], acc3[i]);
        }
        for (; a < a_hi; ++a) {
            const float4 p = pa[a];
            const float u0 = fmaf(flx, p.z, fmaf(fly, p.w, p.x));
            const float v0 = fmaf(flx, p.w, fmaf(nfly, p.z, p.y));
            const float4* __restrict__ wu = win + a * 4 * WL;
            const float4* __restrict__ wv = wu + 2 * WL;
#pragma unroll
            for (int i = 0; i < P; ++i) {
                const float uu = (i == 0) ? u0 : fmaf((float)i, p.w, u0);
                const float vv = (i == 0) ? v0 : fmaf(-(float)i, p.z, v0);
                const int ju = (int)uu;
                const int jv = (int)vv;
                rot_accumulate(uu, vv, wu[ju], wu[WL + ju], wv[jv], wv[WL + jv], acc0[i], acc1[i],
                               acc2[i], acc3[i]);
            }
        }
        __syncthreads();
    }

    float* red = reinterpret_cast<float*>(win);
    if constexpr (S > 1) {
        if (grp > 0) {
#pragma unroll
            for (int i = 0; i < P; ++i) {
                float* r = red + ((grp - 1) * kGroupThreads + tl) * 4 * P + 4 * i;
                r[0] = acc0[i];
                r[1] = acc1[i];
                r[2] = acc2[i];
                r[3] = acc3[i];
            }
        }
        __syncthreads();
        if (grp == 0) {
#pragma unroll
            for (int gg = 1; gg < S; ++gg) {
#pragma unroll
                for (int i = 0; i < P; ++i) {
                    const float* r = red + ((gg - 1) * kGroupThreads + tl) * 4 * P + 4 * i;
                    acc0[i] += r[0];
                    acc1[i] += r[1];
                    acc2[i] += r[2];
                    acc3[i] += r[3];
                }
            }
        }
        __syncthreads();   // reduction buffer fully read before the transpose reuses it
    }

    // p and R^2 p store directly; R p and R^3 p go through LDS so the transposed
    // tiles are written row-contiguously.
    const float scale = (split > 1) ? 1.0f : job.scale;
    const int half = N >> 1;
    const int c = c0 + lx;
    float* x1 = red;                                // [TH][TW + 1]
    float* x3 = red + TH * (TW + 1);
    if (grp == 0) {
#pragma unroll
        for (int i = 0; i < P; ++i) {
            const int ly = ly0 + i;
            const int r = r0 + ly;
            if (c < half && r < half) {
                img[(size_t)r * N + c] = acc0[i] * scale;
                img[(size_t)(N - 1 - r) * N + (N - 1 - c)] = acc2[i] * scale;
            }
            x1[ly * (TW + 1) + lx] = acc1[i] * scale;
            x3[ly * (TW + 1) + lx] = acc3[i] * scale;
        }
    }
    __syncthreads();
    if (grp == 0) {
#pragma unroll
        for (int m = 0; m < P; ++m) {
            const int e = tl + m * kGroupThreads;   // e = a * TH + b: column a = lx, row b = ly
            const int a = e / TH, b = e - (e / TH) * TH;
            if (r0 + b < half && c0 + a < half) {
                // R p of tile element (b, a) sits at (c0 + a, N-1-r0-b); R^3 p at (N-1-c0-a, r0 + b)
                img[(size_t)(c0 + a) * N + (N - 1 - r0 - b)] = x1[b * (TW + 1) + a];
                img[(size_t)(N - 1 - c0 - a) * N + (r0 + b)] = x3[b * (TW + 1) + a];
            }
        }
    }
}

template <int TW, int P, int S, bool ROT, int M>
__device__ __forceinline__ void tile_dispatch(const BpJob& job, const SliceSet<M>& ss, int c0, int r0,
                                              char* smem, int part = 0) {
    if constexpr (ROT) {
        static_assert(M == 1, "quarter-turn shapes backproject one slice per workgroup");
        bp_tile_rot4<TW, P, S>(job, ss.q[0], ss.img[0], c0, r0, smem, part);
    } else {
        bp_tile<TW, P, S, M>(job, ss, c0, r0, smem, part);
    }
}

// Resident waves per SIMD asked of the compiler: four (128 VGPRs), so the batched
// window reads (up to 16 float4 per lane) stay in registers while a CU still
// holds 16 waves.
template <int P, int S, bool ROT, int M>
constexpr int min_waves() { return 4; }

// Slices s0 .. s0 + M - 1 of a strided stack (n_total slices in all).
template <int M>
__device__ __forceinline__ SliceSet<M> stack_slices(const BpJob& job, size_t q_stride, size_t img_stride,
                                                    int s0, int n_total) {
    SliceSet<M> ss;
    ss.n = min(M, n_total - s0);
#pragma unroll
    for (int m = 0; m < M; ++m) {
        const size_t s = (size_t)(m < ss.n ? s0 + m : s0);
        ss.q[m] = job.q + s * q_stride;
        ss.img[m] = job.img + s * img_stride;
    }
    return ss;
}

template <int TW, int P, int S, bool ROT, int M>
__global__ __launch_bounds__(kGroupThreads * S, (min_waves<P, S, ROT, M>())) void bp_grid_kernel(
    BpJob job, size_t q_stride, size_t img_stride, int tiles_per_slice, int n_slices) {
    extern __shared__ float4 smem4[];
    char* smem = reinterpret_cast<char*>(smem4);
    constexpr int TH = Shape<TW, P, S, ROT>::TH;
    const int lb = xcd_logical(blockIdx.x, gridDim.x);
    const int sg = lb / tiles_per_slice;     // slice group: slices sg M .. sg M + M - 1
    const int tt = lb - sg * tiles_per_slice;
    const int ty = tt / job.tiles_x;
    const int tx = tt - ty * job.tiles_x;
    if constexpr (M == 1) {
        if (job.split > 1) {
            // block group sg = (slice s, angle part r); the part's plane takes the sums
            const int s = sg / job.split;
            const int r = sg - s * job.split;
            SliceSet<1> ss;
            ss.n = 1;
            ss.q[0] = job.q + (size_t)s * q_stride;
            ss.img[0] = job.part + ((size_t)s * job.split + r) * ((size_t)job.N * job.N);
            tile_dispatch<TW, P, S, ROT, M>(job, ss, tx * TW, ty * TH, smem, r);
            return;
        }
    }
    const SliceSet<M> ss = stack_slices<M>(job, q_stride, img_stride, sg * M, n_slices);
    tile_dispatch<TW, P, S, ROT, M>(job, ss, tx * TW, ty * TH, smem);
}

template <int TW, int P, int S, bool ROT, int M>
__global__ __launch_bounds__(kGroupThreads * S, (min_waves<P, S, ROT, M>())) void bp_list_kernel(
    const BpListArgs* __restrict__ args) {
    extern __shared__ float4 smem4[];
    char* smem = reinterpret_cast<char*>(smem4);
    const BpListArgs a = load_const(args);
    constexpr int TH = Shape<TW, P, S, ROT>::TH;
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
        const int first = as_const(a.job_index)[lo];
        const BpJob job = load_const(a.jobs + first);
        SliceSet<M> ss;
        if constexpr (M == 1) {
            ss.n = 1;
            ss.q[0] = job.q;
            ss.img[0] = job.img;
        } else {
            // a group: jobs first .. first + n - 1 share the geometry
            ss.n = as_const(a.group_size)[lo];
#pragma unroll
            for (int m = 0; m < M; ++m) {
                const BpJob* jm = a.jobs + first + (m < ss.n ? m : 0);
                ss.q[m] = load_const(&jm->q);
                ss.img[m] = load_const(&jm->img);
            }
        }
        const int tt = it - prefix[lo];
        const int ty = tt / job.tiles_x;
        const int tx = tt - ty * job.tiles_x;
        tile_dispatch<TW, P, S, ROT, M>(job, ss, tx * TW, ty * TH, smem);
    }
}

constexpr TileShape kShapes[kNumTileConfigs] = {
    {32, 2, 16, 4, "32x16 tile, 2 px/lane, 4 angle groups"},
    {16, 2, 32, 4, "16x32 tile, 2 px/lane, 4 angle groups"},
    {32, 4, 32, 2, "32x32 tile, 4 px/lane, 2 angle groups; 2-slice stacks", 0, 2},
    {32, 1, 8, 4, "32x8 tile, 1 px/lane, 4 angle groups"},
    {32, 4, 32, 1, "32x32 tile, 4 px/lane, 1 angle group; 2-slice stacks", 0, 2},
    {16, 2, 32, 2, "16x32 tile, 2 px/lane, 2 angle groups; 2-slice stacks", 0, 2},
    {32, 2, 16, 1, "32x16 tile, 2 px/lane, 1 angle group; 4-slice stacks", 0, 4},
    {16, 1, 16, 4, "16x16 tile, 1 px/lane, 4 angle groups"},
    {16, 4, 64, 4, "16x64 tile, 4 px/lane, 4 angle groups"},
    {16, 2, 32, 4, "16x32 quadrant tile x 4 rotations, 2 px/lane, 4 angle groups", 1},
    {16, 1, 16, 4, "16x16 quadrant tile x 4 rotations, 1 px/lane, 4 angle groups", 1},
    {32, 4, 32, 1, "32x32 quadrant tile x 4 rotations, 4 px/lane, 1 angle group", 1},
    {16, 2, 32, 1, "16x32 quadrant tile x 4 rotations, 2 px/lane, 1 angle group", 1},
    {16, 4, 16, kQtChunks, "16x16 quadrant tile x 4 rotations, 4 px/lane, 16 angle chunks (one per wave), 32-bin windows", 2},
    {16, 4, 16, kQtChunks, "16x16 quadrant tile x 4 rotations, 4 px/lane, 16 angle chunks (one per wave), 64-bin windows", 2},
};

template <int TW, int P, int S, bool ROT, int M>
hipError_t grid_launch(const BpJob& job, int n_slices, size_t q_stride, size_t img_stride,
                       int tiles_per_slice, size_t lds, hipStream_t stream) {
    if (job.split > 1 && M > 1) return hipErrorInvalidValue;
    const unsigned groups = (unsigned)((n_slices + M - 1) / M) * (unsigned)(job.split > 1 ? job.split : 1);
    const unsigned grid = groups * (unsigned)tiles_per_slice;
    return launch_kernel(bp_grid_kernel<TW, P, S, ROT, M>, dim3(grid), dim3(kGroupThreads * S), lds, stream, job,
                         q_stride, img_stride, tiles_per_slice, n_slices);
}

template <int TW, int P, int S, bool ROT, int M>
hipError_t list_launch(const BpListArgs* a, int grid, size_t lds, hipStream_t stream) {
    return launch_kernel(bp_list_kernel<TW, P, S, ROT, M>, dim3(grid), dim3(kGroupThreads * S), lds, stream, a);
}

template <int TW, int P, int S, bool ROT, int M>
int occupancy(size_t lds) {
    int n = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, bp_list_kernel<TW, P, S, ROT, M>, kGroupThreads * S,
                                                     lds) != hipSuccess)
        return 1;
    return n > 0 ? n : 1;
}

// LDS bytes of the cross-group reduction (and of the quarter-turn transpose).
template <int TW, int P, int S, bool ROT, int M>
constexpr int red_bytes() {
    using Sh = Shape<TW, P, S, ROT>;
    return Sh::RED_BYTES * M > Sh::XPOSE_BYTES ? Sh::RED_BYTES * M : Sh::XPOSE_BYTES;
}

// Every compiled kernel: (tile id, TW, P, S, quarter-turn, slices per workgroup).
#define FBP_FOR_EACH_KERNEL(X)   \
    X(0, 32, 2, 4, false, 1)     \
    X(1, 16, 2, 4, false, 1)     \
    X(2, 32, 4, 2, false, 1)     \
    X(2, 32, 4, 2, false, 2)     \
    X(3, 32, 1, 4, false, 1)     \
    X(4, 32, 4, 1, false, 1)     \
    X(4, 32, 4, 1, false, 2)     \
    X(5, 16, 2, 2, false, 1)     \
    X(5, 16, 2, 2, false, 2)     \
    X(6, 32, 2, 1, false, 1)     \
    X(6, 32, 2, 1, false, 4)     \
    X(7, 16, 1, 4, false, 1)     \
    X(8, 16, 4, 4, false, 1)     \
    X(9, 16, 2, 4, true, 1)      \
    X(10, 16, 1, 4, true, 1)     \
    X(11, 32, 4, 1, true, 1)     \
    X(12, 16, 2, 1, true, 1)

constexpr int kernel_key(int cfg, int m) { return cfg * 8 + m; }

}  // namespace

const TileShape& tile_shape(int cfg) { return kShapes[cfg]; }

int bp_lds_bytes(int cfg, int m, int WL, int KB) {
    if (cfg == kQtCfg32 || cfg == kQtCfg64) return m == 1 ? 0 : -1;   // static LDS
    int red = -1;
    switch (kernel_key(cfg, m)) {
#define X(id, tw, p, s, rot, mm) case kernel_key(id, mm): red = red_bytes<tw, p, s, rot, mm>(); break;
        FBP_FOR_EACH_KERNEL(X)
#undef X
        default: break;
    }
    if (red < 0) return -1;
    if (tile_shape(cfg).rot) {
        const int win = WL * KB * 64;
        return kRotPrmBytes + (win > red ? win : red);
    }
    const int st = (m == 1) ? 1 : (m | 1);
    const int win = WL * KB * 16 * st;
    return kPrmBytes + (win > red ? win : red);
}

hipError_t launch_bp_grid(int cfg, int m, const BpJob& job, int n_slices, size_t q_stride,
                          size_t img_stride, int tiles_per_slice, hipStream_t stream) {
    if (cfg == kQtCfg32 || cfg == kQtCfg64) {
        if (m != 1 || job.split > 1) return hipErrorInvalidValue;
        return launch_bp_qt_grid(job, n_slices, q_stride, img_stride, tiles_per_slice, stream);
    }
    const int lds = bp_lds_bytes(cfg, m, job.WL, job.KB);
    if (lds < 0) return hipErrorInvalidValue;
    switch (kernel_key(cfg, m)) {
#define X(id, tw, p, s, rot, mm)                                                                              \
        case kernel_key(id, mm):                                                                              \
            return grid_launch<tw, p, s, rot, mm>(job, n_slices, q_stride, img_stride, tiles_per_slice,     \
                                                  (size_t)lds, stream);
        FBP_FOR_EACH_KERNEL(X)
#undef X
        default: return hipErrorInvalidValue;
    }
}

hipError_t launch_bp_list(int cfg, int m, const BpListArgs* a, int grid, size_t lds, hipStream_t stream) {
    if (cfg == kQtCfg32 || cfg == kQtCfg64)
        return m == 1 ? launch_bp_qt_list(cfg == kQtCfg32 ? 32 : 64, a, grid, stream) : hipErrorInvalidValue;
    switch (kernel_key(cfg, m)) {
#define X(id, tw, p, s, rot, mm) case kernel_key(id, mm): return list_launch<tw, p, s, rot, mm>(a, grid, lds, stream);
        FBP_FOR_EACH_KERNEL(X)
#undef X
        default: return hipErrorInvalidValue;
    }
}

// Fixed-order sum of the angle parts, four pixels per thread (float4 loads, the
// parts read in order 0 .. R-1, coalesced across the wave); plane % 4 == 0.
__global__ __launch_bounds__(256) void combine_parts_kernel(const float4* __restrict__ part, float4* __restrict__ img,
                                                           int R, size_t plane4, size_t total4, float scale) {
    for (size_t i = (size_t)blockIdx.x * 256 + threadIdx.x; i < total4; i += (size_t)gridDim.x * 256) {
        const size_t s = i / plane4;
        const size_t p = i - s * plane4;
        const float4* src = part + s * (size_t)R * plane4 + p;
        float4 v[kMaxSplit];   // every part's load in flight before the first add
#pragma unroll
        for (int r = 0; r < kMaxSplit; ++r)
            if (r < R) v[r] = src[(size_t)r * plane4];
        float4 acc = v[0];
#pragma unroll
        for (int r = 1; r < kMaxSplit; ++r) {
            if (r < R) {
                acc.x += v[r].x;
                acc.y += v[r].y;
                acc.z += v[r].z;
                acc.w += v[r].w;
            }
        }
        img[i] = make_float4(acc.x * scale, acc.y * scale, acc.z * scale, acc.w * scale);
    }
}

// The same for planes of any size, one pixel per thread.
__global__ __launch_bounds__(256) void combine_parts_kernel_1(const float* __restrict__ part, float* __restrict__ img,
                                                             int R, size_t plane, size_t total, float scale) {
    for (size_t i = (size_t)blockIdx.x * 256 + threadIdx.x; i < total; i += (size_t)gridDim.x * 256) {
        const size_t s = i / plane;
        const size_t p = i - s * plane;
        const float* src = part + s * (size_t)R * plane + p;
        float acc = src[0];
        for (int r = 1; r < R; ++r) acc += src[(size_t)r * plane];
        img[i] = acc * scale;
    }
}

hipError_t launch_combine_parts(const float* part, float* img, int n_slices, int R, size_t plane,
                                float scale, hipStream_t stream) {
    const size_t total = (size_t)n_slices * plane;
    if (total == 0) return hipSuccess;
    const bool vec = (plane % 4 == 0) && (reinterpret_cast<uintptr_t>(part) % 16 == 0) &&
                     (reinterpret_cast<uintptr_t>(img) % 16 == 0);
    if (vec) {
        const size_t total4 = total / 4;
        const size_t blocks = std::min<size_t>((total4 + 255) / 256, 8192);
        return launch_kernel(combine_parts_kernel, dim3((unsigned)blocks), dim3(256), 0, stream,
                             reinterpret_cast<const float4*>(part), reinterpret_cast<float4*>(img), R, plane / 4,
                             total4, scale);
    }
    const size_t blocks = std::min<size_t>((total + 255) / 256, 8192);
    return launch_kernel(combine_parts_kernel_1, dim3((unsigned)blocks), dim3(256), 0, stream, part, img, R, plane,
                         total, scale);
}

int bp_occupancy(int cfg, int m, size_t lds) {
    if (cfg == kQtCfg32 || cfg == kQtCfg64) return 1;   // one 16-wave workgroup per CU
    switch (kernel_key(cfg, m)) {
#define X(id, tw, p, s, rot, mm) case kernel_key(id, mm): return occupancy<tw, p, s, rot, mm>(lds);
        FBP_FOR_EACH_KERNEL(X)
#undef X
        default: return 1;
    }
}

}  // namespace fbp
