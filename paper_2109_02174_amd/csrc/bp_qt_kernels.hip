// Quarter-turn backprojection with one contiguous angle chunk per wave.
//
// Computes Eq. 2 of arXiv 2109.02174 (section "Computed tomography") with the
// pi/K weight (or per-angle weights) and linear interpolation, for angle lists
// closed under +pi/2 (theta_{k+K/2} = theta_k + pi/2) and N >= 2:
//     img[r][c] = w * sum_k Q~_k(u_k),  u_k = (x_c cos th_k + y_r sin th_k)/dt + (D-1)/2.
//
// Design:
//  * A workgroup of 16 waves owns a 16 x 16 tile T of the top-left image quadrant
//    and its three 90-degree turns (1024 pixels).  The quadrant is rows [0, N/2)
//    by columns [0, (N+1)/2): for odd N a pinwheel piece, whose four turns cover
//    every pixel but the centre, which the slice's first tile adds on its own.  Rotating a pixel by +90 degrees
//    and its angle by +pi/2 leaves the ray coordinate unchanged, so for an angle
//    pair (theta, theta + pi/2) the four turned copies of a pixel need two local
//    coordinates, U (the tile) and V (its turn), for eight updates.
//  * Every wave covers the whole tile (lane: one column, four rows) and takes one
//    contiguous chunk of the K/2 angle pairs: wave w sums pairs
//    [w K/32, (w+1) K/32) in ascending order, from zero.  The 16 chunk sums are
//    added in wave order at the end through LDS.  The summation order therefore
//    depends on K alone, and the same kernel serves single slices, stacks and
//    batches, which so give bitwise-equal images.
//  * Each wave stages its own windows in its own LDS region, so the main loop has
//    no workgroup barrier: a wave synchronises only with itself (LDS operations
//    of one wave complete in order).  Per pair it stages the window of bins the
//    tile sees at theta and at theta + pi/2 (U) and the same for the turned tile
//    (V); a window bin j holds (A_j, dL_j) for the forward and the reversed row,
//    dL_j = L[j+1] - L[j] and A_j = L[j] - j dL_j, so the interpolated value at
//    local coordinate u in [j, j+1) is A_j + u dL_j (one FMA, no fraction).
//  * Windows have a fixed pitch of WP bins (a template parameter), so one address
//    register per coordinate serves the four 16-byte reads of a pair (immediate
//    offsets for the second plane, the turned window and the next pair).
//  * Per (tile, pair) the window origin is FP64 (from the tile's corner bounds);
//    lanes work in FP32 coordinates local to it.  The window starts one bin below
//    the tile's smallest coordinate, so local coordinates are positive and
//    truncation is floor.
//  * The next block's filtered rows are loaded into registers while the current
//    block is computed, with buffer loads whose range check supplies the zeros
//    beyond the detector ends.
//  * Each pixel is written once by one thread; no atomics.
#include <algorithm>

#include "fbp_internal.hpp"

namespace fbp {

namespace {

constexpr int kWaves = kQtChunks;     // angle chunks = waves per workgroup
constexpr int kThreads = 64 * kWaves;
constexpr int kTile = kQtTile;        // quadrant tile width
constexpr int kTileH = kQtTileH;      // quadrant tile height
constexpr int kRows = kQtRows;        // rows per lane: 64 lanes x kRows rows = kTile x kTileH
constexpr int kBufferWord3 = 0x00020000;
constexpr int kPartPitch = kTile + 1; // row pitch of the chunk sums in LDS
// Resident waves per SIMD asked of the compiler: four (one 16-wave workgroup per CU;
// two rows per lane with twice the waves measured 30% slower).
constexpr int kWavesPerSimd = 4;

__device__ __forceinline__ void wave_sync() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// Angle pairs whose window origins a wave makes at once (one per lane).
constexpr int kRound = 64;

// LDS of a workgroup: per wave, the constants of a round of pairs (float4 + int2
// per pair) and B pairs x 4 planes x WP bins of float4; after the 16 wave regions,
// the chunk sums [wave][turn][row][kPartPitch], in a region of their own so that a
// workgroup that runs several tiles loads its next tile's first windows while the
// current tile's chunk sums are added.
// SEP = false (a workgroup per tile): the chunk sums reuse the window regions.
template <int WP, int B, bool SEP>
struct QtLds {
    static constexpr int PRM = kRound * 24;
    static constexpr int REGION = PRM + B * 4 * WP * 16;
    static constexpr int WINDOWS = kWaves * REGION;
    static constexpr int PARTS = kWaves * 4 * kTileH * kPartPitch * 4;
    static constexpr int PARTS_AT = SEP ? WINDOWS : 0;
    static constexpr int BYTES = SEP ? WINDOWS + PARTS : (WINDOWS > PARTS ? WINDOWS : PARTS);
};
static_assert(QtLds<32, 2, true>::BYTES <= 160 * 1024 && QtLds<64, 1, true>::BYTES <= 160 * 1024, "LDS");

// The eight updates of one angle pair (theta, theta + pi/2) for a pixel p and its
// turns R p, R^2 p, R^3 p (R(x, y) = (-y, x)), from the coordinates U = u_theta(p)
// and V = u_theta(R p) and the window bins read there; "rev" is the reversed row
// (the point reflection R^2 p reads it at the same local coordinate):
//     p     : theta fwd at U,   theta+pi/2 rev at V
//     R p   : theta fwd at V,   theta+pi/2 fwd at U
//     R^2 p : theta rev at U,   theta+pi/2 fwd at V
//     R^3 p : theta rev at V,   theta+pi/2 rev at U
// The theta term is added first, then the theta + pi/2 term.
__device__ __forceinline__ void pair_update(float u, float v, const float4& qu0, const float4& qu1,
                                            const float4& qv0, const float4& qv1, float& a0, float& a1,
                                            float& a2, float& a3) {
    a0 += fmaf(u, qu0.y, qu0.x);
    a0 += fmaf(v, qv1.w, qv1.z);
    a2 += fmaf(u, qu0.w, qu0.z);
    a2 += fmaf(v, qv1.y, qv1.x);
    a1 += fmaf(v, qv0.y, qv0.x);
    a1 += fmaf(u, qu1.y, qu1.x);
    a3 += fmaf(v, qv0.w, qv0.z);
    a3 += fmaf(u, qu1.w, qu1.z);
}

// One tile of one slice: the slice's rows ([K][D]) and image ([N][N]), the fields
// of its job the kernel reads (by value: a pointer to a kernel argument would put
// the argument in private memory), and the top-left corner (c0, r0) of the
// quadrant tile.
struct QtTile {
    const float* q;
    float* img;
    const double* cs;
    const float* wscale;
    double half_pix, centre_det;
    float scale;
    int N, K, D, c0, r0;
};

__device__ __forceinline__ void set_job(QtTile& tl, const BpJob& job) {
    tl.cs = job.cs;
    tl.wscale = job.wscale;
    tl.half_pix = job.half_pix;
    tl.centre_det = job.centre_det;
    tl.scale = job.scale;
    tl.N = job.N;
    tl.K = job.K;
    tl.D = job.D;
}

// Backprojects the tiles next() hands out, one after another (one for a single
// slice's grid), each exactly as a workgroup of its own would: the summation order
// depends on the tile's geometry alone.  While a tile's chunk sums are added, the
// window origins and first rows of the next tile are already loading.  smem holds
// QtLds<WP, B, SEP>::BYTES; without SEP next() must hand out one tile only.  WSM: 0
// no job has per-angle weights, 1 every job has them, 2 either (a separate
// instantiation keeps the uniform path free of the weights' scalar loads, which
// would otherwise order the staging's LDS operations).
template <int WP, int B, int WSM, bool SEP, class Next>
__device__ __forceinline__ void qt_run(Next next, char* smem) {
    using L = QtLds<WP, B, SEP>;
    constexpr int WPASS = 64 / WP;            // windows staged per pass of the wave
    constexpr int NPASS = 2 * B / WPASS;      // passes per block (two windows per pair)
    static_assert(WPASS >= 1 && NPASS * WPASS == 2 * B, "staging passes");

    const int t = threadIdx.x;
    const int wave = __builtin_amdgcn_readfirstlane(t >> 6);
    const int lane = t & 63;
    char* region = smem + wave * L::REGION;
    float4* prm = reinterpret_cast<float4*>(region);                // [kRound] {bU, bV, cos/dt, sin/dt}
    int2* pri = reinterpret_cast<int2*>(region + kRound * 16);      // [kRound] {iU, iV}
    float4* win = reinterpret_cast<float4*>(region + L::PRM);       // [B][4][WP]
    float* part = reinterpret_cast<float*>(smem + L::PARTS_AT);     // [wave][turn][row][kPartPitch]

    const int lx = lane & (kTile - 1);
    const int ly0 = (lane >> 4) * kRows;
    const float flx = (float)lx;
    const float fly = (float)ly0;
    const float nfly = -fly;
    const int jl = lane & (WP - 1);             // window bin of this lane when staging
    const int wl = (WPASS == 2) ? (lane >> 5) : 0;

    // the tile's values every phase uses; wave w sums the pairs [lo, hi)
    struct Vals {
        QtTile tl;
        int KH, lo, hi, n, d4;
        double x0, y0;
    };
    auto vals = [&](const QtTile& tl) {
        Vals v;
        v.tl = tl;
        v.KH = tl.K >> 1;
        v.lo = (int)(((long long)wave * v.KH) / kWaves);
        v.hi = (int)(((long long)(wave + 1) * v.KH) / kWaves);
        v.n = v.hi - v.lo;
        v.d4 = (tl.D - 1) * 4;
        v.x0 = (double)tl.c0 - tl.half_pix;
        v.y0 = (double)tl.r0 - tl.half_pix;
        return v;
    };

    float acc0[kRows], acc1[kRows], acc2[kRows], acc3[kRows];
    auto zero = [&]() {
#pragma unroll
        for (int i = 0; i < kRows; ++i) {
            acc0[i] = 0.0f;
            acc1[i] = 0.0f;
            acc2[i] = 0.0f;
            acc3[i] = 0.0f;
        }
    };

    // window origins (FP64) of the pairs lo + rs .. lo + rs + 63 of a round, one per lane
    auto params = [&](const Vals& v, int rs) {
        const int k = v.lo + rs + lane;
        if (k < v.hi) {
            const double cd = v.tl.cs[2 * k];
            const double sd = v.tl.cs[2 * k + 1];
            const double uo = v.x0 * cd + v.y0 * sd + v.tl.centre_det;
            const double umin = uo + fmin(0.0, (double)(kTile - 1) * cd) + fmin(0.0, (double)(kTileH - 1) * sd);
            const double vo = v.x0 * sd - v.y0 * cd + v.tl.centre_det;
            const double vmin = vo + fmin(0.0, (double)(kTile - 1) * sd) + fmin(0.0, -(double)(kTileH - 1) * cd);
            const int iu = (int)floor(umin) - 1;
            const int iv = (int)floor(vmin) - 1;
            prm[lane] = make_float4((float)(uo - (double)iu), (float)(vo - (double)iv), (float)cd, (float)sd);
            pri[lane] = make_int2(iu, iv);
        }
    };
    // staging: pass ps covers windows ps*WPASS .. ps*WPASS + WPASS - 1 (window s =
    // 2 b + w: pair b, w = 0 the tile's window U, w = 1 the turned tile's V); each
    // lane loads one bin and the next of the forward and reversed rows at theta and
    // theta + pi/2 (the next bin from memory rather than from the next lane: the
    // kernel is bound by LDS instructions, and this takes four per pair off them)
    float pf[NPASS][4], pn[NPASS][4];
    // The neighbour's byte offset is formed from an opaque 4, so the compiler does not
    // fuse a bin's load and its neighbour's into one two-dword load: that load's range
    // check would return zero for both when only the neighbour is off the detector.
    int four;
    asm volatile("v_mov_b32 %0, 4" : "=v"(four));
    // kb: first pair of the block within the round (lo + rnd + kb overall)
    int rnd = 0;
    auto load = [&](const Vals& v, int kb, int nr) {
        const int nb = min(B, nr - kb);
        const int D = v.tl.D;
#pragma unroll
        for (int ps = 0; ps < NPASS; ++ps) {
            const int s0 = ps * WPASS;            // first window of the pass (uniform)
            const int b = s0 >> 1;                // pair (uniform: a pass never spans two pairs)
            if (b < nb) {
                const int w = (WPASS == 2) ? wl : (s0 & 1);
                const int k = v.lo + rnd + kb + b;
                const __amdgpu_buffer_rsrc_t ra = __builtin_amdgcn_make_buffer_rsrc(
                    const_cast<float*>(v.tl.q + (size_t)k * (size_t)D), (short)0, D * 4, kBufferWord3);
                const __amdgpu_buffer_rsrc_t rb = __builtin_amdgcn_make_buffer_rsrc(
                    const_cast<float*>(v.tl.q + (size_t)(k + v.KH) * (size_t)D), (short)0, D * 4, kBufferWord3);
                const int2 io = pri[kb + b];
                const int g4 = ((w ? io.y : io.x) + jl) * 4;
                pf[ps][0] = __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(ra, g4, 0, 0));
                pf[ps][1] = __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(ra, v.d4 - g4, 0, 0));
                pf[ps][2] = __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(rb, g4, 0, 0));
                pf[ps][3] = __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(rb, v.d4 - g4, 0, 0));
                const int gn = g4 + four, dn = v.d4 - g4 - four;
                pn[ps][0] = __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(ra, gn, 0, 0));
                pn[ps][1] = __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(ra, dn, 0, 0));
                pn[ps][2] = __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(rb, gn, 0, 0));
                pn[ps][3] = __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(rb, dn, 0, 0));
            }
        }
    };
    auto store = [&](const Vals& v, int kb, int nr) {
        const int nb = min(B, nr - kb);
        float nx[NPASS][4];
#pragma unroll
        for (int ps = 0; ps < NPASS; ++ps) {
            const int b = (ps * WPASS) >> 1;
            if (b < nb) {
                bool ws = WSM == 1;
                if constexpr (WSM == 2) ws = v.tl.wscale != nullptr;
                if (WSM != 0 && ws) {   // angle weights / (pi/K): scalar loads
                    const float* __restrict__ wscale = v.tl.wscale;
                    const int k = v.lo + rnd + kb + b;
                    const float ca = wscale[k], cb = wscale[k + v.KH];
                    pf[ps][0] *= ca;
                    pf[ps][1] *= ca;
                    pf[ps][2] *= cb;
                    pf[ps][3] *= cb;
                    pn[ps][0] *= ca;
                    pn[ps][1] *= ca;
                    pn[ps][2] *= cb;
                    pn[ps][3] *= cb;
                }
#pragma unroll
                for (int c = 0; c < 4; ++c) nx[ps][c] = pn[ps][c];
            }
        }
        const float jj = (float)jl;
#pragma unroll
        for (int ps = 0; ps < NPASS; ++ps) {
            const int s0 = ps * WPASS;
            const int b = s0 >> 1;
            if (b < nb) {
                const int w = (WPASS == 2) ? wl : (s0 & 1);
                float d[4];
#pragma unroll
                for (int c = 0; c < 4; ++c) d[c] = nx[ps][c] - pf[ps][c];
                float4* dst = win + (b * 4 + w * 2) * WP + jl;
                dst[0] = make_float4(fmaf(-jj, d[0], pf[ps][0]), d[0], fmaf(-jj, d[1], pf[ps][1]), d[1]);
                dst[WP] = make_float4(fmaf(-jj, d[2], pf[ps][2]), d[2], fmaf(-jj, d[3], pf[ps][3]), d[3]);
            }
        }
    };
    auto compute = [&](int kb, int nr) {
        const int nb = min(B, nr - kb);
#pragma unroll
        for (int b = 0; b < B; ++b) {
            if (b < nb) {
                // raised priority while the pair's window reads are issued, so that
                // waves queue their reads early and do their updates in the shadow
                // of other waves' reads
                __builtin_amdgcn_sched_barrier(0);
                __builtin_amdgcn_s_setprio(3);
                const float4 p = prm[kb + b];    // bU, bV, cos, sin
                const float u0 = fmaf(flx, p.z, fmaf(fly, p.w, p.x));
                const float v0 = fmaf(flx, p.w, fmaf(nfly, p.z, p.y));
                const float4* __restrict__ wu = win + b * 4 * WP;
                const float4* __restrict__ wv = wu + 2 * WP;
                float u[kRows], v[kRows];
                float4 qu0[kRows], qu1[kRows], qv0[kRows], qv1[kRows];
#pragma unroll
                for (int i = 0; i < kRows; ++i) {
                    u[i] = (i == 0) ? u0 : fmaf((float)i, p.w, u0);
                    v[i] = (i == 0) ? v0 : fmaf(-(float)i, p.z, v0);
                    const int ju = (int)u[i];   // both > 0: truncation is floor
                    const int jv = (int)v[i];
                    qu0[i] = wu[ju];
                    qu1[i] = wu[WP + ju];
                    qv0[i] = wv[jv];
                    qv1[i] = wv[WP + jv];
                }
                __builtin_amdgcn_sched_barrier(0);
                __builtin_amdgcn_s_setprio(0);
#pragma unroll
                for (int i = 0; i < kRows; ++i)
                    pair_update(u[i], v[i], qu0[i], qu1[i], qv0[i], qv1[i], acc0[i], acc1[i], acc2[i], acc3[i]);
            }
        }
    };
    // the first round's window origins and the first block's rows of a tile
    auto begin = [&](const Vals& v) {
        rnd = 0;
        if (v.n > 0) {
            params(v, 0);
            wave_sync();
            load(v, 0, min(kRound, v.n));
        }
    };

    QtTile tile;
    if (!next(tile)) return;
    Vals cur = vals(tile);
    zero();
    begin(cur);
    for (;;) {
        // rounds of up to kRound pairs (one for K <= 2048): the window origins of the
        // round, then blocks of B pairs, the next block's rows loaded during the
        // current (the first round's origins and rows were started by begin)
        for (rnd = 0; rnd < cur.n; rnd += kRound) {
            const int nr = min(kRound, cur.n - rnd);
            if (rnd > 0) {
                params(cur, rnd);
                wave_sync();
                load(cur, 0, nr);
            }
            for (int kb = 0; kb < nr; kb += B) {
                store(cur, kb, nr);
                wave_sync();
                if (kb + B < nr) load(cur, kb + B, nr);
                compute(kb, nr);
                wave_sync();
            }
        }

        // chunk sums through LDS, added in wave order; each output written once
        // every thread is done adding the previous tile's chunk sums (and, when the sums
        // reuse the window regions, every wave is done with its windows)
        __syncthreads();
#pragma unroll
        for (int i = 0; i < kRows; ++i) {
            float* pp = part + ((wave * 4) * kTileH + ly0 + i) * kPartPitch + lx;
            pp[0 * kTileH * kPartPitch] = acc0[i];
            pp[1 * kTileH * kPartPitch] = acc1[i];
            pp[2 * kTileH * kPartPitch] = acc2[i];
            pp[3 * kTileH * kPartPitch] = acc3[i];
        }
        const bool more = SEP && next(tile);
        Vals nxt;
        if (more) {   // the next tile's first windows load while these sums are added
            nxt = vals(tile);
            zero();
            begin(nxt);
        }
        __syncthreads();
        const int N = cur.tl.N;
        const int turn = t >> 8;       // 0: p, 1: R p, 2: R^2 p, 3: R^3 p
        const int e = t & 255;         // tile element (threads past kTile * kTileH idle)
        // p and R^2 p run along tile rows, R p and R^3 p along tile columns, so that
        // consecutive threads write consecutive image addresses
        const int ty = (turn & 1) ? (e % kTileH) : (e / kTile);
        const int tx = (turn & 1) ? (e / kTileH) : (e % kTile);
        const float* src = part + (turn * kTileH + ty) * kPartPitch + tx;
        float sum = 0.0f;
#pragma unroll
        for (int w = 0; w < kWaves; ++w) sum += src[w * 4 * kTileH * kPartPitch];
        // the base region: rows [0, N/2), columns [0, (N+1)/2) (for odd N a pinwheel
        // quadrant: its four turns cover every pixel but the centre)
        const int r = cur.tl.r0 + ty, c = cur.tl.c0 + tx;
        if (e < kTile * kTileH && r < (N >> 1) && c < ((N + 1) >> 1)) {
            size_t o;
            if (turn == 0) o = (size_t)r * N + c;
            else if (turn == 1) o = (size_t)c * N + (N - 1 - r);
            else if (turn == 2) o = (size_t)(N - 1 - r) * N + (N - 1 - c);
            else o = (size_t)(N - 1 - c) * N + r;
            cur.tl.img[o] = sum * cur.tl.scale;
        }
        // odd N: the centre pixel (x = y = 0, so u = (D-1)/2 on every angle), summed by
        // wave 0 of the workgroup that owns the slice's first tile over all K angles in
        // a fixed order (lane l takes angles l, l + 64, ...; then a fixed butterfly)
        if ((N & 1) && cur.tl.r0 == 0 && cur.tl.c0 == 0 && wave == 0) {
            const int D = cur.tl.D, K = cur.tl.K, jc = (D - 1) >> 1;
            const bool between = (D & 1) == 0;          // (D-1)/2 midway between bins jc and jc + 1
            const float* __restrict__ wsc = cur.tl.wscale;
            float csum = 0.0f;
            for (int k = lane; k < K; k += 64) {
                const float* __restrict__ row = cur.tl.q + (size_t)k * D;
                float v = between ? 0.5f * (row[jc] + row[jc + 1]) : row[jc];
                if (WSM != 0 && wsc) v *= wsc[k];
                csum += v;
            }
#pragma unroll
            for (int o = 32; o > 0; o >>= 1) csum += __shfl_xor(csum, o);
            if (lane == 0) cur.tl.img[(size_t)(N >> 1) * N + (N >> 1)] = csum * cur.tl.scale;
        }
        if (!more) break;
        cur = nxt;
    }
}

// Grid form over n slices of one geometry (tiles_per_slice each).  PERSIST = false:
// a workgroup per tile, blocks mapped to tiles XCD-aware.  PERSIST: a smaller grid
// of persistent workgroups, each XCD taking a contiguous range of tiles (whole
// slices of a stack, which share an L2) split among its workgroups.
template <int WP, int B, bool WS, bool PERSIST>
__global__ __launch_bounds__(kThreads, kWavesPerSimd) void bp_qt_grid_kernel(BpJob job, size_t q_stride, size_t img_stride,
                                                              int tiles_per_slice, int total) {
    __shared__ __attribute__((aligned(16))) char smem[QtLds<WP, B, PERSIST>::BYTES];
    const int G = gridDim.x, b = blockIdx.x;
    int it, end, step;
    if (!PERSIST || G >= total) {
        it = xcd_logical(b, G);
        end = it + 1;
        step = 1;
    } else if ((G & 7) == 0) {
        const int x = b & 7, per = G >> 3;
        it = (int)(((long long)x * total) >> 3) + (b >> 3);
        end = (int)(((long long)(x + 1) * total) >> 3);
        step = per;
    } else {
        it = b;
        end = total;
        step = G;
    }
    auto next = [&](QtTile& tl) {
        if (it >= end) return false;
        const int s = it / tiles_per_slice;
        const int tt = it - s * tiles_per_slice;
        const int ty = tt / job.tiles_x;
        const int tx = tt - ty * job.tiles_x;
        set_job(tl, job);
        tl.q = job.q + (size_t)s * q_stride;
        tl.img = job.img + (size_t)s * img_stride;
        tl.c0 = tx * kTile;
        tl.r0 = ty * kTileH;
        it += step;
        return true;
    };
    qt_run<WP, B, WS ? 1 : 0, PERSIST>(next, smem);
}

// Persistent form over a mixed list (same arguments as the other list kernels):
// tile index -> job by binary search in the tile prefix; one job per slice.
template <int WP, int B>
__global__ __launch_bounds__(kThreads, kWavesPerSimd) void bp_qt_list_kernel(const BpListArgs* __restrict__ args) {
    __shared__ __attribute__((aligned(16))) char smem[QtLds<WP, B, true>::BYTES];
    const BpListArgs a = load_const(args);
    const auto* __restrict__ prefix = as_const(a.tile_prefix);
    const int n_sel = *as_const(a.counts);
    if (n_sel <= 0) return;
    const int total = prefix[n_sel];
    const int G = gridDim.x;
    int it = xcd_logical(blockIdx.x, G);
    BpJob job;
    auto next = [&](QtTile& tl) {
        if (it >= total) return false;
        int lo = 0, hi = n_sel - 1;
        while (lo < hi) {
            const int mid = (lo + hi + 1) >> 1;
            if (prefix[mid] <= it) lo = mid; else hi = mid - 1;
        }
        job = load_const(a.jobs + as_const(a.job_index)[lo]);
        const int tt = it - prefix[lo];
        const int ty = tt / job.tiles_x;
        const int tx = tt - ty * job.tiles_x;
        set_job(tl, job);
        tl.q = job.q;
        tl.img = job.img;
        tl.c0 = tx * kTile;
        tl.r0 = ty * kTileH;
        it += G;
        return true;
    };
    qt_run<WP, B, 2, true>(next, smem);
}

}  // namespace

int qt_pitch_for(int WL) {
    if (WL <= 31) return 32;
    if (WL <= 63) return 64;
    return 0;
}

int qt_block_pairs(int WP) { return WP == 32 ? 2 : 1; }

hipError_t launch_bp_qt_grid(const BpJob& job, int n_slices, size_t q_stride, size_t img_stride,
                             int tiles_per_slice, hipStream_t stream) {
    const long long total = (long long)n_slices * tiles_per_slice;
    if (total <= 0) return hipSuccess;
    if (total > 0x7fffffffLL) return hipErrorInvalidValue;
    // one 16-wave workgroup per CU at a time: a workgroup per tile up to one per CU,
    // persistent workgroups (several tiles each) beyond
    const int cus = current_device_cus();
    const int grid = (int)std::min<long long>(total, cus);
    const int tot = (int)total;
    constexpr int B32 = 2, B64 = 1;
    const dim3 g((unsigned)grid), b(kThreads);
    const bool ws = job.wscale != nullptr, persist = grid < tot;
#define FBP_QT_GRID(WP, BB)                                                                                       \
    (persist ? (ws ? launch_kernel(bp_qt_grid_kernel<WP, BB, true, true>, g, b, 0, stream, job, q_stride,           \
                                   img_stride, tiles_per_slice, tot)                                                \
                   : launch_kernel(bp_qt_grid_kernel<WP, BB, false, true>, g, b, 0, stream, job, q_stride,          \
                                   img_stride, tiles_per_slice, tot))                                               \
             : (ws ? launch_kernel(bp_qt_grid_kernel<WP, BB, true, false>, g, b, 0, stream, job, q_stride,          \
                                   img_stride, tiles_per_slice, tot)                                                \
                   : launch_kernel(bp_qt_grid_kernel<WP, BB, false, false>, g, b, 0, stream, job, q_stride,         \
                                   img_stride, tiles_per_slice, tot)))
    if (job.WL == 32) return FBP_QT_GRID(32, B32);
    if (job.WL == 64) return FBP_QT_GRID(64, B64);
#undef FBP_QT_GRID
    return hipErrorInvalidValue;
}

hipError_t launch_bp_qt_list(int WP, const BpListArgs* a, int grid, hipStream_t stream) {
    constexpr int B32 = 2, B64 = 1;
    if (WP == 32) return launch_kernel(bp_qt_list_kernel<32, B32>, dim3(grid), dim3(kThreads), 0, stream, a);
    if (WP == 64) return launch_kernel(bp_qt_list_kernel<64, B64>, dim3(grid), dim3(kThreads), 0, stream, a);
    return hipErrorInvalidValue;
}

}  // namespace fbp
