// Ram-Lak ramp filter as a GEMM on the gfx950 matrix cores.
//
// The filtered projection Q = P * H of arXiv 2109.02174 (section "Computed
// tomography") with the Ram-Lak kernel is, for all rows at once,
//     Q[R][D] = P[R][D] x T,   T[m][n] = tap(n - m) = dt h(n - m),
// a dense contraction over the D input bins (linear convolution: the kernel
// spans every |n - m| <= D-1, so nothing is truncated).
//
// The kernel vanishes at even nonzero offsets, so an even output bin n = 2n'
// only sees odd input bins m = 2m'+1 and an odd output only even inputs:
//     Q[2n'+s] = tap(0) P[2n'+s] + sum_m' to(n' - m' + s) P[2m' + 1 - s],
//     to(j) = tap(2j - 1),
// two half-size Toeplitz GEMMs (half the MACs of the dense product) plus the
// centre tap, which is applied in FP32 in the epilogue.  No T matrix exists in
// memory: each workgroup copies the slice of the 1D odd-tap table its outputs
// need into LDS and feeds the B operand from there.
//
// Workgroup: a group of 256 lanes = 4 waves per tile of 32 rows x kGemmBN output
// bins (FP32 tiles also 32 or 96 bins wide; FP32 grids with no more tiles than
// CUs run two groups per tile, each taking half of every chunk's k-steps).  Wave
// w of a group owns rows 16 (w/2) .. +16 and the output bins of parity w%2 (one
// 16x16 MFMA block per 16 bins of that parity).
// A ring of register buffers keeps several chunks of sinogram rows in flight
// while the current one is multiplied; the LDS panel they are staged into is
// double-buffered, so each barrier step needs one barrier (FP32 two-group tiles
// stage two chunks per step, the others one).
//   FP32:       v_mfma_f32_16x16x4_f32, 32 inputs per parity per chunk.
//   BF16/FP16:  v_mfma_f32_16x16x32_{bf16,f16}, 64 per parity per chunk; the rows
//               are rounded to 16 bits (RNE) as they are staged, and the tap slice
//               is kept in LDS as eight copies shifted by one element so every
//               8-tap fragment is one aligned 16-byte read.
#include "fbp_internal.hpp"

namespace fbp {

namespace {

typedef float v4f __attribute__((ext_vector_type(4)));
typedef __bf16 v8bf __attribute__((ext_vector_type(8)));
typedef _Float16 v8h __attribute__((ext_vector_type(8)));
typedef unsigned short v8u16 __attribute__((ext_vector_type(8)));

constexpr int kTM = kGemmBM;        // rows per tile (32)
constexpr int kTN = kGemmBN;        // output bins per tile (64 = 32 per parity)
constexpr int kHalfN = kTN / 2;
constexpr int kNB = kHalfN / 16;     // 16x16 MFMA blocks per wave

__device__ __forceinline__ unsigned short to_bf16_rne(float x) {
    unsigned int u = __float_as_uint(x);
    u += 0x7FFFu + ((u >> 16) & 1u);
    return (unsigned short)(u >> 16);
}

__device__ __forceinline__ unsigned short to_f16_rne(float x) {
    _Float16 h = (_Float16)x;
    return __builtin_bit_cast(unsigned short, h);
}

template <int PREC>
__device__ __forceinline__ float round_operand(float x) {
    if constexpr (PREC == kBF16) return __uint_as_float((unsigned int)to_bf16_rne(x) << 16);
    else if constexpr (PREC == kFP16) return (float)(_Float16)x;
    else return x;
}

// Buffer resource over rows m0 .. m0 + rows - 1 of P (row length D): loads at byte
// offsets past the end return 0, so the padded rows and columns of a tile read
// as zeros without branches (which would make the compiler wait for every load
// in flight before each chunk instead of only the one it consumes).
constexpr int kBufWord3 = 0x00020000;   // 32-bit data format, raw (stride 0) buffer
constexpr int kOutOfRange = 0x7FFFFFF0;

__device__ __forceinline__ __amdgpu_buffer_rsrc_t tile_rows(const float* P, int m0, int rows, int D) {
    return __builtin_amdgcn_make_buffer_rsrc(const_cast<float*>(P + (size_t)m0 * D), (short)0, rows * D * 4,
                                             kBufWord3);
}

__device__ __forceinline__ float load_elem(__amdgpu_buffer_rsrc_t rows, int row, int col, int D) {
    const int off = (col < D) ? (row * D + col) * 4 : kOutOfRange;
    return __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(rows, off, 0, 0));
}

// Column weights (job.colw: one factor per input column, applied to P before the
// product, e.g. the fan-beam cosine pre-weights); columns past D read 0.
__device__ __forceinline__ __amdgpu_buffer_rsrc_t col_weights(const GemmJob& job) {
    return __builtin_amdgcn_make_buffer_rsrc(const_cast<float*>(job.colw), (short)0, job.colw ? job.D * 4 : 0,
                                             kBufWord3);
}

__device__ __forceinline__ float load_weight(__amdgpu_buffer_rsrc_t wcol, int col) {
    return __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(wcol, col * 4, 0, 0));
}

// Centre-tap inputs of a 16x16 output block, loaded at the start of the tile so
// their latency hides behind the product: lane l gets P[row0 + 4 (l/16) + i][n]
// (times the column weight with CW), n = 2 (nh0 + l % 16) + sg; prow covers rows
// m0 .. (out-of-range rows and columns read 0).
template <bool CW>
__device__ __forceinline__ void load_centre(float (&pre)[4], __amdgpu_buffer_rsrc_t prow,
                                            __amdgpu_buffer_rsrc_t wcol, int D, int row0m, int nh0, int sg) {
    const int l = threadIdx.x & 63;
    const int n = 2 * (nh0 + (l & 15)) + sg;
    const float w = CW ? load_weight(wcol, n) : 1.0f;
#pragma unroll
    for (int i = 0; i < 4; ++i) {
        pre[i] = load_elem(prow, row0m + 4 * (l >> 4) + i, n, D);
        if constexpr (CW) pre[i] *= w;
    }
}

// Epilogue: lane l of a 16x16 block holds rows 4 (l/16) + i, column l % 16; pre:
// its centre-tap inputs (load_centre), used by kernels without even taps.
template <int PREC>
__device__ __forceinline__ void store_block(const v4f& acc, const float (&pre)[4], const GemmJob& job, int row0,
                                            int nh0, int sg) {
    const int l = threadIdx.x & 63;
    const int n = 2 * (nh0 + (l & 15)) + sg;
    if (n >= job.D) return;
#pragma unroll
    for (int i = 0; i < 4; ++i) {
        const int m = row0 + 4 * (l >> 4) + i;
        if (m < job.R) {
            float v = acc[i];
            if (!job.full) v = fmaf(job.diag, round_operand<PREC>(pre[i]), v);
            job.q[(size_t)m * job.D + n] = v * job.out_scale;
        }
    }
}

// ---------------------------------------------------------------- FP32 operands

constexpr int kK32 = 32;                  // inputs per parity per chunk
constexpr int kPD = 4;                    // chunks in flight (register ring)
constexpr int kAS32 = kK32 + 4;           // LDS row stride (floats): 16-byte rows, no bank conflicts
constexpr int kPar32 = kTM * kAS32 + 32;  // parity plane stride (floats; 32 banks apart, so the two
                                          // parities' stores of one column pair never share a bank)
constexpr int kABuf32 = 2 * kPar32;       // floats per panel buffer

// Tap copies of the FP32 path: y runs over [jlo, jhi], jhi = nh0 + HN (HN output
// bins per parity); copy s (s = 0..3) holds to(jhi - (x + s)) at x, so the eight
// taps a lane needs for the eight k-steps of a chunk (descending y) are eight
// consecutive floats of one copy starting at a multiple of four: two aligned
// 16-byte reads.  The copies sit 16 banks apart (stride = 16 mod 64 floats), so the
// 16 lanes of a row, which read four offsets in each of the four copies, cover the
// 64 banks once.
__host__ __device__ constexpr int copy_stride32(int mpad, int hn) {
    const int s = (mpad + hn + 8 + 3) & ~3;
    return s + ((16 - s % 64) + 64) % 64;
}

// FULL: the kernel also has even taps; even outputs then take even inputs through
// te and odd outputs odd inputs (the same-parity half of the panel), doubling the
// MFMAs of the parity-split product.
//
// The inputs of a chunk are assigned to the MFMA k-steps as m' = mh0 + 8 q + kk
// (q = lane / 16, kk = k-step 0..7), so a lane's A values and B values over the
// chunk's eight k-steps are eight consecutive floats in LDS (16-byte reads instead
// of one 4-byte read per k-step).  k-steps 0..3 of every chunk go into accumulator
// set 0 and k-steps 4..7 into set 1; the output is set 0 + set 1.
//
// G: groups of four waves.  G = 1: one group does both sets.  G = 2 (small grids,
// where one group per CU leaves one wave per SIMD): group g does set g of every
// chunk on the shared panel, and group 1 hands its sums to group 0 through LDS.
// Every accumulator sees the same MFMAs in the same order either way, so the two
// forms give the same bits and the host may pick either per launch.
template <bool FULL, bool CW, int NB, int G, int CPB>
__device__ __forceinline__ void gemm_tile_f32(const GemmJob& job, int mt, int nt, char* smem) {
    static_assert(G == 1 || G == 2, "groups");
    static_assert(CPB == 1 || CPB == 2, "chunks per barrier");
    constexpr int HN = 16 * NB;                          // output bins per parity of the tile
    constexpr int NT = 256 * G;                          // threads
    constexpr int KS = kK32 / 4;                         // k-steps per chunk
    constexpr int NS = 2 / G;                            // accumulator sets per group
    constexpr int KG = KS / 2;                           // k-steps per set
    float* As = reinterpret_cast<float*>(smem);          // [2 buffers][CPB chunks][2 parity planes][32 rows][kAS32]
    float* Tc = As + 2 * CPB * kABuf32;                  // 4 copies of the odd taps, then of the even taps
    const int tid = threadIdx.x;
    const int grp = G == 1 ? 0 : __builtin_amdgcn_readfirstlane(tid >> 8);
    const int t = tid & 255;                             // thread within its group
    const int w = t >> 6, l = t & 63;
    const int wm = w >> 1, sg = w & 1;                   // row half, output parity
    const int m0 = mt * kTM, nh0 = nt * HN;
    const int R = job.R, D = job.D, Dh = job.Dh, Dhp = job.Dhp;
    const float* __restrict__ taps = static_cast<const float*>(job.taps);
    const float* __restrict__ P = job.p;
    const int mpad = (Dh + kK32 - 1) / kK32 * kK32;       // inputs per parity, padded
    const int jhi = nh0 + HN;
    const int cstride = copy_stride32(mpad, HN);
    float* Te = Tc + 4 * cstride;                        // even-tap copies (FULL)

    // ring of kPD chunks of 64 input columns in registers: chunk c + kPD - 1 is
    // loaded while chunk c is multiplied, hiding several chunks of load latency
    // ring entry: a thread's EL elements of a chunk (all in column c0 + tid % 64) and,
    // with column weights (CW), that column's weight
    constexpr int EL = 2048 / NT;
    constexpr int RE = CW ? EL + 1 : EL;
    constexpr int RP = CPB == 1 ? kPD : 3 * CPB;         // ring entries (chunks)
    float pf[RP][RE];
    const __amdgpu_buffer_rsrc_t prow = tile_rows(P, m0, min(kTM, R - m0), D);
    const __amdgpu_buffer_rsrc_t wcol = col_weights(job);
    auto load = [&](float (&r)[RE], int c0) {   // columns c0 .. c0+63 of rows m0 .. m0+31
#pragma unroll
        for (int i = 0; i < EL; ++i) {
            const int e = tid + i * NT;
            r[i] = load_elem(prow, e >> 6, c0 + (e & 63), D);
        }
        if constexpr (CW) r[RE - 1] = load_weight(wcol, c0 + (tid & 63));
    };
    auto store = [&](const float (&r)[RE], float* Ab) {
#pragma unroll
        for (int i = 0; i < EL; ++i) {
            const int e = tid + i * NT;
            const int row = e >> 6, col = e & 63;
            Ab[(col & 1) * kPar32 + row * kAS32 + (col >> 1)] = CW ? r[i] * r[RE - 1] : r[i];
        }
    };

    // the first chunks, the centre-tap inputs and the taps are all requested before
    // the first wait, so their memory latencies overlap
#pragma unroll
    for (int c = 0; c < RP - CPB; ++c) load(pf[c], c * 2 * kK32);
    float pre[NB][4];
    if constexpr (!FULL) {
        if (grp == 0) {
#pragma unroll
            for (int j = 0; j < NB; ++j) load_centre<CW>(pre[j], prow, wcol, D, wm * 16, nh0 + 16 * j, sg);
        }
    }
    __syncthreads();   // LDS reuse across tiles of a persistent workgroup
    // one load per tap, stored into the four copies (element x - c of copy c)
#pragma unroll 2
    for (int x = tid; x < cstride + 3; x += NT) {
        const int idx = jhi - x + Dhp;                   // table index of to(jhi - x)
        const bool in = idx >= 0 && idx <= 2 * Dhp;
        const float v = in ? taps[idx] : 0.0f;
        float ve = 0.0f;
        if constexpr (FULL) ve = in ? static_cast<const float*>(job.taps_even)[idx] : 0.0f;
#pragma unroll
        for (int c = 0; c < 4; ++c) {
            const int y = x - c;
            if (y >= 0 && y < cstride) {
                Tc[c * cstride + y] = v;
                if constexpr (FULL) Te[c * cstride + y] = ve;
            }
        }
    }

    v4f acc[NS][NB];
#pragma unroll
    for (int h = 0; h < NS; ++h)
#pragma unroll
        for (int j = 0; j < NB; ++j) acc[h][j] = v4f{0.f, 0.f, 0.f, 0.f};
    const int q = l >> 4;
    const int k0 = G == 1 ? 0 : KG * grp;                // first k-step of this group
    const int arow = (wm * 16 + (l & 15)) * kAS32 + 8 * q + k0;
    const float* __restrict__ Arow = As + (1 - sg) * kPar32 + arow;
    const float* __restrict__ ArowS = As + sg * kPar32 + arow;   // same parity (FULL)
    // B: x0 = jhi - (n' - m' + s) at kk = 0, n' = nh0 + 16 j + l % 16, m' = mh0 + 8 q;
    // its residue mod 4 (the copy) is the same for every chunk and block
    const int xl = jhi - nh0 - (l & 15) - sg + 8 * q;
    const int cs = xl & 3;
    const float* __restrict__ Bl = Tc + cs * cstride + (xl - cs) + k0;
    const int xle = xl + sg;                               // even taps: y = n' - m'
    const int cse = xle & 3;
    const float* __restrict__ Ble = Te + cse * cstride + (xle - cse) + k0;
    const int nch = (D + 2 * kK32 - 1) / (2 * kK32);
    // every chunk load is issued unconditionally (chunks past the end read zeros),
    // so the wait before a chunk's store covers only that chunk.  CPB chunks are
    // stored per barrier; the ring holds RP - CPB chunks ahead of the ones stored.
    for (int cb = 0; cb < nch; cb += RP) {
#pragma unroll
        for (int u = 0; u < RP; u += CPB) {
            const int c = cb + u;
#pragma unroll
            for (int i = 0; i < CPB; ++i) load(pf[(u + RP - CPB + i) % RP], (c + RP - CPB + i) * 2 * kK32);
            // double-buffered panel: every wave finished the chunks of the step before
            // the last (same buffer) before it passed the last step's barrier, so one
            // barrier per step suffices
            const int ab0 = ((c / CPB) & 1) * CPB * kABuf32;
#pragma unroll
            for (int i = 0; i < CPB; ++i) store(pf[u + i], As + ab0 + i * kABuf32);
            __syncthreads();
#pragma unroll
            for (int i = 0; i < CPB; ++i) {
                if (c + i < nch) {
                    const int ab = ab0 + i * kABuf32;
                    const int mh0 = (c + i) * kK32;
                    // this group's k-steps of the chunk: A and B fragments (four floats each
                    // per set), then the MFMAs, the sets interleaved
                    auto product = [&](const float* arow_p, const float* brow_p) {
                        float a[NS][KG], b[NS][NB][KG];
#pragma unroll
                        for (int h = 0; h < NS; ++h) {
                            const float4 av = *reinterpret_cast<const float4*>(arow_p + ab + KG * h);
                            a[h][0] = av.x; a[h][1] = av.y; a[h][2] = av.z; a[h][3] = av.w;
#pragma unroll
                            for (int j = 0; j < NB; ++j) {
                                const float4 bv = *reinterpret_cast<const float4*>(brow_p + mh0 - 16 * j + KG * h);
                                b[h][j][0] = bv.x; b[h][j][1] = bv.y; b[h][j][2] = bv.z; b[h][j][3] = bv.w;
                            }
                        }
                        __builtin_amdgcn_sched_barrier(0);   // keep the reads ahead of the MFMAs
#pragma unroll
                        for (int k = 0; k < KG; ++k)
#pragma unroll
                            for (int h = 0; h < NS; ++h)
#pragma unroll
                                for (int j = 0; j < NB; ++j)
                                    acc[h][j] = __builtin_amdgcn_mfma_f32_16x16x4f32(a[h][k], b[h][j][k], acc[h][j], 0, 0, 0);
                    };
                    static_assert(KG == 4, "four k-steps per set");
                    product(Arow, Bl);
                    if constexpr (FULL) product(ArowS, Ble);
                }
            }
        }
    }
    if constexpr (G == 1) {
#pragma unroll
        for (int j = 0; j < NB; ++j)
            store_block<kFP32>(acc[0][j] + acc[1][j], pre[j], job, m0 + wm * 16, nh0 + 16 * j, sg);
    } else {
        // set 1 (group 1) through LDS to group 0, which adds set 0 + set 1
        __syncthreads();   // every panel read
        v4f* xch = reinterpret_cast<v4f*>(smem);   // [NB][256]
        if (grp == 1) {
#pragma unroll
            for (int j = 0; j < NB; ++j) xch[j * 256 + t] = acc[0][j];
        }
        __syncthreads();
        if (grp == 0) {
#pragma unroll
            for (int j = 0; j < NB; ++j)
                store_block<kFP32>(acc[0][j] + xch[j * 256 + t], pre[j], job, m0 + wm * 16, nh0 + 16 * j, sg);
        }
    }
}

// ---------------------------------------------------------------- 16-bit operands

constexpr int kK16 = 64;                  // inputs per parity per chunk
constexpr int kPD16 = 3;                  // chunks in flight (register ring)
constexpr int kAS16 = kK16 + 8;           // LDS row stride (16-bit), 16-byte aligned rows
constexpr int kABuf16 = 2 * kTM * kAS16;  // 16-bit elements per panel buffer

__device__ __forceinline__ int copy_stride16(int mpad) { return (mpad + kHalfN + 8 + 7 + 7) & ~7; }

template <int PREC, bool FULL, bool CW>
__device__ __forceinline__ void gemm_tile_16(const GemmJob& job, int mt, int nt, char* smem) {
    unsigned short* As = reinterpret_cast<unsigned short*>(smem);   // [2 buffers][2][32][kAS16]
    unsigned short* Tc = As + 2 * kABuf16;                          // 8 shifted tap copies
    const int t = threadIdx.x;
    const int w = t >> 6, l = t & 63;
    const int wm = w >> 1, sg = w & 1;
    const int m0 = mt * kTM, nh0 = nt * kHalfN;
    const int R = job.R, D = job.D, Dh = job.Dh, Dhp = job.Dhp;
    const unsigned short* __restrict__ taps = static_cast<const unsigned short*>(job.taps);
    const float* __restrict__ P = job.p;
    const int mpad = (Dh + kK16 - 1) / kK16 * kK16;
    // B fragment of lane l: to(n' - m' + s) for m' = mb + 8 (l/16) + i, i = 0..7, with
    // n' = nh0 + 16 ntile + l%16.  As y = m' - n' - s rises, tr(y) = to(-y) is read
    // forward; slice index = y - ylo.
    const int ylo = -(nh0 + kHalfN);
    const int cstride = copy_stride16(mpad);

    unsigned short* Te = Tc + 8 * cstride;                          // the same for te (FULL)

    // ring entry: a thread's 16 elements of a chunk (all in column c0 + t % 128) and,
    // with column weights (CW), that column's weight
    constexpr int RE = CW ? 17 : 16;
    float pf[kPD16][RE];
    const __amdgpu_buffer_rsrc_t prow = tile_rows(P, m0, min(kTM, R - m0), D);
    const __amdgpu_buffer_rsrc_t wcol = col_weights(job);
    auto load = [&](float (&r)[RE], int c0) {   // columns c0 .. c0+127 of rows m0 .. m0+31
#pragma unroll
        for (int i = 0; i < 16; ++i) {
            const int e = t + i * kBpThreads;
            r[i] = load_elem(prow, e >> 7, c0 + (e & 127), D);
        }
        if constexpr (CW) r[RE - 1] = load_weight(wcol, c0 + (t & 127));
    };
    auto store = [&](const float (&r)[RE], unsigned short* Ab) {
#pragma unroll
        for (int i = 0; i < 16; ++i) {
            const int e = t + i * kBpThreads;
            const int row = e >> 7, col = e & 127;
            const float x = CW ? r[i] * r[RE - 1] : r[i];
            Ab[((col & 1) * kTM + row) * kAS16 + (col >> 1)] = (PREC == kBF16) ? to_bf16_rne(x) : to_f16_rne(x);
        }
    };

    // the first chunks, the centre-tap inputs and the taps are all requested before
    // the first wait, so their memory latencies overlap
#pragma unroll
    for (int c = 0; c < kPD16 - 1; ++c) load(pf[c], c * 2 * kK16);
    float pre[kNB][4];
    if constexpr (!FULL) {
#pragma unroll
        for (int j = 0; j < kNB; ++j) load_centre<CW>(pre[j], prow, wcol, D, wm * 16, nh0 + 16 * j, sg);
    }
    __syncthreads();
    // copy c element y holds to(-(ylo + y + c)) (and te the same for FULL: te(n' - m')
    // is read at y + s); one load per tap, stored into the eight copies
#pragma unroll 2
    for (int x = t; x < cstride + 7; x += kBpThreads) {
        const int idx = -(ylo + x) + Dhp;                // table index of to(-(ylo + x))
        const bool in = idx >= 0 && idx <= 2 * Dhp;
        const unsigned short v = in ? taps[idx] : (unsigned short)0;
        unsigned short ve = 0;
        if constexpr (FULL) ve = in ? static_cast<const unsigned short*>(job.taps_even)[idx] : (unsigned short)0;
#pragma unroll
        for (int c = 0; c < 8; ++c) {
            const int y = x - c;
            if (y >= 0 && y < cstride) {
                Tc[c * cstride + y] = v;
                if constexpr (FULL) Te[c * cstride + y] = ve;
            }
        }
    }

    v4f acc[2][kNB];
#pragma unroll
    for (int j = 0; j < kNB; ++j) acc[0][j] = acc[1][j] = v4f{0.f, 0.f, 0.f, 0.f};
    const unsigned short* Arow = As + ((1 - sg) * kTM + wm * 16 + (l & 15)) * kAS16 + 8 * (l >> 4);
    const unsigned short* ArowS = As + (sg * kTM + wm * 16 + (l & 15)) * kAS16 + 8 * (l >> 4);   // same parity
    const int kq = 8 * (l >> 4);
    const int nch = (D + 2 * kK16 - 1) / (2 * kK16);
    for (int cb = 0; cb < nch; cb += kPD16) {
#pragma unroll
        for (int u = 0; u < kPD16; ++u) {
            const int c = cb + u;
            load(pf[(u + kPD16 - 1) % kPD16], (c + kPD16 - 1) * 2 * kK16);
            const int ab = (c & 1) * kABuf16;   // double-buffered panel, one barrier
            store(pf[u], As + ab);
            __syncthreads();
            if (c < nch) {
                const int mh0 = c * kK16;
                // all fragments of the chunk first, then the MFMAs (two accumulator sets)
                constexpr int KS = kK16 / 32;
                v8u16 av[KS], bv[KS][kNB];
#pragma unroll
                for (int k = 0; k < KS; ++k) {
                    av[k] = *reinterpret_cast<const v8u16*>(Arow + ab + 32 * k);
                    const int ya = (mh0 + 32 * k + kq) - (nh0 + (l & 15)) - sg - ylo;
#pragma unroll
                    for (int j = 0; j < kNB; ++j) {
                        const int y = ya - 16 * j;
                        const int cy = y & 7;
                        bv[k][j] = *reinterpret_cast<const v8u16*>(Tc + cy * cstride + (y - cy));
                    }
                }
                __builtin_amdgcn_sched_barrier(0);
                auto mfma = [&](const v8u16& x, const v8u16& y, v4f& c) {
                    if constexpr (PREC == kBF16)
                        c = __builtin_amdgcn_mfma_f32_16x16x32_bf16(__builtin_bit_cast(v8bf, x),
                                                                    __builtin_bit_cast(v8bf, y), c, 0, 0, 0);
                    else
                        c = __builtin_amdgcn_mfma_f32_16x16x32_f16(__builtin_bit_cast(v8h, x),
                                                                   __builtin_bit_cast(v8h, y), c, 0, 0, 0);
                };
#pragma unroll
                for (int k = 0; k < KS; ++k)
#pragma unroll
                    for (int j = 0; j < kNB; ++j) mfma(av[k], bv[k][j], acc[k & 1][j]);
                if constexpr (FULL) {
#pragma unroll
                    for (int k = 0; k < KS; ++k) {
                        av[k] = *reinterpret_cast<const v8u16*>(ArowS + ab + 32 * k);
                        const int ya = (mh0 + 32 * k + kq) - (nh0 + (l & 15)) - ylo;   // + s - s
#pragma unroll
                        for (int j = 0; j < kNB; ++j) {
                            const int y = ya - 16 * j;
                            const int cy = y & 7;
                            bv[k][j] = *reinterpret_cast<const v8u16*>(Te + cy * cstride + (y - cy));
                        }
                    }
                    __builtin_amdgcn_sched_barrier(0);
#pragma unroll
                    for (int k = 0; k < KS; ++k)
#pragma unroll
                        for (int j = 0; j < kNB; ++j) mfma(av[k], bv[k][j], acc[k & 1][j]);
                }
            }
        }
    }
#pragma unroll
    for (int j = 0; j < kNB; ++j) store_block<PREC>(acc[0][j] + acc[1][j], pre[j], job, m0 + wm * 16, nh0 + 16 * j, sg);
}

// One instantiation per (operand precision, kernel with or without even taps), so
// the Ram-Lak path keeps its register budget.
template <int PREC, bool FULL, bool CW = false, int NB = kNB, int G = 1, int CPB = 1>
__device__ __forceinline__ void gemm_tile(const GemmJob& job, int mt, int nt, char* smem) {
    if constexpr (PREC == kFP32)
        gemm_tile_f32<FULL, CW, NB, G, CPB>(job, mt, nt, smem);
    else
        gemm_tile_16<PREC, FULL, CW>(job, mt, nt, smem);
}

// CW: the job has column weights (job.colw); a separate instantiation keeps the
// unweighted filter's ring and stores as they were
// NB: 16-wide MFMA blocks per wave and parity (2: 64-bin tiles; FP32 also 1: 32-bin, 3: 96-bin)
// G: groups of four waves (FP32: 1 or 2)
// CPB: chunks staged per panel barrier (FP32: 1 or 2; the same bits)
template <int PREC, bool FULL, bool CW, int NB, int G, int CPB>
__global__ __launch_bounds__(kBpThreads * G) void gemm_grid_kernel(GemmJob job) {
    extern __shared__ float4 smem4[];
    // logical tile: column tiles fastest, so the tiles of one row block (which all read
    // that block's rows) run on one XCD and share its L2
    const int b = xcd_logical(blockIdx.x, gridDim.x);
    const int mt = b / job.tiles_n, nt = b - mt * job.tiles_n;
    gemm_tile<PREC, FULL, CW, NB, G, CPB>(job, mt, nt, reinterpret_cast<char*>(smem4));
}

template <int PREC, bool FULL>
__global__ __launch_bounds__(kBpThreads) void gemm_list_kernel(const GemmListArgs* __restrict__ args) {
    extern __shared__ float4 smem4[];
    const GemmListArgs a = load_const(args);
    const auto* __restrict__ prefix = as_const(a.tile_prefix);
    const int n_jobs = *as_const(a.counts);
    if (n_jobs <= 0) return;
    const int total = prefix[n_jobs];
    for (int it = xcd_logical(blockIdx.x, gridDim.x); it < total; it += gridDim.x) {
        int lo = 0, hi = n_jobs - 1;
        while (lo < hi) {
            const int mid = (lo + hi + 1) >> 1;
            if (prefix[mid] <= it) lo = mid; else hi = mid - 1;
        }
        const GemmJob job = load_const(a.jobs + lo);
        const int tt = it - prefix[lo];
        const int mt = tt / job.tiles_n, nt = tt - mt * job.tiles_n;
        gemm_tile<PREC, FULL>(job, mt, nt, reinterpret_cast<char*>(smem4));
    }
}

template <int PREC, bool FULL>
int occ(int lds) {
    int n = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, gemm_list_kernel<PREC, FULL>, kBpThreads, lds) !=
        hipSuccess)
        return 1;
    return n > 0 ? n : 1;
}

// Every compiled filter kernel: (precision, kernel with even taps).
#define FBP_FOR_EACH_GEMM16(X) \
    X(kBF16, false)            \
    X(kBF16, true)             \
    X(kFP16, false)            \
    X(kFP16, true)
#define FBP_FOR_EACH_GEMM(X) \
    X(kFP32, false)          \
    X(kFP32, true)           \
    FBP_FOR_EACH_GEMM16(X)

constexpr int gemm_key(int prec, bool full) { return prec * 2 + (full ? 1 : 0); }

}  // namespace

int gemm_lds_bytes(int prec, int Dh, bool full, int nb, int cpb) {
    const int tables = full ? 2 : 1;   // odd taps, and even taps for kernels that have them
    if (prec == kFP32) {
        const int mpad = (Dh + kK32 - 1) / kK32 * kK32;
        // panel (two buffers of the cpb chunks of one barrier step), four copies of each tap table
        return (2 * cpb * kABuf32 + tables * 4 * copy_stride32(mpad, nb > 0 ? 16 * nb : kHalfN)) * 4;
    }
    const int mpad = (Dh + kK16 - 1) / kK16 * kK16;
    return (2 * kABuf16 + tables * 8 * ((mpad + kHalfN + 8 + 7 + 7) & ~7)) * 2;
}

constexpr size_t kMaxLdsBytes = 160 * 1024;   // LDS of one gfx950 CU

// FP32 grid launch with the tile width (NB), group count (G) and chunks per barrier
// (CPB) as template arguments.
template <int NB, int G, int CPB>
hipError_t launch_f32(const GemmJob& job, dim3 g, size_t lds, hipStream_t stream) {
    const dim3 b(kBpThreads * G);
    if (job.full)
        return job.colw ? launch_kernel(gemm_grid_kernel<kFP32, true, true, NB, G, CPB>, g, b, lds, stream, job)
                        : launch_kernel(gemm_grid_kernel<kFP32, true, false, NB, G, CPB>, g, b, lds, stream, job);
    return job.colw ? launch_kernel(gemm_grid_kernel<kFP32, false, true, NB, G, CPB>, g, b, lds, stream, job)
                    : launch_kernel(gemm_grid_kernel<kFP32, false, false, NB, G, CPB>, g, b, lds, stream, job);
}

// Two-group tiles (small grids) stage two chunks per barrier where that panel still
// fits the CU's LDS with the tap copies (long detectors with even taps do not).
template <int NB>
hipError_t launch_f32_groups(const GemmJob& job, dim3 g, hipStream_t stream) {
    const bool full = job.full != 0;
    if (job.groups == 2) {
        const size_t lds2 = (size_t)gemm_lds_bytes(kFP32, job.Dh, full, job.nb, 2);
        if (lds2 <= kMaxLdsBytes) return launch_f32<NB, 2, 2>(job, g, lds2, stream);
        return launch_f32<NB, 2, 1>(job, g, (size_t)gemm_lds_bytes(kFP32, job.Dh, full, job.nb, 1), stream);
    }
    return launch_f32<NB, 1, 1>(job, g, (size_t)gemm_lds_bytes(kFP32, job.Dh, full, job.nb, 1), stream);
}

hipError_t launch_gemm_grid(int prec, const GemmJob& job, hipStream_t stream) {
    const int tiles_m = (job.R + kTM - 1) / kTM;
    const unsigned grid = (unsigned)(tiles_m * job.tiles_n);
    const int nb = job.nb > 0 ? job.nb : kNB;
    if (nb != kNB && (prec != kFP32 || nb > 3 || job.tiles_n != (job.D + 32 * nb - 1) / (32 * nb)))
        return hipErrorInvalidValue;
    if (job.groups != 1 && (prec != kFP32 || job.groups != 2)) return hipErrorInvalidValue;
    const dim3 g(grid);
    if (prec == kFP32) {
        if (nb == 1) return launch_f32_groups<1>(job, g, stream);
        if (nb == 3) return launch_f32_groups<3>(job, g, stream);
        return launch_f32_groups<kNB>(job, g, stream);
    }
    const size_t lds = (size_t)gemm_lds_bytes(prec, job.Dh, job.full != 0, job.nb);
    const dim3 b(kBpThreads);
    switch (gemm_key(prec, job.full != 0)) {
#define X(p, f)                                                                                              \
        case gemm_key(p, f):                                                                                     \
            return job.colw ? launch_kernel(gemm_grid_kernel<p, f, true, kNB, 1, 1>, g, b, lds, stream, job) \
                            : launch_kernel(gemm_grid_kernel<p, f, false, kNB, 1, 1>, g, b, lds, stream, job);
        FBP_FOR_EACH_GEMM16(X)
#undef X
        default: return hipErrorInvalidValue;
    }
}

hipError_t launch_gemm_list(int prec, bool full, const GemmListArgs* a, int grid, size_t lds, hipStream_t stream) {
    switch (gemm_key(prec, full)) {
#define X(p, f) \
        case gemm_key(p, f): return launch_kernel(gemm_list_kernel<p, f>, dim3(grid), dim3(kBpThreads), lds, stream, a);
        FBP_FOR_EACH_GEMM(X)
#undef X
        default: return hipErrorInvalidValue;
    }
}

int gemm_occupancy(int prec, bool full, size_t lds_bytes) {
    const int lds = (int)lds_bytes;
    switch (gemm_key(prec, full)) {
#define X(p, f) case gemm_key(p, f): return occ<p, f>(lds);
        FBP_FOR_EACH_GEMM(X)
#undef X
        default: return 1;
    }
}

}  // namespace fbp
