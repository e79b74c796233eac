// Internal types shared by the HIP kernels and the host runtime of libfbp.
#pragma once

#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

namespace fbp {

// Read-only view of device data in the constant address space: uniform loads
// through it compile to scalar loads (descriptor tables read by whole waves).
template <typename T>
__device__ __forceinline__ const __attribute__((address_space(4))) T* as_const(const T* p) {
    return (const __attribute__((address_space(4))) T*)p;
}

// Copy of a descriptor struct read through the constant address space.
template <typename T>
__device__ __forceinline__ T load_const(const T* p) {
    static_assert(sizeof(T) % 4 == 0, "descriptor size");
    T v;
    const __attribute__((address_space(4))) unsigned int* src =
        (const __attribute__((address_space(4))) unsigned int*)p;
    unsigned int* dst = reinterpret_cast<unsigned int*>(&v);
#pragma unroll
    for (unsigned i = 0; i < sizeof(T) / 4; ++i) dst[i] = src[i];
    return v;
}

// XCD-aware block order: the hardware places block b on XCD b % 8, and each XCD has
// its own L2.  xcd_logical gives each XCD a contiguous range of logical work items
// (a bijection of [0, G)), so items that read the same rows share an L2.
__device__ __forceinline__ int xcd_logical(int b, int G) {
    const int x = b & 7;
    const int slot = b >> 3;
    const int per = G >> 3;
    const int extra = G & 7;
    return x * per + min(x, extra) + slot;
}

// Launch with the error returned by the launch itself (not a thread's sticky
// last-error state, which an unrelated earlier call may have set).
template <typename T>
struct nondeduced {
    using type = T;
};
template <typename... A>
inline hipError_t launch_kernel(void (*kernel)(A...), dim3 grid, dim3 block, size_t lds, hipStream_t stream,
                                typename nondeduced<A>::type... args) {
    void* argv[] = {static_cast<void*>(&args)..., nullptr};
    return hipLaunchKernel(reinterpret_cast<const void*>(kernel), grid, block, argv, lds, stream);
}

// ------------------------------------------------------------------ backprojection

// Everything one slice's backprojection needs, as the kernels see it.
struct BpJob {
    const float* q;       // filtered rows [K][D]
    float* img;           // image [N][N]
    const double* cs;     // [K][2]: cos(theta_k)/dt, sin(theta_k)/dt in FP64 (window origins)
    const float* cs32;    // [K][2]: the same rounded to FP32 (pixel steps)
    double half_pix;      // (N-1)/2
    double centre_det;    // (D-1)/2
    int32_t N, K, D;
    int32_t WL;           // window length (bins) staged per angle for this job's tile shape
    int32_t KB;           // angles staged per LDS block
    int32_t seg_shift;    // log2 of the 63-bin staging segments per angle (>= WL / 63)
    int32_t tiles_x;      // tile columns of the half image
    float scale;          // pi/K
    float* part;          // angle-split partial sums [n][split][N][N] (split > 1 only)
    const float* wscale;  // [K] angle weight / (pi/K), or null for pi/K throughout
    int32_t split;        // angle parts: workgroup part r takes the angles r, r + split, ...
    int32_t pad_;
};
static_assert(sizeof(BpJob) % 8 == 0, "BpJob layout");

// Compile-time tile shapes of the backprojector.  A workgroup has s groups of
// 256 lanes; lane t of a group owns column t % tw and p consecutive rows starting
// at (t / tw) * p, for its pixel and the pixel's point reflection through the
// image centre.  Group g takes the angles g, g+s, g+2s, ... of every staged block;
// the groups' partial sums are added in fixed order at the end.
struct TileShape {
    int32_t tw, p, th, s;
    const char* name;
    int32_t rot = 0;      // 1: quadrant tile and its three 90-degree rotations (angle pairs);
                          // 2: the same with one contiguous angle chunk per wave (bp_qt_kernels)
    int32_t multi = 1;    // slices per workgroup of the stack variant (1: none)
};

constexpr int kGroupThreads = 256;
constexpr int kBpThreads = 256;   // threads of the GEMM workgroups
constexpr int kNumTileConfigs = 15;
// Chunked quarter-turn shapes (rot == 2): tile ids, angle chunks (= waves per
// workgroup) and quadrant tile side.  The two ids differ only in the LDS pitch of
// the staged windows (32 or 64 bins), not in their arithmetic.
constexpr int kQtCfg32 = 13;
constexpr int kQtCfg64 = 14;
constexpr int kQtChunks = 16;
constexpr int kQtTile = 16;                 // tile width (columns); one column per lane of a 16-lane row
constexpr int kQtRows = 4;                  // rows per lane
constexpr int kQtTileH = 4 * kQtRows;       // tile height: four 16-lane rows of a wave
constexpr int kMaxKB = 64;
// Most angle parts a single slice's backprojection is split into (one-group shapes).
constexpr int kMaxSplit = 16;
constexpr int kStageE = 4;        // staged (angle, bin) elements per thread per block
// Staged elements per thread per block for a shape with s angle groups: the
// one-group shapes have a quarter of the waves, so each stages more.
constexpr int stage_elems(int s) { return s == 1 ? 8 : kStageE; }
// Dynamic LDS budget of one backprojection workgroup (bytes).
constexpr int kBpLdsBudget = 48 * 1024;
// Budget of a workgroup that backprojects several slices of one geometry.
constexpr int kBpMultiLdsBudget = 64 * 1024;
// LDS bytes of the per-angle constants of the current and next block (float4 each).
constexpr int kBpPrmBytes = 2 * kMaxKB * 16;
// Rotation-symmetric shapes: float4 + int2 per angle pair, two blocks.
constexpr int kBpRotPrmBytes = 2 * kMaxKB * 24;
// LDS budget of the rotation-symmetric shapes (two windows of 32-byte bins per pair).
constexpr int kBpRotLdsBudget = 64 * 1024;

const TileShape& tile_shape(int cfg);

// Window length for a tile shape: bins covering every pixel centre of a TW x TH
// tile at any angle, plus interpolation and rounding margin.  span_max is the
// largest (TW-1)|cos|/dt + (TH-1)|sin|/dt over the angles.
inline int window_length(double span_max) { return (int)span_max + 5; }

// LDS bytes of a backprojection workgroup of tile shape cfg that backprojects m
// slices at once, with window WL and block KB; -1 if no such kernel is compiled.
int bp_lds_bytes(int cfg, int m, int WL, int KB);

// Backprojection of n_slices slices of one geometry (tile grid from blockIdx), m
// slices per workgroup (m = 1, or tile_shape(cfg).multi).
hipError_t launch_bp_grid(int cfg, int m, const BpJob& job, int n_slices, size_t q_stride,
                          size_t img_stride, int tiles_per_slice, hipStream_t stream);

// img[s][i] = scale * (part[s][0][i] + part[s][1][i] + ... + part[s][R-1][i]), summed
// in that order, for the angle-split partial sums of n_slices slices of N*N pixels.
hipError_t launch_combine_parts(const float* part, float* img, int n_slices, int R, size_t plane,
                                float scale, hipStream_t stream);

// Persistent backprojection over a mixed list: tile index -> job by binary search in
// tile_prefix (n_jobs + 1 entries, device); jobs and prefix live in device memory,
// counts are read on the device (so a captured graph serves any batch).
struct BpListArgs {
    const BpJob* jobs;          // device [n_jobs]
    const int32_t* job_index;   // device [n_sel]: jobs of this tile shape, cost-ordered
    const int32_t* tile_prefix; // device [n_sel + 1]: exclusive prefix of tile counts
    const int32_t* counts;      // device: counts[0] = n_sel
    // Lists of the multi-slice kernels: entry s is the group of group_size[s] jobs
    // job_index[s] .. job_index[s] + group_size[s] - 1 (one geometry).  Unused (null)
    // by the one-slice kernels.
    const int32_t* group_size;
};
// `args` is a DEVICE pointer (the batch header in the workspace).
hipError_t launch_bp_list(int cfg, int m, const BpListArgs* args, int grid, size_t lds_bytes,
                          hipStream_t stream);
int bp_occupancy(int cfg, int m, size_t lds_bytes);   // resident workgroups per CU

// Chunked quarter-turn backprojector (bp_qt_kernels.hip): job.WL is the window
// pitch (32 or 64 bins); its LDS is static, one 1024-thread workgroup per tile.
int qt_pitch_for(int WL);          // pitch that holds a window of WL bins, 0 if none
int qt_block_pairs(int WP);        // angle pairs staged per block
hipError_t launch_bp_qt_grid(const BpJob& job, int n_slices, size_t q_stride, size_t img_stride,
                             int tiles_per_slice, hipStream_t stream);
hipError_t launch_bp_qt_list(int WP, const BpListArgs* args, int grid, hipStream_t stream);

// Compute units of the current device (cached; runtime.cpp).
int current_device_cus();

// ------------------------------------------------------------------ forward projector

// Everything the projector (adjoint of the backprojector) needs for one geometry.
struct ProjJob {
    const float* pimg;    // padded copies, [n][2][N+1][pitch]: rows, then columns (see launch_pad)
    float* sino;          // [n][K][D]
    const double* cs;     // [K][2]: cos/dt, sin/dt (FP64)
    const float* wscale;  // [K] angle weight / (pi/K), or null
    double half_pix;      // (N-1)/2
    double centre_det;    // (D-1)/2
    int32_t N, K, D;
    float scale;          // pi/K
    int32_t T;            // pixels read per line
    int32_t fast3;        // 1: three taps, 1 <= r <= 1.5 on every angle
    int32_t pad, pitch;   // zeros before each line; floats per padded line
};
// Tap count, kernel choice and padded-copy layout of a geometry's projector (cs as
// in ProjJob); T == 0 when unsupported.
struct ProjLayout {
    int T = 0;
    bool fast3 = false;
    int pad = 0, pitch = 0;
    size_t slice_floats = 0;   // floats of the two padded planes of one slice
    double margin = 0.0;       // fan beam: the margin its window bound holds on
};
ProjLayout project_layout(const double* cs, int K, int N);
hipError_t launch_project(const ProjJob& job, int n_slices, hipStream_t stream);
// Padded row and column copies of n N x N slices into out (n * slice_floats floats).
hipError_t launch_pad(const float* img, float* out, int N, int pad, int pitch, int n_slices, hipStream_t stream);

// Fan-beam forward projector (the adjoint of the fan-beam backprojector), reading
// the same padded copies.
struct FanProjJob {
    const float* pimg;    // padded copies, [n][2][N+1][pitch] (launch_pad)
    float* sino;          // [n][K][D]
    const double* cs;     // [K][2]: cos b, sin b (FP64)
    double R, ds;         // source distance, bin width
    double half_pix;      // (N-1)/2
    double centre_det;    // (D-1)/2
    double margin;        // m: window half-widths are bounded over each line grown by m pixels
    int32_t N, K, D;
    int32_t pad, pitch;
    float scale;          // 2 pi / K
};
// Half-width (pixels along image line lc, a row when `rows`, else a column)
// bounding 1 / |du/dq|, the spacing of neighbouring rays of view (cb, sb) along
// the line, over the line's pixels and `margin` pixels beyond both ends:
//     rows:    1/|du/dx| = ds L^2 / (R |y - R sb|),  columns: ds L^2 / (R |R cb - x|),
// L = R - x cb - y sb largest at the far end of the grown line.  Inflated by
// 2^-12 (relative and absolute) so that FP32 evaluation still bounds it; the same
// function sizes the layout on the host and the windows in the kernel.
template <typename F>
__host__ __device__ inline F fan_line_half_width(F cb, F sb, F R, F ds, F half_pix, F margin, F lc, bool rows) {
    const F ext = half_pix + F(0.5) + margin;
    const F across = rows ? fabs(lc - R * sb) : fabs(R * cb - lc);
    const F Lmax = rows ? R + ext * fabs(cb) - lc * sb : R + ext * fabs(sb) - lc * cb;
    return ds * Lmax * Lmax / (R * across) * F(1.000244140625) + F(0.000244140625);
}
hipError_t launch_fan_project(const FanProjJob& job, int n_slices, hipStream_t stream);

// ------------------------------------------------------------------ fan beam

// Distance-weighted fan-beam backprojection of one geometry (flat detector
// through the rotation centre, source at distance R).
struct FanJob {
    const float* q;       // [n][K][D] filtered views
    float* img;           // [n][N][N]
    const double* cs;     // [K][2]: cos b, sin b (FP64)
    double R, ds;         // source distance, bin width
    double inv_R, inv_dsR;   // 1/R, 1/(ds R)
    double half_span;     // bound on |u - u(tile centre)| over a tile's pixels, in bins
    double half_pix;      // (N-1)/2
    double centre_det;    // (D-1)/2
    int32_t N, K, D;
    int32_t WL;           // window pairs staged per view (bound over tiles and views)
    int32_t KB;           // views per staged block
    int32_t tiles_x;      // ceil(N / kFanTile); quarter-turn form: ceil(((N+1)/2) / kFanTile)
    float scale;          // 2 pi / K
    float* part;          // split > 1: [split][N][N] partial sums (one slice, M = 1)
    int32_t split;        // view parts of a single slice (1: none)
};
constexpr int kFanTile = 16;
constexpr size_t kFanLdsBudget = 48 * 1024;
size_t fan_lds_bytes(int KB, int WL, int M);
// n_slices through the M-slice kernel (M = 2 or 4, KBm views per block) in groups,
// the remainder (and everything when M = 1) one slice per workgroup.
hipError_t launch_fan_bp(const FanJob& job, int n_slices, int M, int KBm, hipStream_t stream);
// Quarter-turn form (N >= 2; K = 4 K4 with view k + i K4 at angle b_k + i pi/2):
// a workgroup owns a tile of the base region, rows [0, N/2) by columns [0, (N+1)/2)
// (tiles_x = ceil(((N+1)/2) / kFanTile), ceil((N/2) / kFanTile) tiles down), and its
// three turned copies, plus, for odd N, the first tile the centre pixel; KB (KBm for
// the M-slice groups) base views per block.
bool fan_rot_addressable(int K, int D, int WL);
size_t fan_rot_lds_bytes(int KB, int WL, int M);
hipError_t launch_fan_rot(const FanJob& job, int n_slices, int M, int KBm, hipStream_t stream);
// out[r][m] = in[r][m] * w[m] over rows x D floats.
hipError_t launch_preweight(const float* in, float* out, const float* w, int64_t rows, int D, hipStream_t stream);

// ------------------------------------------------------------------ cone beam (FDK)

// Cone-beam backprojection of one geometry: projections [K][Dv][Du], volume
// [Nz][N][N], source orbit of radius R, flat detector through the axis.
struct ConeJob {
    const float* q;        // [K][Dv][Du] filtered views
    float* vol;            // [Nz][N][N]
    const double* cs;      // [K][2]: cos b, sin b (FP64)
    double R, du, dv;
    double inv_R, inv_duR; // 1/R, 1/(du R)
    double half_span;      // bound on |u - u(tile centre)| over a tile's columns, in detector columns
    double cu, cv;         // (Du-1)/2, (Dv-1)/2
    double half_pix;       // (N-1)/2
    double half_z;         // (Nz-1)/2
    int32_t N, Nz, K, Du, Dv;
    int32_t WL, WV;        // window bounds over tiles, z blocks and views: columns, rows
    int32_t pitch;         // row pitch of a staged window in floats (>= WL + 1)
    int32_t KB;            // views whose windows a block computes (it stages those that fit)
    int32_t cap;           // LDS floats for the staged windows of a block (>= (WV + 1) pitch)
    int32_t vec4;          // stage groups of four columns (Du, pitch multiples of 4, q 16-byte aligned,
                           // pitch >= WL + 7 for the wider aligned windows)
    int32_t tiles_x;       // ceil(N / kConeTile)
    float scale;           // 2 pi / K
};
constexpr int kConeTile = 16;
constexpr int kConeZB = 32;          // voxels in z per lane
constexpr size_t kConeLdsBudget = 40 * 1024;   // four workgroups per CU
// row pitch of the staged windows for a column bound WL (one of a fixed set, else
// WL + 1 rounded up to a multiple of four)
int cone_pitch(int WL);
size_t cone_lds_bytes(int KB, int cap, bool staged);
// staged: detector windows through LDS (cap floats, which must hold the largest
// window of WV + 1 rows of pitch floats); otherwise values are read from global memory.
hipError_t launch_cone_bp(const ConeJob& job, bool staged, hipStream_t stream);

// ------------------------------------------------------------------ ramp filter GEMM

enum Prec : int32_t { kFP32 = 0, kBF16 = 1, kFP16 = 2 };
constexpr int32_t kFFT32 = 3;     // FP32 through the FFT path (no GEMM)

// ------------------------------------------------------------------ FFT filter path

// Ramp filter of R rows by FFT: pairs of rows packed as one complex row, zero
// padded to L = 2^log2L >= 2D - 1, multiplied by the real DFT of the taps.
struct FftJob {
    const float* p;       // [R][D]
    float* q;             // [R][D]
    const float2* tw;     // [L]: e^{-2 pi i m / L}
    const float* H;       // [L]: DFT of the taps t(d), |d| <= D-1, times (output scale) / L
    int32_t R, D;
    int32_t log2L;
    const float* colw;    // [D] factor per column applied on load, or null
};
constexpr int kFftMaxLog2 = 13;   // L <= 8192 (LDS of 64 KiB): D <= 4096
int fft_length_log2(int D);
hipError_t launch_fft_filter(const FftJob& job, hipStream_t stream);

// One ramp-filter GEMM problem: Q[R][D] = P[R][D] x T, T[m][n] = tap(n - m), computed
// as two parity-split half GEMMs over the odd taps to(j) = tap(2j - 1) plus the
// centre tap.
struct GemmJob {
    const float* p;       // [R][D]
    float* q;             // [R][D]
    const void* taps;     // to(j) at index j + Dhp, j in [-Dhp, Dhp]; element type by precision
    int32_t R, D;
    int32_t Dh;           // ceil(D / 2): inputs per parity
    int32_t Dhp;          // Dh rounded up to 64
    float diag;           // tap(0), rounded like the taps (and pre-scaled for FP16)
    float out_scale;      // undoes the FP16 tap pre-scale (1 otherwise)
    int32_t tiles_n;      // ceil(D / 64)
    int32_t full;         // 1: the kernel has even taps too (te(j) = tap(2j) in taps_even,
                          //    same indexing); diag is then 0 and the centre tap is te(0)
    const void* taps_even;
    const float* colw;    // [D] factor per input column applied to P before the product
                          // (fan-beam pre-weights), or null
    int32_t nb;           // FP32 grid launches: tiles of 32 nb output bins (nb = 1, 2, 3; tiles_n =
                          // ceil(D / (32 nb))); 0 = the default 64-bin tiles
    int32_t groups;       // FP32 grid launches: 1 or 2 groups of four waves per tile (same bits)
};
static_assert(sizeof(GemmJob) % 8 == 0, "GemmJob layout");

constexpr int kGemmBM = 32;   // rows per GEMM tile
constexpr int kGemmBN = 64;   // output bins per GEMM tile

hipError_t launch_gemm_grid(int prec, const GemmJob& job, hipStream_t stream);

struct GemmListArgs {
    const GemmJob* jobs;        // device [n_jobs]
    const int32_t* tile_prefix; // device [n_jobs + 1]
    const int32_t* counts;      // device: counts[0] = n_jobs
};
// `args` is a DEVICE pointer (the batch header in the workspace).
hipError_t launch_gemm_list(int prec, bool full, const GemmListArgs* args, int grid, size_t lds_bytes,
                            hipStream_t stream);
// LDS of a filter workgroup; full: the kernel has even taps too (their copies
// double the tap area); nb: FP32 tiles of 32 nb output bins (0: the default 64);
// cpb: FP32 chunks staged per panel barrier (1 or 2).
int gemm_lds_bytes(int prec, int Dh, bool full, int nb = 0, int cpb = 1);
int gemm_occupancy(int prec, bool full, size_t lds_bytes);

// Device address and size of fbp_reconstruct_noalloc's static workspace on the
// current device (looked up once per device).
hipError_t noalloc_workspace(void** ptr, size_t* bytes);

}  // namespace fbp
