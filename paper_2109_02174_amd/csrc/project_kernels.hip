// Forward projector for gfx950: the exact adjoint of the backprojector.
//
// The backprojection of Eq. 2 (arXiv 2109.02174, section "Computed tomography")
// with linear interpolation is a linear map from filtered rows to pixels; its
// adjoint maps an image to projection rows:
//     sino[k][j] = w_k sum_{r,c} img[r][c] max(0, 1 - |u_k(x_c, y_r) - j|),
//     u_k(x, y) = (x cos(theta_k) + y sin(theta_k)) / dt + (D-1)/2,
// with w_k = pi/K (or the angle-gap weights).
//
// It is computed gather-only, one lane per detector bin, walking image lines
// across the ray: rows when |cos| >= |sin|, else columns.  The slice is first
// copied twice, rows and transposed, each line padded with zeros on both sides
// (pad P) and followed by one zero line, so that both walks read along memory and
// a lane's window never needs a bounds test.  On a line the bin's ray crosses at
// p* (pixel units along the line); the pixels with a nonzero weight are the
// integers in (p* - r, p* + r), r = 1/|a| with a the slope of u along the line:
// at most T = ceil(2r), read as T consecutive floats from floor(p* - r) + 1.
// p* advances by the same step on every line, so it is carried in 32.32 fixed
// point (integer part = window start, fraction = phase of the window), stepped
// with a 64-bit integer add and re-anchored from FP64 every 256 lines; the hat
// weights are FP32 functions of the phase.  A wave walks only the lines its 64
// bins can reach; on those lines every bin of the wave lies within 65 r + 3
// pixels of the image (it is within 63 bins of one that reaches it), which
// bounds the pad.  Each bin is written once by its lane; no atomics; fixed
// summation order (line by line).
#include "fbp_internal.hpp"

namespace fbp {

namespace {

constexpr int kProjThreads = 256;
constexpr int kTrTile = 64;
constexpr int kAnchorLines = 256;                   // FP64 re-anchoring period (power of 2)
constexpr double kTwo32 = 4294967296.0;

// Taps of one line: T > 0 fixed, T == 0 job.T at run time.  FAST3: three taps
// with 1 <= r <= 1.5 on every angle (unit detector spacing), where the first tap
// lies left of p* and the third right of it, so only the middle one needs |.|.
template <int T, bool FAST3>
__global__ __launch_bounds__(kProjThreads) void project_kernel(ProjJob job) {
    // block b: (slice, angle, block of 256 bins), bins fastest
    const int nbj = (job.D + kProjThreads - 1) / kProjThreads;
    const int rest = blockIdx.x / nbj;
    const int k = rest % job.K;                     // angle
    const int s = rest / job.K;                     // slice
    const int jw = (blockIdx.x - rest * nbj) * kProjThreads + (threadIdx.x & ~63);   // first bin of the wave
    if (jw >= job.D) return;                        // whole wave past the last bin
    const int j = jw + (threadIdx.x & 63);
    const int N = job.N;
    const int taps = T > 0 ? T : job.T;
    const double c = job.cs[2 * k];                 // cos/dt
    const double sn = job.cs[2 * k + 1];            // sin/dt
    const double half = job.half_pix;               // (N-1)/2
    const double cd = job.centre_det;               // (D-1)/2
    const bool rows = fabs(c) >= fabs(sn);
    const double a = rows ? c : sn;                 // slope of u along the line
    const double b = rows ? sn : c;                 // slope of u across lines
    const double inv_a = 1.0 / a;
    const double r = fabs(inv_a);                   // hat half-width along the line
    const double dl = -b * inv_a;                   // change of p* from one line to the next
    // p*(l) = p0(j) + l dl on line l (y = l - half for rows, x = l - half for columns)
    auto p0_of = [&](int jj) { return ((double)jj - cd + b * half) * inv_a + half; };
    // lines on which some bin of the wave can have a nonzero weight: p* in (-r, N-1+r);
    // p0 is linear in the bin, so the wave's two end bins bound the range
    const int jl = min(jw + 63, job.D - 1);
    const double e0 = p0_of(jw), e1 = p0_of(jl);
    const double lo_p = -r, hi_p = (double)(N - 1) + r;
    int l_lo, l_hi;
    if (dl != 0.0) {
        const double la0 = (lo_p - e0) / dl, lb0 = (hi_p - e0) / dl;
        const double la1 = (lo_p - e1) / dl, lb1 = (hi_p - e1) / dl;
        const double lo = fmin(fmin(la0, lb0), fmin(la1, lb1));
        const double hi = fmax(fmax(la0, lb0), fmax(la1, lb1));
        l_lo = (int)fmin(fmax(floor(lo) - 1.0, 0.0), (double)N);
        l_hi = (int)fmax(fmin(ceil(hi) + 1.0, (double)(N - 1)), -1.0);
    } else {                                        // p* the same on every line
        const bool inside = fmax(e0, e1) > lo_p && fmin(e0, e1) < hi_p;
        l_lo = 0;
        l_hi = inside ? N - 1 : -1;
    }
    l_lo = __builtin_amdgcn_readfirstlane(l_lo);
    l_hi = __builtin_amdgcn_readfirstlane(l_hi);
    float acc = 0.0f;
    if (l_lo <= l_hi) {
        const int pitch = job.pitch;
        const size_t plane = (size_t)(N + 1) * pitch;
        const float* __restrict__ line = job.pimg + (size_t)s * 2 * plane + (rows ? 0 : plane) + (size_t)l_lo * pitch;
        // X(l) = p*(l) - r + P + 1: integer part = window start in the padded line
        const double shift = (double)job.pad + 1.0 - r;
        const double p0 = p0_of(j);
        auto anchor = [&](int l) -> uint64_t {
            const double X = p0 + (double)l * dl + shift;
            const double h = floor(X);
            const double f = fmin((X - h) * kTwo32, kTwo32 - 1.0);
            return ((uint64_t)(uint32_t)(int)h << 32) | (uint64_t)(uint32_t)f;
        };
        const uint64_t step = (uint64_t)(int64_t)llrint(dl * kTwo32);
        const uint32_t st_max = (uint32_t)(pitch - taps);
        const float aa = (float)fabs(a);
        const float na = (float)(-fabs(a) / kTwo32), pa = (float)(fabs(a) / kTwo32);
        const float c1 = (float)(fabs(a) * (2.0 - r)), c2 = (float)(2.0 - 3.0 * fabs(a));
        const float sa = (float)(-a / kTwo32);
        float cm[T > 0 ? T : 1];                    // a (1 - r + m): hat argument of tap m at phase 0
        if constexpr (T > 0) {
#pragma unroll
            for (int m = 0; m < T; ++m) cm[m] = (float)(a * (1.0 - r + (double)m));
        }
        if constexpr (T > 0) {
            auto load = [&](const float* ln, uint64_t x, float& ph, float (&v)[T]) {
                const uint32_t st = min((uint32_t)(x >> 32), st_max);    // in bounds whatever x holds
                ph = (float)(uint32_t)x;                                  // phase * 2^32
                const float* __restrict__ px = ln + st;
#pragma unroll
                for (int m = 0; m < T; ++m) v[m] = px[m];        // one T-dword load
            };
            auto accumulate = [&](float ph, const float (&v)[T]) {
                if constexpr (FAST3) {
                    const float w0 = fmaf(na, ph, aa);                    // |a| (1 - phase)
                    const float w1 = 1.0f - fabsf(fmaf(na, ph, c1));
                    const float w2 = __builtin_amdgcn_fmed3f(fmaf(pa, ph, c2), 0.0f, 1.0f);
                    acc = fmaf(w0, v[0], acc);
                    acc = fmaf(w1, v[1], acc);
                    acc = fmaf(w2, v[2], acc);
                } else {
#pragma unroll
                    for (int m = 0; m < T; ++m) {
                        const float t = fmaf(sa, ph, cm[m]);              // a (tap - p*)
                        const float w = __builtin_amdgcn_fmed3f(1.0f - fabsf(t), 0.0f, 1.0f);
                        acc = fmaf(w, v[m], acc);
                    }
                }
            };
            // lines in runs of kAnchorLines from an FP64 anchor; four lines per round,
            // all four loads issued before the first line's weights
            for (int l0 = l_lo; l0 <= l_hi; l0 += kAnchorLines) {
                const int l1 = min(l0 + kAnchorLines - 1, l_hi);
                uint64_t x = anchor(l0);
                int l = l0;
                for (; l + 3 <= l1; l += 4) {
                    float ph[4];
                    float v[4][T];
#pragma unroll
                    for (int u = 0; u < 4; ++u) {
                        load(line + u * pitch, x, ph[u], v[u]);
                        x += step;
                        asm volatile("" : "+v"(x));         // one 64-bit add per line, no unrolled copies
                    }
#pragma unroll
                    for (int u = 0; u < 4; ++u) accumulate(ph[u], v[u]);
                    line += 4 * pitch;
                }
                for (; l <= l1; ++l) {
                    float ph;
                    float v[T];
                    load(line, x, ph, v);
                    accumulate(ph, v);
                    x += step;
                    asm volatile("" : "+v"(x));
                    line += pitch;
                }
            }
        } else {
            uint64_t x = anchor(l_lo);
            for (int l = l_lo; l <= l_hi; ++l, line += pitch) {
                if (l != l_lo) x = ((l & (kAnchorLines - 1)) == 0) ? anchor(l) : x + step;
                const uint32_t st = min((uint32_t)(x >> 32), st_max);
                const float ph = (float)(uint32_t)x;
                const float* __restrict__ px = line + st;
                for (int m = 0; m < taps; ++m) {
                    const float t = fmaf(sa, ph, (float)(a * (1.0 - r + (double)m)));
                    const float w = __builtin_amdgcn_fmed3f(1.0f - fabsf(t), 0.0f, 1.0f);
                    acc = fmaf(w, px[m], acc);
                }
            }
        }
    }
    if (j < job.D) {
        const float wk = job.wscale ? job.wscale[k] * job.scale : job.scale;
        job.sino[((size_t)s * job.K + k) * job.D + j] = acc * wk;
    }
}

// Fan-beam forward projector: the adjoint of the fan-beam backprojection
//     img(X) = (2 pi / K) sum_k (R / L_k)^2 Q~_k(u_k(X)),  L_k = R - (x cos b_k + y sin b_k),
//     u_k(X) = R (-x sin b_k + y cos b_k) / (L_k ds) + (D-1)/2
// (Kak & Slaney 1988, ch. 3), i.e.
//     sino[k][j] = (2 pi / K) sum_X img(X) (R / L_k)^2 max(0, 1 - |u_k(X) - j|).
// One lane per (view, bin), walking image lines across the rays (rows when
// |sin b| >= |cos b|, else columns) in the padded copies.  On a line u - j = E / L
// with E and L linear in the position q along the line, so the bin's ray crosses
// the line at q* = -E(0) / E'.  Every pixel with a nonzero weight lies within r of
// q*, r bounding the ray spacing 1 / |du/dq| on the line grown by a margin m >= r
// (fan_line_half_width; the same for the whole block, one view and one line):
// T = floor(2r) + 1 taps from floor(q* - r) + 1.  Each tap's weight comes from the
// exact E and L at that pixel (FP64 at the line's first tap, FP32 steps after
// it), so pixels the window takes in beyond the neighbouring rays weigh zero.
// Each bin is written once by its lane, summed line by line in a fixed order; no
// atomics.
__global__ __launch_bounds__(kProjThreads) void fan_project_kernel(FanProjJob job) {
    const int nbj = (job.D + kProjThreads - 1) / kProjThreads;
    const int rest = blockIdx.x / nbj;
    const int k = rest % job.K;                     // view
    const int s = rest / job.K;                     // slice
    const int j = (blockIdx.x - rest * nbj) * kProjThreads + threadIdx.x;
    if (j >= job.D) return;                         // no barrier follows
    const int N = job.N;
    const double cb = job.cs[2 * k], sb = job.cs[2 * k + 1];
    const double R = job.R, hp = job.half_pix;
    const bool rows = fabs(sb) >= fabs(cb);
    // u - j = E / L, E = Ea + Ex x + Ey y
    const double g = job.centre_det - (double)j;
    const double Ea = g * R;
    const double Ex = -R * sb / job.ds - g * cb, Ey = R * cb / job.ds - g * sb;
    const double Eq = rows ? Ex : Ey, El = rows ? Ey : Ex;      // along the line, across lines
    const double Lq = rows ? -cb : -sb, Ll = rows ? -sb : -cb;
    const double inv_Eq = 1.0 / Eq;
    const double q_off = (double)job.pad + hp;      // padded index of line coordinate 0
    const size_t plane = (size_t)(N + 1) * job.pitch;
    const float* __restrict__ line = job.pimg + (size_t)s * 2 * plane + (rows ? 0 : plane);
    const float Eq32 = (float)Eq, Lq32 = (float)Lq, R32 = (float)R;
    const float cb32 = (float)cb, sb32 = (float)sb, ds32 = (float)job.ds, hp32 = (float)hp,
                m32 = (float)job.margin;
    float acc = 0.0f;
    for (int l = 0; l < N; ++l, line += job.pitch) {
        const double lc = (double)l - hp;
        const float r = fan_line_half_width<float>(cb32, sb32, R32, ds32, hp32, m32, (float)lc, rows);
        const int T = (int)(2.0f * r) + 1;          // floor(2r) + 1 (r > 0)
        const double qs = -(Ea + El * lc) * inv_Eq;
        // first tap, clamped into the padded line: a window that leaves the line lies
        // wholly in its zero padding (pad >= T), which the clamped window reads instead
        const int st = (int)fmin(fmax(floor(qs + q_off - (double)r) + 1.0, 0.0), (double)(job.pitch - T));
        const double q0 = (double)st - q_off;
        const float E0 = (float)(Ea + Eq * q0 + El * lc);
        const float L0 = (float)(R + Lq * q0 + Ll * lc);
        const float* __restrict__ px = line + st;
        for (int m = 0; m < T; ++m) {
            const float E = fmaf((float)m, Eq32, E0);
            const float inv = __builtin_amdgcn_rcpf(fmaf((float)m, Lq32, L0));
            const float w = fmaxf(0.0f, 1.0f - fabsf(E * inv));
            const float rl = R32 * inv;
            acc = fmaf(w * rl * rl, px[m], acc);
        }
    }
    job.sino[((size_t)s * job.K + k) * job.D + j] = acc * job.scale;
}

// Padded copies of n slices: per slice, plane 0 holds the rows and plane 1 the
// columns (transposed), each of N+1 lines of `pitch` floats: line l < N holds
// pixel p of the line at index pad + p, zeros elsewhere; line N is all zeros.
// Tiles of 64 x 64 outputs; the transposed plane goes through a padded LDS tile.
__global__ __launch_bounds__(256) void pad_kernel(const float* __restrict__ img, float* __restrict__ out, int N,
                                                  int pad, int pitch, int tiles_l, int tiles_c) {
    __shared__ float tile[kTrTile][kTrTile + 1];
    const int per_plane = tiles_l * tiles_c;
    const int q = blockIdx.x / per_plane;           // slice * 2 + plane
    const int t = blockIdx.x - q * per_plane;
    const int s = q >> 1, transposed = q & 1;
    const int l0 = (t / tiles_c) * kTrTile, c0 = (t % tiles_c) * kTrTile;   // output line, column
    const int tx = threadIdx.x & 63, ty = threadIdx.x >> 6;
    const float* src = img + (size_t)s * N * N;
    float* dst = out + (size_t)q * (N + 1) * pitch;
    if (!transposed) {
#pragma unroll
        for (int i = 0; i < kTrTile; i += 4) {
            const int l = l0 + ty + i, cc = c0 + tx, p = cc - pad;
            if (l <= N && cc < pitch)
                dst[(size_t)l * pitch + cc] = (l < N && p >= 0 && p < N) ? src[(size_t)l * N + p] : 0.0f;
        }
        return;
    }
    // output (line l = image column, index cc = pad + image row): read image rows
    // p0.. p0+63 at columns l0.. l0+63 along memory, write them transposed
    const int p0 = c0 - pad;
#pragma unroll
    for (int i = 0; i < kTrTile; i += 4) {
        const int p = p0 + ty + i, col = l0 + tx;
        tile[ty + i][tx] = (p >= 0 && p < N && col < N) ? src[(size_t)p * N + col] : 0.0f;
    }
    __syncthreads();
#pragma unroll
    for (int i = 0; i < kTrTile; i += 4) {
        const int l = l0 + ty + i, cc = c0 + tx;
        if (l <= N && cc < pitch) dst[(size_t)l * pitch + cc] = tile[tx][ty + i];
    }
}

}  // namespace

ProjLayout project_layout(const double* cs, int K, int N) {
    double r_min = INFINITY, r_max = 0.0;
    for (int k = 0; k < K; ++k) {
        const double r = 1.0 / fmax(fabs(cs[2 * k]), fabs(cs[2 * k + 1]));
        r_min = fmin(r_min, r);
        r_max = fmax(r_max, r);
    }
    ProjLayout L;
    L.fast3 = r_min >= 1.0 && r_max <= 1.5;
    L.T = L.fast3 ? 3 : (int)ceil(2.0 * r_max);
    const double pad = ceil(65.0 * r_max) + L.T + 4.0;
    const double pitch = (double)N + 2.0 * pad;
    if (!(pitch < 1e9)) {
        L.T = 0;                                    // unsupported (detector spacing far above the pixel size)
        return L;
    }
    L.pad = (int)pad;
    L.pitch = (int)pitch;
    L.slice_floats = (size_t)2 * (size_t)(N + 1) * (size_t)L.pitch;
    return L;
}

hipError_t launch_project(const ProjJob& job, int n_slices, hipStream_t stream) {
    if (n_slices <= 0) return hipSuccess;
    if (job.T < 1 || job.pitch < job.N + 2 * job.T || job.pad < job.T) return hipErrorInvalidValue;
    const int64_t blocks = (int64_t)((job.D + kProjThreads - 1) / kProjThreads) * job.K * n_slices;
    if (blocks > INT32_MAX) return hipErrorInvalidValue;
    const dim3 grid((unsigned)blocks), block(kProjThreads);
    if (job.fast3) {
        if (job.T != 3) return hipErrorInvalidValue;
        return launch_kernel(project_kernel<3, true>, grid, block, 0, stream, job);
    }
    switch (job.T) {
        case 1: return launch_kernel(project_kernel<1, false>, grid, block, 0, stream, job);
        case 2: return launch_kernel(project_kernel<2, false>, grid, block, 0, stream, job);
        case 3: return launch_kernel(project_kernel<3, false>, grid, block, 0, stream, job);
        case 4: return launch_kernel(project_kernel<4, false>, grid, block, 0, stream, job);
        default: return launch_kernel(project_kernel<0, false>, grid, block, 0, stream, job);
    }
}

hipError_t launch_fan_project(const FanProjJob& job, int n_slices, hipStream_t stream) {
    if (n_slices <= 0) return hipSuccess;
    if (job.pad < 1 || job.pitch < job.N + 2 * job.pad) return hipErrorInvalidValue;
    const int64_t blocks = (int64_t)((job.D + kProjThreads - 1) / kProjThreads) * job.K * n_slices;
    if (blocks > INT32_MAX) return hipErrorInvalidValue;
    return launch_kernel(fan_project_kernel, dim3((unsigned)blocks), dim3(kProjThreads), 0, stream, job);
}

hipError_t launch_pad(const float* img, float* out, int N, int pad, int pitch, int n_slices, hipStream_t stream) {
    if (n_slices <= 0) return hipSuccess;
    const int tiles_l = (N + 1 + kTrTile - 1) / kTrTile, tiles_c = (pitch + kTrTile - 1) / kTrTile;
    const int64_t blocks = (int64_t)tiles_l * tiles_c * 2 * n_slices;
    if (blocks > INT32_MAX) return hipErrorInvalidValue;
    return launch_kernel(pad_kernel, dim3((unsigned)blocks), dim3(256), 0, stream, img, out, N, pad, pitch, tiles_l,
                         tiles_c);
}

}  // namespace fbp
