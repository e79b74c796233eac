// Forward projector for gfx950: the exact adjoint of the backprojector.
//
// The backprojection of Eq. 2 (arXiv 2109.02174, section "Computed tomography")
// with linear interpolation is a linear map from filtered rows to pixels; its
// adjoint maps an image to projection rows:
//     sino[k][j] = w_k sum_{r,c} img[r][c] max(0, 1 - |u_k(x_c, y_r) - j|),
//     u_k(x, y) = (x cos(theta_k) + y sin(theta_k)) / dt + (D-1)/2,
// with w_k = pi/K (or the angle-gap weights).  It is computed gather-only: one lane
// per detector bin, walking the image lines across the ray direction (rows when
// |cos| >= |sin|, else columns).  On each line the pixels within one bin of u = j
// lie within 1/|a| of the crossing point (a the coordinate's slope along the
// line), at most ceil(2/|a|) + 1 of them; the crossing point is found in FP64 and
// each hat weight 1 - |a (x - x*)| in FP32 from the short difference x - x*, so
// the coordinate keeps FP32 precision far from the image centre.  Each bin is
// written once by its lane; no atomics; fixed summation order (line by line).
#include "fbp_internal.hpp"

namespace fbp {

namespace {

constexpr int kProjThreads = 256;

__global__ __launch_bounds__(kProjThreads) void project_kernel(ProjJob job) {
    // block b: (slice, angle, block of 256 bins), bins fastest
    const int nbj = (job.D + kProjThreads - 1) / kProjThreads;
    const int rest = blockIdx.x / nbj;
    const int k = rest % job.K;                     // angle
    const int s = rest / job.K;                     // slice
    const int j = (blockIdx.x - rest * nbj) * kProjThreads + threadIdx.x;
    if (j >= job.D) return;
    const int N = job.N;
    const float* __restrict__ img = job.img + (size_t)s * N * N;
    const double c = job.cs[2 * k];                 // cos/dt
    const double sn = job.cs[2 * k + 1];            // sin/dt
    const double half = job.half_pix;               // (N-1)/2
    const double cd = job.centre_det;               // (D-1)/2
    // walk along rows (step in x) when |cos| >= |sin|, else along columns (step in y)
    const bool rows = fabs(c) >= fabs(sn);
    const double a = rows ? c : sn;                 // slope of u along the line
    const double b = rows ? sn : c;                 // slope of u across lines
    const double inv_a = 1.0 / a;
    const float af = (float)a;
    const float reach = (float)fabs(inv_a);         // |x - x*| < 1/|a| for a nonzero weight
    float acc = 0.0f;
    for (int l = 0; l < N; ++l) {
        const double across = (double)l - half;     // y (rows) or x (columns) of the line
        // u = a t + b across + cd, t the along-line coordinate; crossing u = j:
        const double t_star = ((double)j - cd - b * across) * inv_a;
        const double p_star = t_star + half;        // in pixel index units
        const int lo = max(0, (int)ceil(p_star - (double)reach));
        const int hi = min(N - 1, (int)floor(p_star + (double)reach));
        const float* __restrict__ line = rows ? img + (size_t)l * N : img + l;
        const size_t step = rows ? 1 : (size_t)N;
        for (int p = lo; p <= hi; ++p) {
            const float d = (float)((double)p - p_star);
            const float w = fmaxf(0.0f, 1.0f - fabsf(af * d));
            acc = fmaf(w, line[(size_t)p * step], acc);
        }
    }
    const float wk = job.wscale ? job.wscale[k] * job.scale : job.scale;
    job.sino[((size_t)s * job.K + k) * job.D + j] = acc * wk;
}

}  // namespace

hipError_t launch_project(const ProjJob& job, int n_slices, hipStream_t stream) {
    if (n_slices <= 0) return hipSuccess;
    const int64_t blocks = (int64_t)((job.D + kProjThreads - 1) / kProjThreads) * job.K * n_slices;
    if (blocks > INT32_MAX) return hipErrorInvalidValue;
    return launch_kernel(project_kernel, dim3((unsigned)blocks), dim3(kProjThreads), 0, stream, job);
}

}  // namespace fbp
