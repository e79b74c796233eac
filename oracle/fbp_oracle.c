/*
 * FP64 CPU oracle for 2D parallel-beam filtered backprojection.
 *
 * TEST INFRASTRUCTURE ONLY.  Only the test-suite, the smoke check and the
 * CPU-baseline leg of the benchmark may load this code.  It shares no code,
 * header, table or constant generator with the HIP library: it is the plain
 * definition of what that library computes, written out slowly and in
 * double precision so that a reader can check it against the paper by eye.
 *
 * The paper (arXiv 2109.02174, section "Computed tomography") fixes:
 *   - each ray as the line  x cos(theta) + y sin(theta) = t;
 *   - the filtered projection  Q_theta(t) = P_theta(t) * H(t)  (a convolution
 *     of every projection row with a filter kernel);
 *   - the image as  f(x,y) = sum_i Q_theta_i( x cos(theta_i) + y sin(theta_i) )
 *     (Eq. 2).
 * It leaves the filter, the angular weight, the interpolation rule and the
 * grid conventions open.  The readings taken here (listed in the design
 * notes of the repository) are:
 *   - H is the band-limited ramp of Ramachandran & Lakshminarayanan (the
 *     "Ram-Lak" kernel, Kak & Slaney 1988, ch. 3):
 *         h(0) = 1/(4 dt^2),  h(d) = 0 for even d != 0,
 *         h(d) = -1/(pi^2 d^2 dt^2) for odd d,
 *     applied as a linear (not circular) convolution over the D detector
 *     bins with zero samples outside the detector, times the sample width dt;
 *   - Eq. 2 is weighted by pi/K (K angles spread over [0, pi));
 *   - Q_theta is evaluated between bins by linear interpolation, with the
 *     filtered row extended by zeros beyond both ends (so the value ramps to
 *     zero over the one bin past each end);
 *   - detector bin j sits at t_j = (j - (D-1)/2) dt; pixel (r, c) of an N x N
 *     image sits at x = c - (N-1)/2, y = r - (N-1)/2 (unit pixels), so image
 *     rows follow y and columns follow x.
 *
 * Every function returns 0 on success and -1 on invalid arguments.  Loops sum
 * in ascending index order.  Parallelism is OpenMP over independent output
 * rows only, so each output value is computed by one thread and the result
 * does not depend on the thread count.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#ifdef _OPENMP
#include <omp.h>
#endif

static const double kPi = 3.14159265358979323846264338327950288;

/* Ram-Lak kernel value h(d) for bin offset d and bin width dt. */
static double ramlak(int64_t d, double dt) {
    if (d == 0) return 1.0 / (4.0 * dt * dt);
    if (d % 2 == 0) return 0.0;
    double dd = (double)d;
    return -1.0 / (kPi * kPi * dd * dd * dt * dt);
}

/*
 * Apodised kernels (the filter variants of the same convolution):
 *   kind 0  Ram-Lak (above);
 *   kind 1  Shepp-Logan, h(d) = -2 / (pi^2 dt^2 (4 d^2 - 1))  (Kak & Slaney, ch. 3),
 *           whose response is the ramp times |sin(w/2)| / (w/2);
 *   kind 2  Hann, the Ram-Lak kernel smoothed by the taps (1/4, 1/2, 1/4):
 *           h(d) = h_RL(d)/2 + (h_RL(d-1) + h_RL(d+1))/4, whose response is the
 *           ramp times cos^2(w/2) (a raised-cosine window falling to 0 at Nyquist).
 */
static double filter_tap(int kind, int64_t d, double dt) {
    if (kind == 1) {
        const double dd = (double)d;
        return -2.0 / (kPi * kPi * dt * dt * (4.0 * dd * dd - 1.0));
    }
    if (kind == 2) return 0.5 * ramlak(d, dt) + 0.25 * (ramlak(d - 1, dt) + ramlak(d + 1, dt));
    return ramlak(d, dt);
}

int oracle_num_threads(void) {
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

void oracle_set_num_threads(int n) {
#ifdef _OPENMP
    if (n > 0) omp_set_num_threads(n);
#else
    (void)n;
#endif
}

/*
 * Filtered projections (the convolution Q = P * H of the section
 * "Computed tomography"):
 *     Q[row][n] = dt * sum_{m=0}^{D-1} h(n - m) * P[row][m],   n = 0..D-1.
 * P and Q are [n_rows][D], row-major.  P and Q must not overlap.
 */
int oracle_filter(const double* P, int64_t n_rows, int32_t D, double dt, double* Q) {
    if (!P || !Q || n_rows < 0 || D < 1 || !(dt > 0.0) || !isfinite(dt)) return -1;
    int64_t row;
#pragma omp parallel for schedule(static)
    for (row = 0; row < n_rows; ++row) {
        const double* p = P + row * (int64_t)D;
        double* q = Q + row * (int64_t)D;
        for (int32_t n = 0; n < D; ++n) {
            double acc = 0.0;
            for (int32_t m = 0; m < D; ++m) acc += ramlak((int64_t)n - m, dt) * p[m];
            q[n] = dt * acc;
        }
    }
    return 0;
}

/* oracle_filter with the kernel of the given kind (0 Ram-Lak, 1 Shepp-Logan, 2 Hann). */
int oracle_filter_kind(const double* P, int64_t n_rows, int32_t D, double dt, int32_t kind, double* Q) {
    if (!P || !Q || n_rows < 0 || D < 1 || !(dt > 0.0) || !isfinite(dt) || kind < 0 || kind > 2) return -1;
    int64_t row;
#pragma omp parallel for schedule(static)
    for (row = 0; row < n_rows; ++row) {
        const double* p = P + row * (int64_t)D;
        double* q = Q + row * (int64_t)D;
        for (int32_t n = 0; n < D; ++n) {
            double acc = 0.0;
            for (int32_t m = 0; m < D; ++m) acc += filter_tap(kind, (int64_t)n - m, dt) * p[m];
            q[n] = dt * acc;
        }
    }
    return 0;
}

/*
 * Angular quadrature weights for an arbitrary angle list (the weight of each
 * term of Eq. 2 when the angles are not evenly spaced).  Parallel rays at
 * theta and theta + pi are the same lines, so every angle is reduced to
 * [0, pi); in that sorted order each angle gets half of the gap to its
 * predecessor plus half of the gap to its successor, the gaps wrapping around
 * the half-turn.  Evenly spaced angles get pi/K each; the weights always sum
 * to pi.  Angles equal modulo pi share their gaps.
 */
int oracle_angle_weights(const double* angles, int32_t K, double* w) {
    if (!angles || !w || K < 1) return -1;
    double* a = (double*)malloc(sizeof(double) * (size_t)K);
    int32_t* order = (int32_t*)malloc(sizeof(int32_t) * (size_t)K);
    if (!a || !order) {
        free(a);
        free(order);
        return -1;
    }
    for (int32_t k = 0; k < K; ++k) {
        double t = fmod(angles[k], kPi);
        if (t < 0.0) t += kPi;
        a[k] = t;
        order[k] = k;
    }
    /* insertion sort by reduced angle, ties by index (plain and obviously correct) */
    for (int32_t i = 1; i < K; ++i) {
        const int32_t cur = order[i];
        int32_t j = i - 1;
        while (j >= 0 && (a[order[j]] > a[cur] || (a[order[j]] == a[cur] && order[j] > cur))) {
            order[j + 1] = order[j];
            --j;
        }
        order[j + 1] = cur;
    }
    for (int32_t i = 0; i < K; ++i) {
        const double prev = (i == 0) ? a[order[K - 1]] - kPi : a[order[i - 1]];
        const double next = (i == K - 1) ? a[order[0]] + kPi : a[order[i + 1]];
        w[order[i]] = 0.5 * (next - prev);
    }
    free(a);
    free(order);
    return 0;
}

/* Filtered row value at bin i, zero outside the detector. */
static double qtilde(const double* q, int32_t D, int64_t i) {
    return (i >= 0 && i < D) ? q[i] : 0.0;
}

/*
 * Backprojection (Eq. 2 with weight pi/K and linear interpolation):
 *     u = (x_c cos(theta_k) + y_r sin(theta_k)) / dt + (D-1)/2
 *     i = floor(u), alpha = u - i
 *     img[r][c] = (pi/K) * sum_k [ (1-alpha) Q~[k][i] + alpha Q~[k][i+1] ].
 * Q is [n_slices][K][D], img is [n_slices][N][N], angles holds K radians.
 */
int oracle_backproject(const double* Q, int32_t n_slices, int32_t K, int32_t D, int32_t N,
                       double dt, const double* angles, double* img) {
    if (!Q || !img || !angles || n_slices < 0 || K < 1 || D < 1 || N < 1 || !(dt > 0.0) ||
        !isfinite(dt))
        return -1;
    double* cs = (double*)malloc(sizeof(double) * 2 * (size_t)K);
    if (!cs) return -1;
    for (int32_t k = 0; k < K; ++k) {
        cs[2 * k] = cos(angles[k]);
        cs[2 * k + 1] = sin(angles[k]);
    }
    const double centre_det = 0.5 * (double)(D - 1);
    const double centre_pix = 0.5 * (double)(N - 1);
    const double weight = kPi / (double)K;
    int64_t sr;
    const int64_t n_rows = (int64_t)n_slices * N;
#pragma omp parallel for schedule(static)
    for (sr = 0; sr < n_rows; ++sr) {
        const int64_t s = sr / N;
        const int32_t r = (int32_t)(sr % N);
        const double y = (double)r - centre_pix;
        const double* qs = Q + s * (int64_t)K * D;
        double* out = img + s * (int64_t)N * N + (int64_t)r * N;
        for (int32_t c = 0; c < N; ++c) {
            const double x = (double)c - centre_pix;
            double acc = 0.0;
            for (int32_t k = 0; k < K; ++k) {
                const double u = (x * cs[2 * k] + y * cs[2 * k + 1]) / dt + centre_det;
                const double fi = floor(u);
                const double alpha = u - fi;
                const int64_t i = (int64_t)fi;
                const double* q = qs + (int64_t)k * D;
                acc += (1.0 - alpha) * qtilde(q, D, i) + alpha * qtilde(q, D, i + 1);
            }
            out[c] = weight * acc;
        }
    }
    free(cs);
    return 0;
}

/*
 * oracle_backproject with a weight per angle in place of pi/K:
 *     img[r][c] = sum_k weights[k] * [ (1-alpha) Q~[k][i] + alpha Q~[k][i+1] ].
 */
int oracle_backproject_weighted(const double* Q, int32_t n_slices, int32_t K, int32_t D, int32_t N,
                                double dt, const double* angles, const double* weights, double* img) {
    if (!Q || !img || !angles || !weights || n_slices < 0 || K < 1 || D < 1 || N < 1 || !(dt > 0.0) ||
        !isfinite(dt))
        return -1;
    const double centre_det = 0.5 * (double)(D - 1);
    const double centre_pix = 0.5 * (double)(N - 1);
    int64_t sr;
    const int64_t n_rows = (int64_t)n_slices * N;
#pragma omp parallel for schedule(static)
    for (sr = 0; sr < n_rows; ++sr) {
        const int64_t s = sr / N;
        const int32_t r = (int32_t)(sr % N);
        const double y = (double)r - centre_pix;
        const double* qs = Q + s * (int64_t)K * D;
        double* out = img + s * (int64_t)N * N + (int64_t)r * N;
        for (int32_t c = 0; c < N; ++c) {
            const double x = (double)c - centre_pix;
            double acc = 0.0;
            for (int32_t k = 0; k < K; ++k) {
                const double u = (x * cos(angles[k]) + y * sin(angles[k])) / dt + centre_det;
                const double fi = floor(u);
                const double alpha = u - fi;
                const int64_t i = (int64_t)fi;
                const double* q = qs + (int64_t)k * D;
                acc += weights[k] * ((1.0 - alpha) * qtilde(q, D, i) + alpha * qtilde(q, D, i + 1));
            }
            out[c] = acc;
        }
    }
    return 0;
}

/*
 * Whole reconstruction: filter every row, then backproject.  The filtered
 * intermediate is allocated here.  P is [n_slices][K][D].
 */
int oracle_fbp(const double* P, int32_t n_slices, int32_t K, int32_t D, int32_t N, double dt,
               const double* angles, double* img) {
    if (!P || !img || !angles || n_slices < 0 || K < 1 || D < 1 || N < 1) return -1;
    const size_t count = (size_t)n_slices * (size_t)K * (size_t)D;
    double* Q = (double*)malloc(sizeof(double) * (count ? count : 1));
    if (!Q) return -1;
    int rc = oracle_filter(P, (int64_t)n_slices * K, D, dt, Q);
    if (rc == 0) rc = oracle_backproject(Q, n_slices, K, D, N, dt, angles, img);
    free(Q);
    return rc;
}

/*
 * Splat (pixel-driven forward) projector, written from its own definition as
 * the exact adjoint of oracle_backproject, for the brute-force adjoint test:
 *     sino[k][j] = (pi/K) * sum_{r,c} img[r][c] * max(0, 1 - |u_k(x_c, y_r) - j|)
 * with u_k as in oracle_backproject.  Every detector bin j is visited for
 * every pixel (O(N^2 K D)); it is meant for tiny grids.
 * img is [n_slices][N][N], sino is [n_slices][K][D].
 */
int oracle_forward_splat(const double* img, int32_t n_slices, int32_t K, int32_t D, int32_t N,
                         double dt, const double* angles, double* sino) {
    if (!img || !sino || !angles || n_slices < 0 || K < 1 || D < 1 || N < 1 || !(dt > 0.0) ||
        !isfinite(dt))
        return -1;
    const double centre_det = 0.5 * (double)(D - 1);
    const double centre_pix = 0.5 * (double)(N - 1);
    const double weight = kPi / (double)K;
    int64_t sk;
    const int64_t n_rows = (int64_t)n_slices * K;
#pragma omp parallel for schedule(static)
    for (sk = 0; sk < n_rows; ++sk) {
        const int64_t s = sk / K;
        const int32_t k = (int32_t)(sk % K);
        const double ck = cos(angles[k]);
        const double sn = sin(angles[k]);
        const double* im = img + s * (int64_t)N * N;
        double* row = sino + sk * (int64_t)D;
        for (int32_t j = 0; j < D; ++j) {
            double acc = 0.0;
            for (int32_t r = 0; r < N; ++r) {
                const double y = (double)r - centre_pix;
                for (int32_t c = 0; c < N; ++c) {
                    const double x = (double)c - centre_pix;
                    const double u = (x * ck + y * sn) / dt + centre_det;
                    const double w = 1.0 - fabs(u - (double)j);
                    if (w > 0.0) acc += w * im[(int64_t)r * N + c];
                }
            }
            row[j] = weight * acc;
        }
    }
    return 0;
}

/* ------------------------------------------------------------------ fan beam
 *
 * Fan-beam geometry with a flat detector (the second geometry of the same
 * filtered-backprojection method; Kak & Slaney 1988, ch. 3, fan beams with
 * equally spaced collinear detectors).  Conventions:
 *   - the source of view k sits at S = R (cos b_k, sin b_k), R > 0 its distance
 *     from the rotation centre (the image centre);
 *   - the detector is the virtual line through the centre perpendicular to the
 *     central ray, with axis e = (-sin b_k, cos b_k); bin j sits at
 *     s_j = (j - (D-1)/2) ds on it;
 *   - a point X = (x, y) lies at depth L = R - (x cos b + y sin b) from the
 *     source along the central ray and is seen at s(X) = R (X . e) / L.
 * The reconstruction is
 *   1. pre-weight   P'[k][m] = P[k][m] * R / sqrt(R^2 + s_m^2);
 *   2. filter       Q[k][n]  = ds * sum_m (h(n-m)/2) * P'[k][m]   (h as above);
 *   3. backproject  img(x,y) = (2 pi / K) * sum_k (R/L)^2 * Q~[k](s(X)/ds + (D-1)/2),
 *      with the same linear interpolation and zero extension as the parallel
 *      beam (the views spread over a full turn).
 * The source must stay outside the image: R > N / sqrt(2) (the half diagonal
 * of the pixel square), so L > 0 for every pixel.
 */

static int fan_args_ok(int32_t N, double R) {
    return isfinite(R) && R > 0.70710678118654752 * (double)N;
}

/* Steps 1-2: rows of P are [n_rows][D] views; Q receives the filtered views. */
int oracle_fan_filter(const double* P, int64_t n_rows, int32_t D, double ds, double R, int32_t kind,
                      double* Q) {
    if (!P || !Q || n_rows < 0 || D < 1 || !(ds > 0.0) || !isfinite(ds) || !(R > 0.0) || !isfinite(R) ||
        kind < 0 || kind > 2)
        return -1;
    double* pw = (double*)malloc(sizeof(double) * (size_t)D);
    if (!pw) return -1;
    for (int32_t m = 0; m < D; ++m) {
        const double s = ((double)m - 0.5 * (double)(D - 1)) * ds;
        pw[m] = R / sqrt(R * R + s * s);
    }
    int64_t row;
#pragma omp parallel for schedule(static)
    for (row = 0; row < n_rows; ++row) {
        const double* p = P + row * (int64_t)D;
        double* q = Q + row * (int64_t)D;
        for (int32_t n = 0; n < D; ++n) {
            double acc = 0.0;
            for (int32_t m = 0; m < D; ++m) acc += 0.5 * filter_tap(kind, (int64_t)n - m, ds) * (pw[m] * p[m]);
            q[n] = ds * acc;
        }
    }
    free(pw);
    return 0;
}

/* Step 3: Q is [n_slices][K][D] filtered views, betas the K source angles
 * (spread over a full turn, weight 2 pi / K each). */
int oracle_fan_backproject(const double* Q, int32_t n_slices, int32_t K, int32_t D, int32_t N, double ds,
                           double R, const double* betas, double* img) {
    if (!Q || !img || !betas || n_slices < 0 || K < 1 || D < 1 || N < 1 || !(ds > 0.0) || !isfinite(ds) ||
        !fan_args_ok(N, R))
        return -1;
    const double centre_det = 0.5 * (double)(D - 1);
    const double centre_pix = 0.5 * (double)(N - 1);
    int64_t sr;
    const int64_t n_rows = (int64_t)n_slices * N;
#pragma omp parallel for schedule(static)
    for (sr = 0; sr < n_rows; ++sr) {
        const int64_t s = sr / N;
        const int32_t r = (int32_t)(sr % N);
        const double y = (double)r - centre_pix;
        const double* qs = Q + s * (int64_t)K * D;
        double* out = img + s * (int64_t)N * N + (int64_t)r * N;
        for (int32_t c = 0; c < N; ++c) {
            const double x = (double)c - centre_pix;
            double acc = 0.0;
            for (int32_t k = 0; k < K; ++k) {
                const double cb = cos(betas[k]), sb = sin(betas[k]);
                const double L = R - (x * cb + y * sb);
                const double sx = R * (-x * sb + y * cb) / L;
                const double u = sx / ds + centre_det;
                const double fi = floor(u);
                const double alpha = u - fi;
                const int64_t i = (int64_t)fi;
                const double* q = qs + (int64_t)k * D;
                const double wk = 2.0 * kPi / (double)K;
                acc += wk * (R / L) * (R / L) * ((1.0 - alpha) * qtilde(q, D, i) + alpha * qtilde(q, D, i + 1));
            }
            out[c] = acc;
        }
    }
    return 0;
}

/* Steps 1-3 with the Ram-Lak kernel and weights 2 pi / K. */
int oracle_fan_fbp(const double* P, int32_t n_slices, int32_t K, int32_t D, int32_t N, double ds, double R,
                   const double* betas, double* img) {
    if (!P || !img || !betas || n_slices < 0 || K < 1 || D < 1 || N < 1) return -1;
    const size_t count = (size_t)n_slices * (size_t)K * (size_t)D;
    double* Q = (double*)malloc(sizeof(double) * (count ? count : 1));
    if (!Q) return -1;
    int rc = oracle_fan_filter(P, (int64_t)n_slices * K, D, ds, R, 0, Q);
    if (rc == 0) rc = oracle_fan_backproject(Q, n_slices, K, D, N, ds, R, betas, img);
    free(Q);
    return rc;
}

/*
 * Adjoint of oracle_fan_backproject (weights 2 pi / K), written from its own
 * definition for the brute-force adjoint test:
 *     sino[k][j] = (2 pi / K) * sum_{r,c} img[r][c] (R/L)^2 max(0, 1 - |u_k(x_c, y_r) - j|).
 * O(N^2 K D): tiny grids only.
 */
int oracle_fan_splat(const double* img, int32_t n_slices, int32_t K, int32_t D, int32_t N, double ds, double R,
                     const double* betas, double* sino) {
    if (!img || !sino || !betas || n_slices < 0 || K < 1 || D < 1 || N < 1 || !(ds > 0.0) || !isfinite(ds) ||
        !fan_args_ok(N, R))
        return -1;
    const double centre_det = 0.5 * (double)(D - 1);
    const double centre_pix = 0.5 * (double)(N - 1);
    const double weight = 2.0 * kPi / (double)K;
    int64_t sk;
    const int64_t n_rows = (int64_t)n_slices * K;
#pragma omp parallel for schedule(static)
    for (sk = 0; sk < n_rows; ++sk) {
        const int64_t s = sk / K;
        const int32_t k = (int32_t)(sk % K);
        const double cb = cos(betas[k]), sb = sin(betas[k]);
        const double* im = img + s * (int64_t)N * N;
        double* row = sino + sk * (int64_t)D;
        for (int32_t j = 0; j < D; ++j) {
            double acc = 0.0;
            for (int32_t r = 0; r < N; ++r) {
                const double y = (double)r - centre_pix;
                for (int32_t c = 0; c < N; ++c) {
                    const double x = (double)c - centre_pix;
                    const double L = R - (x * cb + y * sb);
                    const double u = R * (-x * sb + y * cb) / L / ds + centre_det;
                    const double w = 1.0 - fabs(u - (double)j);
                    if (w > 0.0) acc += (R / L) * (R / L) * w * im[(int64_t)r * N + c];
                }
            }
            row[j] = weight * acc;
        }
    }
    return 0;
}

/* ------------------------------------------------------------------ cone beam (FDK)
 *
 * Circular cone-beam geometry with a flat detector (Feldkamp, Davis & Kress
 * 1984; Kak & Slaney 1988, ch. 3), the 3D extension of the fan beam above:
 *   - the source of view k sits at S = (R cos b_k, R sin b_k, 0);
 *   - the detector is the virtual plane through the rotation axis perpendicular
 *     to the central ray, with axes e = (-sin b_k, cos b_k, 0) (columns) and
 *     (0, 0, 1) (rows); column i sits at s_i = (i - (Du-1)/2) du, row j at
 *     z_j = (j - (Dv-1)/2) dv;
 *   - voxel (p, r, c) of an Nz x N x N volume sits at x = c - (N-1)/2,
 *     y = r - (N-1)/2, z = p - (Nz-1)/2 (unit voxels);
 *   - a point X at depth L = R - (x cos b + y sin b) is seen at
 *     s = R (x, y) . e / L and z' = R z / L.
 * The reconstruction (FDK):
 *   1. pre-weight   P'[k][j][i] = P[k][j][i] R / sqrt(R^2 + s_i^2 + z_j^2);
 *   2. filter every detector row along the columns with half the kernel (as the
 *      fan beam, bin width du);
 *   3. backproject  vol(X) = (2 pi / K) sum_k (R/L)^2 Q~_k(s/du + (Du-1)/2, z'/dv + (Dv-1)/2)
 *      with bilinear interpolation, zero beyond the detector.
 * Projections are [K][Dv][Du]; the source must stay outside the volume's
 * cylinder: R > N / sqrt(2).
 */

/* Steps 1-2 on n_views views [n_views][Dv][Du]. */
int oracle_cone_filter(const double* P, int32_t n_views, int32_t Dv, int32_t Du, double du, double dv, double R,
                       int32_t kind, double* Q) {
    if (!P || !Q || n_views < 0 || Dv < 1 || Du < 1 || !(du > 0.0) || !isfinite(du) || !(dv > 0.0) ||
        !isfinite(dv) || !(R > 0.0) || !isfinite(R) || kind < 0 || kind > 2)
        return -1;
    int64_t row;
    const int64_t n_rows = (int64_t)n_views * Dv;
#pragma omp parallel for schedule(static)
    for (row = 0; row < n_rows; ++row) {
        const int32_t j = (int32_t)(row % Dv);
        const double zj = ((double)j - 0.5 * (double)(Dv - 1)) * dv;
        const double* p = P + row * (int64_t)Du;
        double* q = Q + row * (int64_t)Du;
        for (int32_t n = 0; n < Du; ++n) {
            double acc = 0.0;
            for (int32_t m = 0; m < Du; ++m) {
                const double sm = ((double)m - 0.5 * (double)(Du - 1)) * du;
                const double w = R / sqrt(R * R + sm * sm + zj * zj);
                acc += 0.5 * filter_tap(kind, (int64_t)n - m, du) * (w * p[m]);
            }
            q[n] = du * acc;
        }
    }
    return 0;
}

/* Detector value at (column i, row j), zero off the detector. */
static double qcone(const double* q, int32_t Dv, int32_t Du, int64_t i, int64_t j) {
    return (i >= 0 && i < Du && j >= 0 && j < Dv) ? q[j * (int64_t)Du + i] : 0.0;
}

/* Step 3: Q is [K][Dv][Du] filtered views, vol is [Nz][N][N]. */
int oracle_cone_backproject(const double* Q, int32_t K, int32_t Dv, int32_t Du, int32_t N, int32_t Nz, double du,
                            double dv, double R, const double* betas, double* vol) {
    if (!Q || !vol || !betas || K < 1 || Dv < 1 || Du < 1 || N < 1 || Nz < 1 || !(du > 0.0) || !isfinite(du) ||
        !(dv > 0.0) || !isfinite(dv) || !fan_args_ok(N, R))
        return -1;
    const double cu = 0.5 * (double)(Du - 1), cv = 0.5 * (double)(Dv - 1);
    const double centre_pix = 0.5 * (double)(N - 1), centre_z = 0.5 * (double)(Nz - 1);
    const double weight = 2.0 * kPi / (double)K;
    int64_t pr;
    const int64_t n_rows = (int64_t)Nz * N;
#pragma omp parallel for schedule(static)
    for (pr = 0; pr < n_rows; ++pr) {
        const int32_t p = (int32_t)(pr / N);
        const int32_t r = (int32_t)(pr % N);
        const double z = (double)p - centre_z, y = (double)r - centre_pix;
        double* out = vol + pr * (int64_t)N;
        for (int32_t c = 0; c < N; ++c) {
            const double x = (double)c - centre_pix;
            double acc = 0.0;
            for (int32_t k = 0; k < K; ++k) {
                const double cb = cos(betas[k]), sb = sin(betas[k]);
                const double L = R - (x * cb + y * sb);
                const double u = R * (-x * sb + y * cb) / L / du + cu;
                const double v = R * z / L / dv + cv;
                const double fi = floor(u), fj = floor(v);
                const double a = u - fi, bb = v - fj;
                const int64_t i = (int64_t)fi, j = (int64_t)fj;
                const double* q = Q + (int64_t)k * Dv * Du;
                const double val = (1.0 - a) * (1.0 - bb) * qcone(q, Dv, Du, i, j) +
                                   a * (1.0 - bb) * qcone(q, Dv, Du, i + 1, j) +
                                   (1.0 - a) * bb * qcone(q, Dv, Du, i, j + 1) +
                                   a * bb * qcone(q, Dv, Du, i + 1, j + 1);
                acc += (R / L) * (R / L) * val;
            }
            out[c] = weight * acc;
        }
    }
    return 0;
}

/* Steps 1-3 (Ram-Lak). */
int oracle_cone_fdk(const double* P, int32_t K, int32_t Dv, int32_t Du, int32_t N, int32_t Nz, double du, double dv,
                    double R, const double* betas, double* vol) {
    if (!P || !vol || !betas || K < 1 || Dv < 1 || Du < 1) return -1;
    const size_t count = (size_t)K * (size_t)Dv * (size_t)Du;
    double* Q = (double*)malloc(sizeof(double) * count);
    if (!Q) return -1;
    int rc = oracle_cone_filter(P, K, Dv, Du, du, dv, R, 0, Q);
    if (rc == 0) rc = oracle_cone_backproject(Q, K, Dv, Du, N, Nz, du, dv, R, betas, vol);
    free(Q);
    return rc;
}

/* Adjoint of oracle_cone_backproject, from its own definition (tiny grids):
 *   proj[k][j][i] = (2 pi / K) sum_X vol(X) (R/L)^2 max(0, 1 - |u - i|) max(0, 1 - |v - j|). */
int oracle_cone_splat(const double* vol, int32_t K, int32_t Dv, int32_t Du, int32_t N, int32_t Nz, double du,
                      double dv, double R, const double* betas, double* proj) {
    if (!vol || !proj || !betas || K < 1 || Dv < 1 || Du < 1 || N < 1 || Nz < 1 || !(du > 0.0) || !(dv > 0.0) ||
        !fan_args_ok(N, R))
        return -1;
    const double cu = 0.5 * (double)(Du - 1), cv = 0.5 * (double)(Dv - 1);
    const double centre_pix = 0.5 * (double)(N - 1), centre_z = 0.5 * (double)(Nz - 1);
    const double weight = 2.0 * kPi / (double)K;
    int64_t kj;
    const int64_t n_rows = (int64_t)K * Dv;
#pragma omp parallel for schedule(static)
    for (kj = 0; kj < n_rows; ++kj) {
        const int32_t k = (int32_t)(kj / Dv), j = (int32_t)(kj % Dv);
        const double cb = cos(betas[k]), sb = sin(betas[k]);
        for (int32_t i = 0; i < Du; ++i) {
            double acc = 0.0;
            for (int32_t p = 0; p < Nz; ++p)
                for (int32_t r = 0; r < N; ++r)
                    for (int32_t c = 0; c < N; ++c) {
                        const double x = (double)c - centre_pix, y = (double)r - centre_pix;
                        const double z = (double)p - centre_z;
                        const double L = R - (x * cb + y * sb);
                        const double u = R * (-x * sb + y * cb) / L / du + cu;
                        const double v = R * z / L / dv + cv;
                        const double wu = 1.0 - fabs(u - (double)i), wv = 1.0 - fabs(v - (double)j);
                        if (wu > 0.0 && wv > 0.0)
                            acc += (R / L) * (R / L) * wu * wv * vol[((int64_t)p * N + r) * N + c];
                    }
            proj[kj * (int64_t)Du + i] = weight * acc;
        }
    }
    return 0;
}
