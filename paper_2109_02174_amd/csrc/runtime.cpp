// Host runtime of libfbp: argument validation, per-geometry plans, launches,
// the mixed-size batch path with captured HIP graphs, and tile autotuning.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <array>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <fstream>
#include <map>
#include <memory>
#include <mutex>
#include <sstream>
#include <string>
#include <tuple>
#include <vector>

#include "../../include/fbp.h"
#include "fbp_internal.hpp"

namespace fbp {
namespace {

constexpr double kPi = 3.14159265358979323846264338327950288;
constexpr int32_t kMaxDet = 8192;
constexpr int32_t kMaxImage = 16384;
constexpr int32_t kMaxAngles = 1 << 16;

// ------------------------------------------------------------------ validation

bool aligned4(const void* p) { return (reinterpret_cast<uintptr_t>(p) & 3u) == 0; }

bool overlaps(const void* a, size_t na, const void* b, size_t nb) {
    if (!a || !b || na == 0 || nb == 0) return false;
    const uintptr_t a0 = reinterpret_cast<uintptr_t>(a), b0 = reinterpret_cast<uintptr_t>(b);
    return a0 < b0 + nb && b0 < a0 + na;
}

int check_geom(const fbp_geom* g) {
    if (!g) return FBP_EINVAL;
    if (g->n_angles < 1 || g->n_det < 1 || g->image_size < 1) return FBP_EINVAL;
    if (!std::isfinite(g->det_spacing) || !(g->det_spacing > 0.0)) return FBP_EINVAL;
    if (!g->angles) return FBP_EINVAL;
    for (int32_t k = 0; k < g->n_angles; ++k)
        if (!std::isfinite(g->angles[k])) return FBP_EINVAL;
    if (g->filter < FBP_FILTER_RAMLAK || g->filter > FBP_FILTER_HANN) return FBP_EINVAL;
    if (g->weighting < FBP_WEIGHT_UNIFORM || g->weighting > FBP_WEIGHT_ANGLE_GAPS) return FBP_EINVAL;
    const double R = g->source_distance;
    if (!std::isfinite(R) || R < 0.0) return FBP_EINVAL;
    if (R > 0.0 && !(R > 0.70710678118654752 * (double)g->image_size)) return FBP_EINVAL;   // source in the image
    if (g->n_det > kMaxDet || g->image_size > kMaxImage || g->n_angles > kMaxAngles)
        return FBP_EUNSUPPORTED;
    if (R > 0.0 && g->weighting != FBP_WEIGHT_UNIFORM) return FBP_EUNSUPPORTED;
    return FBP_OK;
}

bool is_fan(const fbp_geom* g) { return g->source_distance > 0.0; }

int check_prec(int32_t p) { return (p == kFP32 || p == kBF16 || p == kFP16 || p == kFFT32) ? FBP_OK : FBP_EINVAL; }

size_t sino_bytes(const fbp_geom* g, int64_t n) {
    return (size_t)n * (size_t)g->n_angles * (size_t)g->n_det * sizeof(float);
}
size_t image_bytes(const fbp_geom* g, int64_t n) {
    return (size_t)n * (size_t)g->image_size * (size_t)g->image_size * sizeof(float);
}

int check_slices(const fbp_geom* g, int32_t n_slices) {
    if (n_slices < 0) return FBP_EINVAL;
    if ((int64_t)n_slices * g->n_angles > INT32_MAX) return FBP_EUNSUPPORTED;
    return FBP_OK;
}

size_t round_up(size_t x, size_t a) { return (x + a - 1) / a * a; }

// ------------------------------------------------------------------ plans

struct GeomKey {
    int device, K, D, N;
    uint64_t dt_bits;
    uint64_t angle_hash;
    int filter = 0, weighting = 0;
    uint64_t r_bits = 0;   // source distance (0: parallel beam)
    bool operator<(const GeomKey& o) const {
        return std::tie(device, K, D, N, dt_bits, angle_hash, filter, weighting, r_bits) <
               std::tie(o.device, o.K, o.D, o.N, o.dt_bits, o.angle_hash, o.filter, o.weighting, o.r_bits);
    }
};

uint64_t hash_angles(const double* a, int32_t K) {
    // 64-bit word hash (multiply-xorshift); plans also compare the full angle list,
    // so a collision can only make a lookup miss, never mix geometries.
    uint64_t h = 0x9E3779B97F4A7C15ull ^ (uint64_t)K;
    for (int32_t k = 0; k < K; ++k) {
        uint64_t w;
        std::memcpy(&w, a + k, 8);
        h = (h ^ w) * 0xBF58476D1CE4E5B9ull;
        h ^= h >> 31;
    }
    return h;
}

GeomKey make_key(int device, const fbp_geom* g) {
    GeomKey k;
    k.device = device;
    k.K = g->n_angles;
    k.D = g->n_det;
    k.N = g->image_size;
    std::memcpy(&k.dt_bits, &g->det_spacing, 8);
    k.angle_hash = hash_angles(g->angles, g->n_angles);
    k.filter = g->filter;
    k.weighting = g->weighting;
    std::memcpy(&k.r_bits, &g->source_distance, 8);
    return k;
}

// How one tile shape runs for a geometry: window length, staging segments, angle
// block, tile grid, stack kernel and angle split.
struct ShapeParams {
    int cfg = -1;
    int WL = 0, KB = 0, seg_shift = 0, tiles_x = 0, tiles_y = 0;
    int multi = 1, KBm = 0;   // slices per workgroup of the stack kernel, its angle block
    int split = 1;            // angle parts of a single slice's launch (one-group shapes)
};

// Angle-split partial sums of one slice (kMaxSplit planes of N*N floats), shared by
// every call on a plan; a call waits for the previous user's combine on its own
// stream before overwriting them.
struct PartBuffer {
    float* ptr = nullptr;
    int planes = 0;
    hipEvent_t free_ev = nullptr;
    bool recorded = false;
    std::mutex mu;
};

// Padded row and column copies of the slices being forward-projected: made on the
// first fbp_project of a plan, for up to `slices` slices at a time (at most 256 MiB
// unless one slice needs more), shared by calls in stream order like PartBuffer.
struct ProjScratch {
    ProjLayout layout;
    float* ptr = nullptr;
    int slices = 0;
    hipEvent_t free_ev = nullptr;
    bool recorded = false;
    std::mutex mu;
};

// Stream-ordered scratch rows owned by a plan (cone-beam pre-weighted views): up
// to `rows` rows of D floats at a time, shared by calls like PartBuffer.
struct RowScratch {
    float* ptr = nullptr;
    int64_t rows = 0;
    hipEvent_t free_ev = nullptr;
    bool recorded = false;
    std::mutex mu;
};

struct Plan {
    int device = 0;
    int K = 0, D = 0, N = 0;
    double dt = 1.0;
    std::vector<double> angles;
    std::vector<double> cs;          // host copy of the device table
    int Dh = 0, Dhp = 0;             // inputs per parity, and that rounded up to 64
    double* d_cs = nullptr;
    float* d_cs32 = nullptr;
    void* d_taps[3] = {nullptr, nullptr, nullptr};
    float out_scale[3] = {1.0f, 1.0f, 1.0f};
    float diag[3] = {0.0f, 0.0f, 0.0f};
    int filter = 0, weighting = 0;   // fbp_filter_kind, fbp_weighting
    float* d_wscale = nullptr;       // [K] angle weights / (pi/K) (angle-gap weighting only)
    ShapeParams one;                 // single slices and short stacks
    ShapeParams stack;               // stacks of kStackMinSlices or more slices
    PartBuffer part;
    ProjScratch proj;
    // fan beam (R > 0): source distance, FP64 (cos b, sin b), pre-weights per bin,
    // backprojection window bound and view block
    double R = 0.0;
    double* d_fcs = nullptr;
    float* d_fanw = nullptr;
    int fan_WL = 0, fan_KB = 0, fan_KB4 = 0;   // window pairs; views per block (one slice, four)
    int fan_split = 1;                          // view parts of a single slice
    bool fan_rot = false;                       // quarter-turn form (a quadrant tile and its turns)
    int fan_rot_KB = 0, fan_rot_M = 1, fan_rot_KBm = 0;   // its base views per block; stack group
    double fan_half_span = 0.0;
    // FFT filter path: twiddles and the taps' DFT for L = 2^fft_log2 (made on first use)
    float2* d_fft_tw = nullptr;
    float* d_fft_H = nullptr;
    int fft_log2 = -1;
    std::mutex mu;
};

// Stacks at least this long take the stack configuration; shorter ones go slice by
// slice through the single-slice configuration (angle-split where it has one).
constexpr int kStackMinSlices = 4;

struct Registry {
    std::mutex mu;
    std::map<GeomKey, std::unique_ptr<Plan>> plans;
    std::map<GeomKey, std::pair<int, int>> tuned;   // (single, stack) tile ids from fbp_autotune or the cache
    std::string tune_cache_loaded;      // path of the tune cache last read ("" = none)
};

Registry& registry() {
    static Registry* r = new Registry();  // never destroyed: plans live until process exit
    return *r;
}

bool angles_equal(const Plan& p, const fbp_geom* g) {
    return (int)p.angles.size() == g->n_angles &&
           std::memcmp(p.angles.data(), g->angles, sizeof(double) * (size_t)g->n_angles) == 0 &&
           p.dt == g->det_spacing && p.filter == g->filter && p.weighting == g->weighting &&
           p.R == g->source_distance;
}

// Angular quadrature of Eq. 2 for an arbitrary angle list: the lines at theta and
// theta + pi coincide, so each angle is taken modulo pi; in that order an angle's
// weight is half the distance between its two neighbours (the first and last
// wrap around the half-turn).  Returned as factors of pi/K (1 for even spacing).
std::vector<double> angle_gap_factors(const std::vector<double>& angles) {
    const size_t K = angles.size();
    std::vector<std::pair<double, size_t>> a(K);
    for (size_t k = 0; k < K; ++k) {
        double t = std::fmod(angles[k], kPi);
        if (t < 0.0) t += kPi;
        a[k] = {t, k};
    }
    std::sort(a.begin(), a.end());
    std::vector<double> f(K);
    for (size_t i = 0; i < K; ++i) {
        const double lo = (i == 0) ? a[K - 1].first - kPi : a[i - 1].first;
        const double hi = (i + 1 == K) ? a[0].first + kPi : a[i + 1].first;
        f[a[i].second] = 0.5 * (hi - lo) * (double)K / kPi;
    }
    return f;
}

double span_for(const TileShape& s, const std::vector<double>& cs) {
    double span = 0.0;
    for (size_t k = 0; k + 1 < cs.size(); k += 2)
        span = std::max(span, (s.tw - 1) * std::fabs(cs[k]) + (s.th - 1) * std::fabs(cs[k + 1]));
    return span;
}


// Angle list closed under +pi/2: theta_{k+K/2} = theta_k + pi/2 for every k < K/2.
bool quarter_turn_symmetric(const std::vector<double>& angles) {
    const size_t K = angles.size();
    if (K < 2 || (K & 1)) return false;
    const size_t h = K / 2;
    for (size_t k = 0; k < h; ++k)
        if (std::fabs(angles[k + h] - angles[k] - 0.5 * kPi) > 1e-12) return false;
    return true;
}

// Quarter-turn fan beam: LDS per workgroup for the staged windows of one slice
// (small blocks: more workgroups per CU hide the staging and barrier latency; 20 KB
// measured best of 16-48 KB at 512^2 / 720 views) and of a stack group (40 KB: two
// base views of four slices), workgroups per CU a single slice's base-view split
// aims at, stack groups tried (largest first).
constexpr size_t kFanRotLds = 20 * 1024;
constexpr size_t kFanRotLdsStack = 40 * 1024;
constexpr int kFanRotWgsPerCu = 8;
constexpr int kFanRotStackM[] = {4, 2};

// Fan-beam views in quarter turns: K = 4 K4 and b_{k + i K4} = b_k + i pi/2 (mod 2 pi)
// for every k < K4 and i = 1..3.
bool fan_quarter_turns(const std::vector<double>& angles) {
    const size_t K = angles.size();
    if (K < 4 || (K & 3)) return false;
    const size_t q = K / 4;
    for (size_t k = 0; k < q; ++k)
        for (size_t i = 1; i < 4; ++i)
            if (std::fabs(std::remainder(angles[k + i * q] - angles[k] - 0.5 * kPi * (double)i, 2.0 * kPi)) > 1e-12)
                return false;
    return true;
}

bool shape_params(int cfg, const std::vector<double>& cs, const std::vector<double>& angles, int N,
                  int cus, ShapeParams* sp) {
    const TileShape& s = tile_shape(cfg);
    sp->cfg = cfg;
    sp->split = 1;
    sp->multi = 1;
    sp->KBm = 0;
    const int waves = kGroupThreads * s.s / 64;
    if (s.rot == 2) {
        // chunked quarter-turn shape: N >= 2 (odd N: pinwheel quadrants and the
        // centre pixel), angles in quarter-turn pairs, and a window that fits this
        // id's pitch (one bin short of it: the staging pairs each bin with the next
        // lane's)
        if (N < 2 || !quarter_turn_symmetric(angles)) return false;
        double span = 0.0;   // the tile and its turn: (W-1)|c| + (H-1)|s| and (W-1)|s| + (H-1)|c|
        for (size_t k = 0; 2 * k + 1 < cs.size(); ++k) {
            const double c = std::fabs(cs[2 * k]), sn = std::fabs(cs[2 * k + 1]);
            span = std::max(span, std::max((kQtTile - 1) * c + (kQtTileH - 1) * sn, (kQtTile - 1) * sn + (kQtTileH - 1) * c));
        }
        if (!(span < 1e6)) return false;
        const int wl = window_length(span);
        const int pitch = (cfg == kQtCfg32) ? 32 : 64;
        if (wl > pitch - 1) return false;
        sp->WL = pitch;
        sp->KB = qt_block_pairs(pitch);
        sp->seg_shift = 0;
        sp->tiles_x = ((N + 1) / 2 + kQtTile - 1) / kQtTile;     // base region: (N+1)/2 columns,
        sp->tiles_y = (N / 2 + kQtTileH - 1) / kQtTileH;         // N/2 rows
        return true;
    }
    if (s.rot) {
        // quadrant tile plus its three rotations: even N, angles in quarter-turn pairs
        if ((N & 1) || !quarter_turn_symmetric(angles)) return false;
        double span = 0.0;
        for (size_t k = 0; 2 * k + 1 < cs.size(); ++k) {
            const double c = std::fabs(cs[2 * k]), sn = std::fabs(cs[2 * k + 1]);
            span = std::max(span, std::max((s.tw - 1) * c + (s.th - 1) * sn, (s.tw - 1) * sn + (s.th - 1) * c));
        }
        if (!(span < 1e6)) return false;
        sp->WL = window_length(span);
        int shift = 0;
        while (63 * (1 << shift) < sp->WL) ++shift;
        sp->seg_shift = shift;
        const int kb_stage = (kStageE * waves) >> (shift + 1);
        const int kb_lds = (kBpRotLdsBudget - kBpRotPrmBytes) / (64 * sp->WL);
        sp->KB = std::min(kMaxKB, std::min(kb_stage, kb_lds));
        if (sp->KB < 1) return false;
        const int half = N / 2;
        sp->tiles_x = (half + s.tw - 1) / s.tw;
        sp->tiles_y = (half + s.th - 1) / s.th;
        if (s.s == 1) {
            const int tiles = sp->tiles_x * sp->tiles_y;
            sp->split = std::max(1, std::min(kMaxSplit, (4 * cus + tiles - 1) / tiles));
        }
        return true;
    }
    const double span = span_for(s, cs);
    if (!(span < 1e6)) return false;
    sp->WL = window_length(span);
    // staging: one wave per (angle, 63-bin segment) per pass, kStageE passes per block
    int shift = 0;
    while (63 * (1 << shift) < sp->WL) ++shift;
    sp->seg_shift = shift;
    const int kb_stage = (stage_elems(s.s) * waves) >> shift;
    const int kb_lds = (kBpLdsBudget - kBpPrmBytes) / (16 * sp->WL);
    sp->KB = std::min(kMaxKB, std::min(kb_stage, kb_lds));
    if (sp->KB < 1) return false;
    // stack kernel: M slices' windows side by side (bin stride M | 1 float4s), one
    // staging slot per (angle, slice, segment)
    if (s.multi > 1) {
        const int m = s.multi, lm = (m == 2) ? 1 : 2;
        const int kbm_stage = (stage_elems(s.s) * waves) >> (shift + lm);
        const int kbm_lds = (kBpMultiLdsBudget - kBpPrmBytes) / (16 * sp->WL * (m | 1));
        const int kbm = std::min(kMaxKB, std::min(kbm_stage, kbm_lds));
        if (kbm >= 1 && bp_lds_bytes(cfg, m, sp->WL, kbm) <= kBpMultiLdsBudget) {
            sp->multi = m;
            sp->KBm = kbm;
        }
    }
    sp->tiles_x = (N + s.tw - 1) / s.tw;
    const int half_rows = (N + 1) / 2;
    sp->tiles_y = (half_rows + s.th - 1) / s.th;
    // one-group shapes split a single slice's angles over workgroups until there are
    // about four workgroups per CU
    if (s.s == 1) {
        const int tiles = sp->tiles_x * sp->tiles_y;
        sp->split = std::max(1, std::min(kMaxSplit, (4 * cus + tiles - 1) / tiles));
    }
    return true;
}

// Shape of a single slice without tuning (measured on MI355X): the one-group
// shapes split their angles over workgroups; the chunked quarter-turn ones need
// N >= 2 and angles closed under +pi/2.
int default_config(int N, bool quarter_turn) {
    if (quarter_turn && N >= 2) return kQtCfg32;
    if (N >= 1024) return 2;
    if (N >= 192) return 4;
    return 7;
}
int default_stack_config(int N, bool quarter_turn) {
    if (quarter_turn && N >= 2) return kQtCfg32;
    return N >= 256 ? 2 : 5;
}

bool qt_family(int cfg) { return cfg == kQtCfg32 || cfg == kQtCfg64; }

std::string tune_cache_path() {
    const char* p = std::getenv("FBP_TUNE_CACHE");
    return p ? std::string(p) : std::string();
}

std::string arch_name(int device) {
    hipDeviceProp_t prop;
    if (hipGetDeviceProperties(&prop, device) != hipSuccess) return "unknown";
    std::string a = prop.gcnArchName;
    const size_t colon = a.find(':');
    return colon == std::string::npos ? a : a.substr(0, colon);
}

// Entries of the tune cache named by FBP_TUNE_CACHE, read when a plan is created
// and the variable names a file other than the one read last.
void load_tune_cache_locked(Registry& R, int device) {
    const std::string path = tune_cache_path();
    if (path == R.tune_cache_loaded) return;
    R.tune_cache_loaded = path;
    if (path.empty()) return;
    std::ifstream in(path);
    if (!in) return;
    const std::string arch = arch_name(device);
    std::string line;
    while (std::getline(in, line)) {
        // one entry per line: arch K D N dt_bits angle_hash single_tile stack_tile filter weighting
        std::istringstream ss(line);
        std::string a;
        GeomKey k;
        int one, stack;
        unsigned long long dtb, ah;
        if (!(ss >> a >> k.K >> k.D >> k.N >> dtb >> ah >> one >> stack >> k.filter >> k.weighting)) continue;
        if (a != arch || one < 0 || one >= kNumTileConfigs || stack < 0 || stack >= kNumTileConfigs) continue;
        k.device = device;
        k.dt_bits = dtb;
        k.angle_hash = ah;
        R.tuned[k] = {one, stack};
    }
}

int env_forced_config() {
    const char* f = std::getenv("FBP_FORCE_CONFIG");
    if (!f || !*f) return -1;
    const int c = std::atoi(f);
    return (c >= 0 && c < kNumTileConfigs) ? c : -1;
}

// The HIP call behind this thread's last FBP_EHIP or FBP_ENOMEM.
thread_local char t_last_error[256] = "";

int hip_fail(hipError_t e, const char* what, int status = FBP_EHIP) {
    std::snprintf(t_last_error, sizeof t_last_error, "%s: %s (%d)", what, hipGetErrorName(e), (int)e);
    return status;
}

#define FBP_TRY_HIP(call)                                                   \
    do {                                                                    \
        const hipError_t fbp_e_ = (call);                                   \
        if (fbp_e_ != hipSuccess) return hip_fail(fbp_e_, #call);           \
    } while (0)

// Compute units of a device (cached).
int cu_count(int device) {
    static std::mutex mu;
    static std::map<int, int> counts;
    std::lock_guard<std::mutex> lock(mu);
    auto it = counts.find(device);
    if (it != counts.end()) return it->second;
    int n = 0;
    if (hipDeviceGetAttribute(&n, hipDeviceAttributeMultiprocessorCount, device) != hipSuccess || n < 1)
        n = 256;
    counts[device] = n;
    return n;
}

// The shape of tile id cfg for a plan's geometry, or of the first shape that fits.
// A chunked quarter-turn id whose window does not fit its pitch takes the other
// pitch (same arithmetic); a geometry neither fits takes the plain shapes.
bool pick_shape(int cfg, const Plan& p, int cus, ShapeParams* sp) {
    if (cfg >= 0 && cfg < kNumTileConfigs && shape_params(cfg, p.cs, p.angles, p.N, cus, sp)) return true;
    if (qt_family(cfg)) {
        if (shape_params(cfg == kQtCfg32 ? kQtCfg64 : kQtCfg32, p.cs, p.angles, p.N, cus, sp)) return true;
        if (shape_params(default_config(p.N, false), p.cs, p.angles, p.N, cus, sp)) return true;
    }
    for (int c = 0; c < kNumTileConfigs; ++c)
        if (shape_params(c, p.cs, p.angles, p.N, cus, sp)) return true;
    return false;
}

// Largest |grad s| (detector coordinate per unit of image length) over the disk
// of radius r around the centre seen from distance R:  R |X - S| / L^2, with
// |X - S|^2 = L^2 + v^2 and v^2 <= r^2 - (R - L)^2 for depth L in [R - r, R + r],
// sampled densely (the function is smooth) and padded by 1%.
double fan_max_gradient(double R, double r) {
    double g = 0.0;
    const int n = 4096;
    for (int i = 0; i <= n; ++i) {
        const double L = (R - r) + 2.0 * r * (double)i / n;
        const double v2 = std::max(0.0, r * r - (R - L) * (R - L));
        g = std::max(g, R * std::sqrt(L * L + v2) / (L * L));
    }
    return 1.01 * g;
}

// Fan-beam tables of a plan: FP64 (cos b, sin b), FP32 pre-weights R/sqrt(R^2+s^2),
// and the backprojection window bound: no pixel of a 16 x 16 tile is farther than
// (kFanTile-1)/sqrt(2) from the tile's centre, so its bin is within half_span =
// that times the largest gradient of s, over dt, of the centre's; a window from
// floor(u_centre - half_span) then needs ceil(2 half_span) + 2 pairs, plus two
// for rounding.  Views per block: up to 64 for one slice, 16 for four (four
// slices' windows; small blocks keep the LDS per workgroup low).
int make_fan_plan(Plan* p) {
    const double r = 0.70710678118654752 * (double)(p->N - 1);
    p->fan_half_span = (double)(kFanTile - 1) * 0.70710678118654752 * fan_max_gradient(p->R, r) / p->dt;
    if (!(p->fan_half_span < 2048.0)) return FBP_EUNSUPPORTED;
    p->fan_WL = (int)std::ceil(2.0 * p->fan_half_span) + 4;
    p->fan_KB = (int)std::min<size_t>(64, (kFanLdsBudget - 64 * 36) / (8 * (size_t)p->fan_WL));
    if (p->fan_KB < 1) return FBP_EUNSUPPORTED;
    p->fan_KB4 = (int)std::min<size_t>(16, (kFanLdsBudget - 64 * 36) / (4 * 8 * (size_t)p->fan_WL));
    // quarter-turn form when the views come in quarter turns (N >= 2): base views
    // per block for one slice, and the largest stack group whose block fits
    p->fan_rot = p->N >= 2 && fan_quarter_turns(p->angles) && fan_rot_addressable(p->K, p->D, p->fan_WL);
    if (p->fan_rot) {
        p->fan_rot_KB = (int)std::min<size_t>(64, kFanRotLds / fan_rot_lds_bytes(1, p->fan_WL, 1));
        p->fan_rot = p->fan_rot_KB >= 1;
        for (int m : kFanRotStackM) {
            const int kb = (int)std::min<size_t>(64, kFanRotLdsStack / fan_rot_lds_bytes(1, p->fan_WL, m));
            if (kb >= 2) {
                p->fan_rot_M = m;
                p->fan_rot_KBm = kb;
                break;
            }
        }
    }
    // single slices: views (base views) split over enough parts for about 16
    // workgroups per CU, partial sums in planes owned by the plan (images up to 2048^2)
    const int tx = p->fan_rot ? ((p->N + 1) / 2 + kFanTile - 1) / kFanTile : (p->N + kFanTile - 1) / kFanTile;
    const int ty = p->fan_rot ? (p->N / 2 + kFanTile - 1) / kFanTile : tx;
    const int tiles = tx * ty;
    const int cus = cu_count(p->device);
    const int per_cu = p->fan_rot ? kFanRotWgsPerCu : 16;
    p->fan_split = std::max(1, std::min({kMaxSplit, p->fan_rot ? p->K / 4 : p->K, (per_cu * cus + tiles / 2) / tiles}));
    const size_t plane = (size_t)p->N * p->N;
    if (p->fan_split > 1 && plane <= (size_t)2048 * 2048) {
        hipError_t e = hipMalloc(&p->part.ptr, sizeof(float) * plane * p->fan_split);
        if (e == hipSuccess) e = hipEventCreateWithFlags(&p->part.free_ev, hipEventDisableTiming);
        if (e != hipSuccess) {
            if (p->part.ptr) (void)hipFree(p->part.ptr);
            p->part.ptr = nullptr;
            return hip_fail(e, "hipMalloc (fan-beam partial sums)", FBP_ENOMEM);
        }
        p->part.planes = p->fan_split;
    } else {
        p->fan_split = 1;
    }
    std::vector<double> fcs(2 * (size_t)p->K);
    for (int k = 0; k < p->K; ++k) {
        fcs[2 * k] = std::cos(p->angles[k]);
        fcs[2 * k + 1] = std::sin(p->angles[k]);
    }
    std::vector<float> w(p->D);
    for (int m = 0; m < p->D; ++m) {
        const double sm = ((double)m - 0.5 * (double)(p->D - 1)) * p->dt;
        w[m] = (float)(p->R / std::sqrt(p->R * p->R + sm * sm));
    }
    hipError_t e = hipMalloc(&p->d_fcs, sizeof(double) * fcs.size());
    if (e == hipSuccess) e = hipMalloc(&p->d_fanw, sizeof(float) * w.size());
    if (e == hipSuccess) e = hipMemcpy(p->d_fcs, fcs.data(), sizeof(double) * fcs.size(), hipMemcpyHostToDevice);
    if (e == hipSuccess) e = hipMemcpy(p->d_fanw, w.data(), sizeof(float) * w.size(), hipMemcpyHostToDevice);
    if (e != hipSuccess) {
        if (p->d_fcs) (void)hipFree(p->d_fcs);
        if (p->d_fanw) (void)hipFree(p->d_fanw);
        p->d_fcs = nullptr;
        p->d_fanw = nullptr;
        return hip_fail(e, "fan-beam tables", FBP_ENOMEM);
    }
    return FBP_OK;
}

// Padded-copy layout of the fan-beam projector: the bound r on every line's ray
// spacing must hold on the line grown by a margin m >= r (so a bin whose ray
// crosses the grown line outside it has no pixel of the image in its window); m
// is raised until it does.  T = 0: unsupported (a detector reaching R or beyond,
// whose outer rays can run along the walked lines, or a source so close to the
// image that no margin works).
ProjLayout fan_project_layout(const Plan& p) {
    ProjLayout L;
    if (!(0.5 * (double)(p.D - 1) * p.dt < p.R)) return L;
    const double hp = 0.5 * (double)(p.N - 1);
    double m = 2.0, r_max = -1.0;
    for (int it = 0; it < 12 && r_max < 0.0; ++it) {
        double r_all = 0.0;
        for (double b : p.angles) {
            const double cb = std::cos(b), sb = std::sin(b);
            const bool rows = std::fabs(sb) >= std::fabs(cb);
            const double ext = hp + 0.5 + m;
            for (int l = 0; l < p.N; ++l) {
                const double lc = (double)l - hp;
                // the source stays beyond the grown line (L > 0 all along it)
                const double Lmin = rows ? p.R - ext * std::fabs(cb) - lc * sb : p.R - ext * std::fabs(sb) - lc * cb;
                if (!(Lmin > 0.0)) return L;
                r_all = std::max(r_all, fan_line_half_width<double>(cb, sb, p.R, p.dt, hp, m, lc, rows));
            }
        }
        if (!(r_all < 1024.0)) return L;
        if (r_all <= m) r_max = r_all;
        else m = std::ceil(r_all) + 1.0;
    }
    if (!(r_max > 0.0)) return L;
    const int T = (int)std::floor(2.0 * r_max) + 1;
    L.T = T;
    L.margin = m;
    L.pad = T + 2;                       // >= every line's tap count, whatever its rounding
    L.pitch = p.N + 2 * L.pad;
    L.slice_floats = (size_t)2 * (size_t)(p.N + 1) * (size_t)L.pitch;
    return L;
}

bool plan_matches(const Plan& p, const fbp_geom* g) {
    return p.K == g->n_angles && p.D == g->n_det && p.N == g->image_size && angles_equal(p, g);
}

// The plan this thread found last, on its device: found again without hashing the
// angle list when the next call passes the same geometry (every field and every
// angle compared).  Plans live until process exit, so the pointer stays valid.
struct LastPlan {
    int device = -1;
    Plan* plan = nullptr;
};
thread_local LastPlan t_last_plan;

int get_plan_slow(int device, const fbp_geom* g, Plan** out);

// Look up or create the plan of a validated geometry on the current device.
int get_plan(const fbp_geom* g, Plan** out) {
    int device = 0;
    FBP_TRY_HIP(hipGetDevice(&device));
    if (t_last_plan.plan && t_last_plan.device == device && plan_matches(*t_last_plan.plan, g)) {
        *out = t_last_plan.plan;
        return FBP_OK;
    }
    const int rc = get_plan_slow(device, g, out);
    if (rc == FBP_OK) t_last_plan = LastPlan{device, *out};
    return rc;
}

// Look up or create the plan (registry under its lock).
int get_plan_slow(int device, const fbp_geom* g, Plan** out) {
    const GeomKey key = make_key(device, g);
    Registry& R = registry();
    std::lock_guard<std::mutex> lock(R.mu);
    auto it = R.plans.find(key);
    if (it != R.plans.end() && angles_equal(*it->second, g)) {
        *out = it->second.get();
        return FBP_OK;
    }
    if (it != R.plans.end()) return FBP_EUNSUPPORTED;  // 64-bit hash collision: refuse, never mix
    load_tune_cache_locked(R, device);

    auto p = std::make_unique<Plan>();
    p->device = device;
    p->K = g->n_angles;
    p->D = g->n_det;
    p->N = g->image_size;
    p->dt = g->det_spacing;
    p->filter = g->filter;
    p->weighting = g->weighting;
    p->angles.assign(g->angles, g->angles + g->n_angles);
    p->cs.resize(2 * (size_t)p->K);
    for (int k = 0; k < p->K; ++k) {
        p->cs[2 * k] = std::cos(p->angles[k]) / p->dt;
        p->cs[2 * k + 1] = std::sin(p->angles[k]) / p->dt;
    }
    p->Dh = (p->D + 1) / 2;
    p->Dhp = (int)round_up((size_t)p->Dh, 64);
    p->R = g->source_distance;
    if (p->R > 0.0) {
        const int rc = make_fan_plan(p.get());
        if (rc != FBP_OK) return rc;
        *out = p.get();
        R.plans[key] = std::move(p);
        return FBP_OK;
    }
    const bool qt = quarter_turn_symmetric(p->angles);
    int one = default_config(p->N, qt), stack = default_stack_config(p->N, qt);
    auto t = R.tuned.find(key);
    if (t != R.tuned.end()) std::tie(one, stack) = t->second;
    const int forced = env_forced_config();
    if (forced >= 0) one = stack = forced;
    const int cus = cu_count(device);
    // an unsupported choice falls back to any shape whose window fits, else the geometry is refused
    if (!pick_shape(one, *p, cus, &p->one) || !pick_shape(stack, *p, cus, &p->stack)) return FBP_EUNSUPPORTED;
    std::vector<float> cs32(p->cs.size());
    for (size_t i = 0; i < cs32.size(); ++i) cs32[i] = (float)p->cs[i];
    hipError_t e = hipMalloc(&p->d_cs, sizeof(double) * p->cs.size());
    if (e != hipSuccess) return hip_fail(e, "hipMalloc (angle table)", FBP_ENOMEM);
    e = hipMalloc(&p->d_cs32, sizeof(float) * cs32.size());
    if (e != hipSuccess) {
        (void)hipFree(p->d_cs);
        return hip_fail(e, "hipMalloc (angle table)", FBP_ENOMEM);
    }
    e = hipMemcpy(p->d_cs, p->cs.data(), sizeof(double) * p->cs.size(), hipMemcpyHostToDevice);
    if (e == hipSuccess)
        e = hipMemcpy(p->d_cs32, cs32.data(), sizeof(float) * cs32.size(), hipMemcpyHostToDevice);
    if (e != hipSuccess) {
        (void)hipFree(p->d_cs);
        (void)hipFree(p->d_cs32);
        return hip_fail(e, "hipMemcpy (angle table)");
    }
    if (p->weighting == FBP_WEIGHT_ANGLE_GAPS) {
        const std::vector<double> f = angle_gap_factors(p->angles);
        std::vector<float> f32(f.begin(), f.end());
        e = hipMalloc(&p->d_wscale, sizeof(float) * f32.size());
        if (e == hipSuccess)
            e = hipMemcpy(p->d_wscale, f32.data(), sizeof(float) * f32.size(), hipMemcpyHostToDevice);
        if (e != hipSuccess) {
            (void)hipFree(p->d_cs);
            (void)hipFree(p->d_cs32);
            if (p->d_wscale) (void)hipFree(p->d_wscale);
            return hip_fail(e, "angle weights", FBP_ENOMEM);
        }
    }
    // partial sums of angle-split single slices (any shape's split fits); none for
    // images over 2048^2, which then run unsplit
    const size_t plane = (size_t)p->N * p->N;
    if (plane <= (size_t)2048 * 2048) {
        e = hipMalloc(&p->part.ptr, sizeof(float) * plane * kMaxSplit);
        if (e == hipSuccess) e = hipEventCreateWithFlags(&p->part.free_ev, hipEventDisableTiming);
        if (e != hipSuccess) {
            (void)hipFree(p->d_cs);
            (void)hipFree(p->d_cs32);
            if (p->part.ptr) (void)hipFree(p->part.ptr);
            return hip_fail(e, "hipMalloc (angle-split partial sums)", FBP_ENOMEM);
        }
        p->part.planes = kMaxSplit;
    }
    *out = p.get();
    R.plans[key] = std::move(p);
    return FBP_OK;
}

// The existing plan of a validated geometry on the current device, never creating
// one: FBP_ENOTREADY when there is none.
int find_plan(const fbp_geom* g, Plan** out) {
    int device = 0;
    FBP_TRY_HIP(hipGetDevice(&device));
    const GeomKey key = make_key(device, g);
    Registry& R = registry();
    std::lock_guard<std::mutex> lock(R.mu);
    auto it = R.plans.find(key);
    if (it == R.plans.end()) return FBP_ENOTREADY;
    if (!angles_equal(*it->second, g)) return FBP_EUNSUPPORTED;
    *out = it->second.get();
    return FBP_OK;
}

// ------------------------------------------------------------------ filter taps

uint16_t bf16_bits_rne(float x) {
    uint32_t u;
    std::memcpy(&u, &x, 4);
    u += 0x7FFFu + ((u >> 16) & 1u);
    return (uint16_t)(u >> 16);
}

uint16_t f16_bits_rne(float x) {
    _Float16 h = (_Float16)x;
    uint16_t b;
    std::memcpy(&b, &h, 2);
    return b;
}

// tap(d) = dt h(d): the Ram-Lak kernel times the bin width.
// tap(d) = dt h(d) for the plan's kernel: Ram-Lak, Shepp-Logan (Kak & Slaney,
// ch. 3) or Ram-Lak smoothed by (1/4, 1/2, 1/4) (Hann, response ramp x cos^2(w/2)).
double ramlak_tap(int d, double dt) {
    if (d == 0) return 1.0 / (4.0 * dt);
    if (d % 2 == 0) return 0.0;
    const double dd = (double)d;
    return -1.0 / (kPi * kPi * dd * dd * dt);
}

double filter_tap(int kind, int d, double dt) {
    if (kind == FBP_FILTER_SHEPP_LOGAN) {
        const double dd = (double)d;
        return -2.0 / (kPi * kPi * dt * (4.0 * dd * dd - 1.0));
    }
    if (kind == FBP_FILTER_HANN)
        return 0.5 * ramlak_tap(d, dt) + 0.25 * (ramlak_tap(d - 1, dt) + ramlak_tap(d + 1, dt));
    return ramlak_tap(d, dt);
}

// Tap tables in the operand precision, each indexed j + Dhp for j in [-Dhp, Dhp]
// (zero where the offset exceeds D - 1): the odd taps to(j) = tap(2j - 1) and, for
// kernels that do not vanish at even offsets, the even taps te(j) = tap(2j) after
// them.  Ram-Lak keeps only its centre tap, applied in FP32 in the GEMM epilogue.
// FFT path tables: L = 2^ceil(log2(2D-1)); tw[m] = e^{-2 pi i m/L}; H[f] = the DFT of
// the (even) taps, t(0) + 2 sum_{d=1}^{D-1} t(d) cos(2 pi f d / L), in FP64, times
// the output scale (1/2 for fan beam) and 1/L (the inverse transform's factor).
int ensure_fft(Plan* p) {
    std::lock_guard<std::mutex> lock(p->mu);
    if (p->d_fft_H) return FBP_OK;
    const int lg = fft_length_log2(p->D);
    if (lg > kFftMaxLog2) return FBP_EUNSUPPORTED;
    const int L = 1 << lg;
    std::vector<double> ctab(L);
    std::vector<float2> tw(L);
    for (int m = 0; m < L; ++m) {
        const double a = 2.0 * kPi * (double)m / (double)L;
        ctab[m] = std::cos(a);
        tw[m] = make_float2((float)std::cos(a), (float)-std::sin(a));
    }
    std::vector<double> t(p->D);
    for (int d = 0; d < p->D; ++d) t[d] = filter_tap(p->filter, d, p->dt);
    const double scale = (p->R > 0.0 ? 0.5 : 1.0) / (double)L;
    std::vector<float> H(L);
    for (int f = 0; f < L; ++f) {
        double acc = t[0];
        for (int d = 1; d < p->D; ++d) acc += 2.0 * t[d] * ctab[(size_t)((int64_t)f * d % L)];
        H[f] = (float)(acc * scale);
    }
    hipError_t e = hipMalloc(&p->d_fft_tw, sizeof(float2) * L);
    if (e == hipSuccess) e = hipMalloc(&p->d_fft_H, sizeof(float) * L);
    if (e == hipSuccess) e = hipMemcpy(p->d_fft_tw, tw.data(), sizeof(float2) * L, hipMemcpyHostToDevice);
    if (e == hipSuccess) e = hipMemcpy(p->d_fft_H, H.data(), sizeof(float) * L, hipMemcpyHostToDevice);
    if (e != hipSuccess) {
        if (p->d_fft_tw) (void)hipFree(p->d_fft_tw);
        if (p->d_fft_H) (void)hipFree(p->d_fft_H);
        p->d_fft_tw = nullptr;
        p->d_fft_H = nullptr;
        return hip_fail(e, "FFT filter tables", FBP_ENOMEM);
    }
    p->fft_log2 = lg;
    return FBP_OK;
}

int ensure_taps(Plan* p, int prec) {
    if (prec == kFFT32) return ensure_fft(p);
    std::lock_guard<std::mutex> lock(p->mu);
    if (p->d_taps[prec]) return FBP_OK;
    const int Dhp = p->Dhp, D = p->D;
    const bool full = p->filter != FBP_FILTER_RAMLAK;
    const size_t len = 2 * (size_t)Dhp + 1;
    std::vector<double> taps(full ? 2 * len : len, 0.0);
    for (int j = -Dhp; j <= Dhp; ++j) {
        const int d = 2 * j - 1;
        if (d >= -(D - 1) && d <= D - 1) taps[(size_t)(j + Dhp)] = filter_tap(p->filter, d, p->dt);
        if (full && 2 * j >= -(D - 1) && 2 * j <= D - 1)
            taps[len + (size_t)(j + Dhp)] = filter_tap(p->filter, 2 * j, p->dt);
    }
    const double centre = full ? 0.0 : filter_tap(p->filter, 0, p->dt);
    void* dev = nullptr;
    size_t bytes = 0;
    std::vector<float> f32;
    std::vector<uint16_t> h16;
    float out_scale = 1.0f, diag = (float)centre;
    if (prec == kFP32) {
        f32.resize(taps.size());
        for (size_t i = 0; i < taps.size(); ++i) f32[i] = (float)taps[i];
        bytes = f32.size() * 4;
    } else {
        double scale = 1.0;
        if (prec == kFP16) {
            // Pre-scale by 2^s so the smallest nonzero tap is a normal binary16 number
            // (>= 2^-14) while the largest stays below 2^15.
            double tmax = 0.0, tmin = 0.0;
            if (centre != 0.0) tmax = tmin = std::fabs(centre);
            for (double v : taps)
                if (v != 0.0) {
                    tmax = std::max(tmax, std::fabs(v));
                    tmin = (tmin == 0.0) ? std::fabs(v) : std::min(tmin, std::fabs(v));
                }
            if (tmax > 0.0) {
                int s = (int)std::ceil(-14.0 - std::log2(tmin));
                s = std::min(s, (int)std::floor(15.0 - std::log2(tmax)));
                scale = std::ldexp(1.0, s);
                out_scale = (float)std::ldexp(1.0, -s);
            }
        }
        h16.resize(taps.size());
        for (size_t i = 0; i < taps.size(); ++i) {
            const float v = (float)(taps[i] * scale);
            h16[i] = (prec == kBF16) ? bf16_bits_rne(v) : f16_bits_rne(v);
        }
        if (!full) {
            // The centre tap is applied in the FP32 epilogue, so it stays FP32 and takes
            // the value that makes the rounded kernel sum to the exact one: with rows of
            // large smooth projections, the rounded odd taps' sum error would otherwise
            // leak the rows' mean into the filtered rows.
            double exact = centre, rounded = 0.0;
            for (int d = 1; d <= D - 1; d += 2) exact += 2.0 * filter_tap(p->filter, d, p->dt);
            for (size_t i = 0; i < taps.size(); ++i) {
                if (taps[i] == 0.0) continue;
                const uint32_t u = (prec == kBF16) ? (uint32_t)h16[i] << 16 : 0u;
                float r;
                if (prec == kBF16) std::memcpy(&r, &u, 4);
                else r = (float)(_Float16)(float)(taps[i] * scale);
                rounded += (double)r;
            }
            diag = (float)(exact * scale - rounded);
        }
        bytes = h16.size() * 2;
    }
    hipError_t e = hipMalloc(&dev, bytes);
    if (e != hipSuccess) return hip_fail(e, "hipMalloc (filter taps)", FBP_ENOMEM);
    const void* src = (prec == kFP32) ? (const void*)f32.data() : (const void*)h16.data();
    e = hipMemcpy(dev, src, bytes, hipMemcpyHostToDevice);
    if (e != hipSuccess) {
        (void)hipFree(dev);
        return hip_fail(e, "hipMemcpy (filter taps)");
    }
    p->out_scale[prec] = out_scale;
    p->diag[prec] = diag;
    p->d_taps[prec] = dev;
    return FBP_OK;
}

// ------------------------------------------------------------------ launch helpers

GemmJob gemm_job(const Plan& p, int prec, const float* sino, float* filt, int rows) {
    GemmJob j{};
    j.p = sino;
    j.q = filt;
    j.taps = p.d_taps[prec];
    j.R = rows;
    j.D = p.D;
    j.Dh = p.Dh;
    j.Dhp = p.Dhp;
    j.diag = p.diag[prec];
    j.out_scale = p.out_scale[prec] * (p.R > 0.0 ? 0.5f : 1.0f);   // fan beam: half the kernel
    j.full = (p.filter != FBP_FILTER_RAMLAK) ? 1 : 0;
    j.taps_even = j.full ? static_cast<const char*>(p.d_taps[prec]) +
                               (2 * (size_t)p.Dhp + 1) * (prec == kFP32 ? 4 : 2)
                         : nullptr;
    j.tiles_n = (p.D + kGemmBN - 1) / kGemmBN;
    j.groups = 1;
    return j;
}

// Descriptor of one slice (or, with multi, of the first slice of a group).
BpJob bp_job(const Plan& p, const ShapeParams& sh, const float* filt, float* img, bool multi = false) {
    BpJob j{};
    j.q = filt;
    j.img = img;
    j.cs = p.d_cs;
    j.cs32 = p.d_cs32;
    j.half_pix = 0.5 * (double)(p.N - 1);
    j.centre_det = 0.5 * (double)(p.D - 1);
    j.N = p.N;
    j.K = p.K;
    j.D = p.D;
    j.WL = sh.WL;
    j.KB = multi ? sh.KBm : sh.KB;
    j.seg_shift = sh.seg_shift;
    j.tiles_x = sh.tiles_x;
    j.scale = (float)(kPi / (double)p.K);
    j.part = nullptr;
    j.split = 1;
    j.wscale = p.d_wscale;
    return j;
}

// Whether the filter tables of `prec` exist (ensure_taps made them).
bool taps_ready(Plan* p, int prec) {
    std::lock_guard<std::mutex> lock(p->mu);
    return prec == kFFT32 ? p->d_fft_H != nullptr : p->d_taps[prec] != nullptr;
}

int hip_status(hipError_t e, const char* what) { return e == hipSuccess ? FBP_OK : hip_fail(e, what); }

// A call that queued work on a plan-owned buffer and then failed still records the
// buffer's event, so later users of the buffer wait for the work already queued.
int fail_after_queued(int rc, hipEvent_t free_ev, bool* recorded, hipStream_t s) {
    if (hipEventRecord(free_ev, s) == hipSuccess) *recorded = true;
    return rc;
}

// rows x D: the GEMM in the operand precision, or the FFT path.
hipError_t launch_filter_rows(const Plan& p, int prec, const float* in, float* out, int rows, hipStream_t s,
                              const float* colw = nullptr) {
    if (prec == kFFT32) {
        FftJob j{};
        j.p = in;
        j.q = out;
        j.tw = p.d_fft_tw;
        j.H = p.d_fft_H;
        j.R = rows;
        j.D = p.D;
        j.log2L = p.fft_log2;
        j.colw = colw;
        return launch_fft_filter(j, s);
    }
    GemmJob j = gemm_job(p, prec, in, out, rows);
    j.colw = colw;
    if (prec == kFP32) {
        // Tile width (the same arithmetic per output bin at every width, so the same
        // bits): 32-bin tiles when even those leave each CU at most one tile (very
        // small grids); else 96-bin tiles where they leave fewer tiles on the most
        // loaded CU than 64-bin ones (in units of 32 bins)
        const int64_t tm = (rows + kGemmBM - 1) / kGemmBM, cus = cu_count(p.device);
        const int64_t t32 = tm * ((p.D + 31) / 32), t64 = tm * ((p.D + 63) / 64), t96 = tm * ((p.D + 95) / 96);
        if (t32 <= cus) {
            j.nb = 1;
            j.tiles_n = (p.D + 31) / 32;
        } else if ((t96 + cus - 1) / cus * 3 < (t64 + cus - 1) / cus * 2) {
            j.nb = 3;
            j.tiles_n = (p.D + 95) / 96;
        }
        // two groups of four waves per tile when the grid leaves about one wave per
        // SIMD (same bits as one group)
        if (tm * j.tiles_n <= cus) j.groups = 2;
    }
    return launch_gemm_grid(prec, j, s);
}

// Fan beam: the cosine pre-weights R / sqrt(R^2 + s^2) are column weights of the
// filter kernels, applied to each value as it is loaded (the same FP32 product a
// separate pre-weighting pass would store).
int run_fan_filter(Plan& p, int prec, int32_t n, const float* sino, float* filt, hipStream_t s) {
    return hip_status(launch_filter_rows(p, prec, sino, filt, n * p.K, s, p.d_fanw), "fan-beam filter launch");
}

int run_filter(Plan& p, int prec, int32_t n, const float* sino, float* filt, hipStream_t s) {
    if (n == 0) return FBP_OK;
    if (p.R > 0.0) return run_fan_filter(p, prec, n, sino, filt, s);
    return hip_status(launch_filter_rows(p, prec, sino, filt, n * p.K, s), "filter kernel launch");
}

int run_fan_backproject(Plan& p, int32_t n, const float* filt, float* img, hipStream_t s) {
    FanJob j{};
    j.q = filt;
    j.img = img;
    j.cs = p.d_fcs;
    j.R = p.R;
    j.ds = p.dt;
    j.inv_R = 1.0 / p.R;
    j.inv_dsR = 1.0 / (p.dt * p.R);
    j.half_span = p.fan_half_span;
    j.half_pix = 0.5 * (double)(p.N - 1);
    j.centre_det = 0.5 * (double)(p.D - 1);
    j.N = p.N;
    j.K = p.K;
    j.D = p.D;
    j.WL = p.fan_WL;
    j.KB = p.fan_KB;
    j.tiles_x = p.fan_rot ? ((p.N + 1) / 2 + kFanTile - 1) / kFanTile : (p.N + kFanTile - 1) / kFanTile;
    j.scale = (float)(2.0 * kPi / (double)p.K);
    j.part = nullptr;
    j.split = 1;
    if (p.fan_rot) j.KB = p.fan_rot_KB;
    auto launch = [&](const FanJob& jj, int ns, int m) {
        return p.fan_rot ? launch_fan_rot(jj, ns, m, p.fan_rot_KBm, s) : launch_fan_bp(jj, ns, m, p.fan_KB4, s);
    };
    // stacks of 4 or more share each pixel's map over several slices per workgroup
    const int M = p.fan_rot ? ((n >= kStackMinSlices && p.fan_rot_KBm >= 1) ? p.fan_rot_M : 1)
                            : ((n >= kStackMinSlices && p.fan_KB4 >= 1) ? 4 : 1);
    if (M == 1 && p.fan_split > 1 && p.part.ptr) {
        // slice by slice, the views split over parts summed in a fixed order
        PartBuffer& pb = p.part;
        std::lock_guard<std::mutex> lock(pb.mu);
        if (pb.recorded) FBP_TRY_HIP(hipStreamWaitEvent(s, pb.free_ev, 0));
        const size_t qs = (size_t)p.K * p.D, is = (size_t)p.N * p.N;
        for (int32_t i = 0; i < n; ++i) {
            FanJob ji = j;
            ji.q = filt + i * qs;
            ji.part = pb.ptr;
            ji.split = p.fan_split;
            hipError_t e = launch(ji, 1, 1);
            if (e == hipSuccess) e = launch_combine_parts(pb.ptr, img + i * is, 1, p.fan_split, is, j.scale, s);
            if (e != hipSuccess) {
                const int rc = e == hipErrorInvalidValue ? FBP_EUNSUPPORTED
                                                         : hip_status(e, "fan-beam backprojection launch");
                return i > 0 ? fail_after_queued(rc, pb.free_ev, &pb.recorded, s) : rc;
            }
        }
        FBP_TRY_HIP(hipEventRecord(pb.free_ev, s));
        pb.recorded = true;
        return FBP_OK;
    }
    const hipError_t e = launch(j, n, M);
    return e == hipErrorInvalidValue ? FBP_EUNSUPPORTED : hip_status(e, "fan-beam backprojection launch");
}

// n slices of a stack with shape sh: groups of sh.multi slices per workgroup, the
// rest one slice per workgroup; both give bitwise the same slices.
int run_stack(const Plan& p, const ShapeParams& sh, int32_t n, const float* filt, float* img, hipStream_t s) {
    const int tiles = sh.tiles_x * sh.tiles_y;
    const size_t qs = (size_t)p.K * p.D, is = (size_t)p.N * p.N;
    const int32_t grouped = (sh.multi > 1) ? n - n % sh.multi : 0;
    if (grouped > 0) {
        if ((int64_t)(grouped / sh.multi) * tiles > INT32_MAX) return FBP_EUNSUPPORTED;
        const BpJob j = bp_job(p, sh, filt, img, true);
        const int rc = hip_status(launch_bp_grid(sh.cfg, sh.multi, j, grouped, qs, is, tiles, s),
                                  "backprojection kernel launch");
        if (rc != FBP_OK) return rc;
    }
    const int32_t rest = n - grouped;
    if (rest == 0) return FBP_OK;
    if ((int64_t)rest * tiles > INT32_MAX) return FBP_EUNSUPPORTED;
    const BpJob j = bp_job(p, sh, filt + (size_t)grouped * qs, img + (size_t)grouped * is);
    return hip_status(launch_bp_grid(sh.cfg, 1, j, rest, qs, is, tiles, s), "backprojection kernel launch");
}

// One slice with shape sh.  An angle-split shape backprojects its parts into the
// partial-sum buffer (one workgroup per tile and part) and adds them in part order;
// the buffer is used by one call at a time, in stream order.
int run_single(const Plan& p, const ShapeParams& sh, PartBuffer* pb, const float* filt, float* img, hipStream_t s) {
    if (sh.split <= 1 || !pb || !pb->ptr || pb->planes < sh.split) return run_stack(p, sh, 1, filt, img, s);
    const int tiles = sh.tiles_x * sh.tiles_y;
    if ((int64_t)tiles * sh.split > INT32_MAX) return FBP_EUNSUPPORTED;
    std::lock_guard<std::mutex> lock(pb->mu);
    if (pb->recorded) FBP_TRY_HIP(hipStreamWaitEvent(s, pb->free_ev, 0));
    BpJob j = bp_job(p, sh, filt, img);
    j.part = pb->ptr;
    j.split = sh.split;
    const size_t qs = (size_t)p.K * p.D, is = (size_t)p.N * p.N;
    int rc = hip_status(launch_bp_grid(sh.cfg, 1, j, 1, qs, is, tiles, s), "backprojection kernel launch");
    if (rc != FBP_OK) return rc;
    rc = hip_status(launch_combine_parts(pb->ptr, img, 1, sh.split, is, j.scale, s), "partial-sum kernel launch");
    if (rc != FBP_OK) return fail_after_queued(rc, pb->free_ev, &pb->recorded, s);
    FBP_TRY_HIP(hipEventRecord(pb->free_ev, s));
    pb->recorded = true;
    return FBP_OK;
}

// n slices: long stacks with the stack shape, short ones slice by slice with the
// single-slice shape.
int run_backproject(Plan& p, const ShapeParams& one, const ShapeParams& stack, int32_t n, const float* filt,
                    float* img, hipStream_t s) {
    if (n == 0) return FBP_OK;
    if (p.R > 0.0) return run_fan_backproject(p, n, filt, img, s);
    if (n >= kStackMinSlices) return run_stack(p, stack, n, filt, img, s);
    const size_t qs = (size_t)p.K * p.D, is = (size_t)p.N * p.N;
    for (int32_t i = 0; i < n; ++i) {
        const int rc = run_single(p, one, &p.part, filt + (size_t)i * qs, img + (size_t)i * is, s);
        if (rc != FBP_OK) return rc;
    }
    return FBP_OK;
}

// ------------------------------------------------------------------ batch path

// Header at the start of a batch workspace.  The list kernels read their
// arguments from here, so one captured graph per workspace serves every batch.
// gemm[0] lists the Ram-Lak jobs, gemm[1] the jobs whose kernel has even taps;
// bp[c] lists single slices of tile shape c, bpm[c] groups of slices that share
// a geometry (stack kernel of shape c).
struct BatchHeader {
    GemmListArgs gemm[2];
    BpListArgs bp[kNumTileConfigs];
    BpListArgs bpm[kNumTileConfigs];
    int32_t counts[2 + 2 * kNumTileConfigs];
};

struct BatchLayout {
    size_t gemm_jobs = 0, gemm_prefix = 0;
    size_t bp_jobs = 0, bp_index = 0, bp_prefix = 0, bp_gsize = 0;
    size_t desc_end = 0;          // end of the descriptor area (the uploaded bytes)
    std::vector<size_t> q_off;    // per job: offset of its filtered rows
    size_t total = 0;
};

BatchLayout batch_layout(const fbp_job* jobs, int32_t n) {
    BatchLayout L;
    size_t o = round_up(sizeof(BatchHeader), 256);
    L.gemm_jobs = o;
    o = round_up(o + sizeof(GemmJob) * (size_t)n, 256);
    L.gemm_prefix = o;
    o = round_up(o + sizeof(int32_t) * (size_t)(n + 2), 256);
    L.bp_jobs = o;
    o = round_up(o + sizeof(BpJob) * (size_t)n, 256);
    L.bp_index = o;
    o = round_up(o + sizeof(int32_t) * (size_t)n, 256);
    L.bp_prefix = o;
    o = round_up(o + sizeof(int32_t) * (size_t)(n + 2 * kNumTileConfigs), 256);
    L.bp_gsize = o;
    o = round_up(o + sizeof(int32_t) * (size_t)n, 256);
    L.desc_end = o;
    L.q_off.resize((size_t)n);
    for (int32_t i = 0; i < n; ++i) {
        L.q_off[(size_t)i] = o;
        o = round_up(o + sino_bytes(&jobs[i].geom, 1), 256);
    }
    L.total = o;
    return L;
}

// Index of the first of jobs[0 .. n) with each distinct geometry struct (bytewise:
// the same fields and the same angle array), so that a batch checks each geometry
// and looks up its plan once; first[i] = i for the first job of a geometry.
std::vector<int32_t> first_of_geometry(const fbp_job* jobs, int32_t n) {
    using Bytes = std::array<unsigned char, sizeof(fbp_geom)>;
    std::map<Bytes, int32_t> seen;
    std::vector<int32_t> first((size_t)n);
    for (int32_t i = 0; i < n; ++i) {
        Bytes b;
        std::memcpy(b.data(), &jobs[i].geom, sizeof(fbp_geom));
        first[(size_t)i] = seen.emplace(b, i).first->second;
    }
    return first;
}

int check_jobs(const fbp_job* jobs, int32_t n) {
    if (n < 0) return FBP_EINVAL;
    if (n > 0 && !jobs) return FBP_EINVAL;
    const std::vector<int32_t> first = first_of_geometry(jobs, n);
    for (int32_t i = 0; i < n; ++i) {
        if (first[(size_t)i] == i) {
            const int rc = check_geom(&jobs[i].geom);
            if (rc != FBP_OK) return rc;
        }
        if (!jobs[i].sino || !jobs[i].image) return FBP_EINVAL;
        if (!aligned4(jobs[i].sino) || !aligned4(jobs[i].image)) return FBP_EINVAL;
        if (overlaps(jobs[i].sino, sino_bytes(&jobs[i].geom, 1), jobs[i].image,
                     image_bytes(&jobs[i].geom, 1)))
            return FBP_EINVAL;
    }
    return FBP_OK;
}

// Pinned host staging buffers for descriptor uploads; one is reused once the copy
// that last read it has completed on the device.
struct Staging {
    void* host = nullptr;
    size_t cap = 0;
    hipEvent_t done = nullptr;
    bool busy = false;
    bool recorded = false;
};

struct GraphKey {
    int device;
    int prec;
    uintptr_t ws;
    uint32_t cfg_mask;     // tile shapes with single-slice entries
    uint32_t multi_mask;   // tile shapes with slice groups
    int gemm_kinds;        // bit 0: Ram-Lak filter jobs, bit 1: jobs with even taps
    int gemm_lds;
    int bp_lds;
    int bpm_lds;
    bool operator<(const GraphKey& o) const {
        return std::tie(device, prec, ws, cfg_mask, multi_mask, gemm_kinds, gemm_lds, bp_lds, bpm_lds) <
               std::tie(o.device, o.prec, o.ws, o.cfg_mask, o.multi_mask, o.gemm_kinds, o.gemm_lds, o.bp_lds,
                        o.bpm_lds);
    }
};

struct BatchState {
    std::mutex mu;
    std::vector<std::unique_ptr<Staging>> staging;
    std::map<GraphKey, hipGraphExec_t> graphs;
    std::map<int, hipStream_t> capture_stream;   // per device, default priority
};

BatchState& batch_state() {
    static BatchState* s = new BatchState();
    return *s;
}

bool graphs_disabled() {
    const char* e = std::getenv("FBP_DISABLE_GRAPHS");
    return e && *e && *e != '0';
}

Staging* acquire_staging(size_t need) {
    BatchState& S = batch_state();
    std::lock_guard<std::mutex> lock(S.mu);
    for (auto& st : S.staging) {
        if (st->busy || st->cap < need) continue;
        if (st->recorded && hipEventQuery(st->done) != hipSuccess) continue;
        st->busy = true;
        return st.get();
    }
    auto st = std::make_unique<Staging>();
    st->cap = round_up(std::max(need, (size_t)65536), 65536);
    if (hipHostMalloc(&st->host, st->cap, hipHostMallocDefault) != hipSuccess) return nullptr;
    if (hipEventCreateWithFlags(&st->done, hipEventDisableTiming) != hipSuccess) {
        (void)hipHostFree(st->host);
        return nullptr;
    }
    st->busy = true;
    S.staging.push_back(std::move(st));
    return S.staging.back().get();
}

void release_staging(Staging* st, bool recorded) {
    BatchState& S = batch_state();
    std::lock_guard<std::mutex> lock(S.mu);
    st->recorded = recorded;
    st->busy = false;
}

// The batch kernels: grouped GEMM over every job, then persistent backprojection
// launches (slice groups first, then single slices) per tile shape present, all
// reading the header at ws.
hipError_t enqueue_batch_kernels(const GraphKey& key, int cus, hipStream_t s) {
    const BatchHeader* hdr = reinterpret_cast<const BatchHeader*>(key.ws);
    hipError_t e = hipSuccess;
    for (int kind = 0; kind < 2; ++kind) {
        if (!(key.gemm_kinds & (1 << kind))) continue;
        const int g_occ = gemm_occupancy(key.prec, kind == 1, (size_t)key.gemm_lds);
        e = launch_gemm_list(key.prec, kind == 1, &hdr->gemm[kind], cus * g_occ, (size_t)key.gemm_lds, s);
        if (e != hipSuccess) return e;
    }
    for (int c = 0; c < kNumTileConfigs; ++c) {
        if (key.multi_mask & (1u << c)) {
            const int m = tile_shape(c).multi;
            const int occ = bp_occupancy(c, m, (size_t)key.bpm_lds);
            e = launch_bp_list(c, m, &hdr->bpm[c], cus * occ, (size_t)key.bpm_lds, s);
            if (e != hipSuccess) return e;
        }
        if (key.cfg_mask & (1u << c)) {
            const int occ = bp_occupancy(c, 1, (size_t)key.bp_lds);
            e = launch_bp_list(c, 1, &hdr->bp[c], cus * occ, (size_t)key.bp_lds, s);
            if (e != hipSuccess) return e;
        }
    }
    return hipSuccess;
}

int launch_batch(const GraphKey& key, int cus, hipStream_t s) {
    if (graphs_disabled()) return hip_status(enqueue_batch_kernels(key, cus, s), "batch kernel launch");
    BatchState& S = batch_state();
    hipGraphExec_t exec = nullptr;
    {
        std::lock_guard<std::mutex> lock(S.mu);
        auto it = S.graphs.find(key);
        if (it != S.graphs.end()) exec = it->second;
    }
    if (!exec) {
        hipStream_t cs = nullptr;
        {
            std::lock_guard<std::mutex> lock(S.mu);
            auto it = S.capture_stream.find(key.device);
            if (it == S.capture_stream.end()) {
                FBP_TRY_HIP(hipStreamCreateWithFlags(&cs, hipStreamNonBlocking));
                S.capture_stream[key.device] = cs;
            } else {
                cs = it->second;
            }
        }
        std::lock_guard<std::mutex> lock(S.mu);   // one capture at a time on the shared stream
        auto it = S.graphs.find(key);
        if (it != S.graphs.end()) {
            exec = it->second;
        } else {
            hipGraph_t graph = nullptr;
            FBP_TRY_HIP(hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal));
            const hipError_t le = enqueue_batch_kernels(key, cus, cs);
            const hipError_t ce = hipStreamEndCapture(cs, &graph);
            if (le != hipSuccess || ce != hipSuccess || !graph) {
                if (graph) (void)hipGraphDestroy(graph);
                return hip_fail(le != hipSuccess ? le : ce, "batch graph capture");
            }
            const hipError_t ie = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
            (void)hipGraphDestroy(graph);
            if (ie != hipSuccess) return hip_fail(ie, "hipGraphInstantiate");
            S.graphs[key] = exec;
        }
    }
    return hip_status(hipGraphLaunch(exec, s), "hipGraphLaunch");
}

// The parallel-beam jobs of a batch (arguments checked by reconstruct_batch), with
// layout L of these jobs in ws.
int reconstruct_batch_parallel(const fbp_job* jobs, int32_t n, const BatchLayout& L, void* ws, int32_t prec,
                               hipStream_t s) {
    int rc = FBP_OK;
    std::vector<Plan*> plans((size_t)n);
    const std::vector<int32_t> first = first_of_geometry(jobs, n);
    for (int32_t i = 0; i < n; ++i) {
        const int32_t f = first[(size_t)i];
        if (f < i) {   // the same geometry struct as an earlier job: its plan
            plans[(size_t)i] = plans[(size_t)f];
            continue;
        }
        rc = get_plan(&jobs[i].geom, &plans[(size_t)i]);
        if (rc == FBP_OK) rc = ensure_taps(plans[(size_t)i], prec);
        if (rc != FBP_OK) return rc;
    }
    char* wsc = static_cast<char*>(ws);
    std::vector<char> img(L.desc_end, 0);
    BatchHeader* hdr = reinterpret_cast<BatchHeader*>(img.data());
    GemmJob* gj = reinterpret_cast<GemmJob*>(img.data() + L.gemm_jobs);
    int32_t* gp = reinterpret_cast<int32_t*>(img.data() + L.gemm_prefix);
    BpJob* bj = reinterpret_cast<BpJob*>(img.data() + L.bp_jobs);
    int32_t* bidx = reinterpret_cast<int32_t*>(img.data() + L.bp_index);
    int32_t* bpre = reinterpret_cast<int32_t*>(img.data() + L.bp_prefix);
    int32_t* bgsz = reinterpret_cast<int32_t*>(img.data() + L.bp_gsize);

    int max_dh = 0, max_bp_lds = 0, max_bpm_lds = 0;
    uint32_t mask = 0, mmask = 0;
    std::vector<float*> qptr((size_t)n);
    for (int32_t i = 0; i < n; ++i) {
        qptr[(size_t)i] = reinterpret_cast<float*>(wsc + L.q_off[(size_t)i]);
        max_dh = std::max(max_dh, plans[(size_t)i]->Dh);
    }
    // filter jobs: the Ram-Lak ones first, then those with even taps, each list with
    // its own tile prefix
    int gemm_kinds = 0;
    int32_t n_gemm[2] = {0, 0};
    {
        int pos_g = 0, pre_g = 0;
        for (int kind = 0; kind < 2; ++kind) {
            int64_t tiles = 0;
            gp[pre_g] = 0;
            for (int32_t i = 0; i < n; ++i) {
                const Plan& p = *plans[(size_t)i];
                if ((p.filter != FBP_FILTER_RAMLAK) != (kind == 1)) continue;
                gj[pos_g] = gemm_job(p, prec, jobs[i].sino, qptr[(size_t)i], p.K);
                tiles += (int64_t)((p.K + kGemmBM - 1) / kGemmBM) * gj[pos_g].tiles_n;
                if (tiles > INT32_MAX) return FBP_EUNSUPPORTED;
                ++pos_g;
                gp[pre_g + ++n_gemm[kind]] = (int32_t)tiles;
            }
            GemmListArgs& a = hdr->gemm[kind];
            a.jobs = reinterpret_cast<const GemmJob*>(wsc + L.gemm_jobs) + (pos_g - n_gemm[kind]);
            a.tile_prefix = reinterpret_cast<const int32_t*>(wsc + L.gemm_prefix) + pre_g;
            a.counts = reinterpret_cast<const int32_t*>(wsc + offsetof(BatchHeader, counts)) + kind;
            hdr->counts[kind] = n_gemm[kind];
            if (n_gemm[kind] > 0) gemm_kinds |= 1 << kind;
            pre_g += n_gemm[kind] + 1;
        }
    }
    // Jobs of a plan with kStackMinSlices or more jobs in the batch take its stack
    // shape: groups of sh.multi slices (consecutive in the job table) and the rest
    // singly; jobs of other plans go singly with the single-slice shape (unsplit: the
    // batch fills the GPU).  Each list is in descending cost order (angles x per-tile
    // work), ties by first job index.
    struct Item {
        std::vector<int32_t> jobs;
        const ShapeParams* sh;
    };
    int pos = 0, idx_off = 0, pre_off = 0, cnt_off = 2;
    auto add_list = [&](BpListArgs& a, const std::vector<Item>& items, bool multi) -> int {
        int64_t tiles = 0;
        bpre[pre_off] = 0;
        for (size_t g = 0; g < items.size(); ++g) {
            const Plan& p = *plans[(size_t)items[g].jobs[0]];
            const ShapeParams& sh = *items[g].sh;
            bidx[idx_off + (int)g] = pos;
            bgsz[idx_off + (int)g] = (int32_t)items[g].jobs.size();
            for (int32_t i : items[g].jobs) bj[pos++] = bp_job(p, sh, qptr[(size_t)i], jobs[i].image, multi);
            tiles += (int64_t)sh.tiles_x * sh.tiles_y;
            if (tiles > INT32_MAX) return FBP_EUNSUPPORTED;
            bpre[pre_off + (int)g + 1] = (int32_t)tiles;
        }
        a.jobs = reinterpret_cast<const BpJob*>(wsc + L.bp_jobs);
        a.job_index = reinterpret_cast<const int32_t*>(wsc + L.bp_index) + idx_off;
        a.tile_prefix = reinterpret_cast<const int32_t*>(wsc + L.bp_prefix) + pre_off;
        a.group_size = reinterpret_cast<const int32_t*>(wsc + L.bp_gsize) + idx_off;
        a.counts = reinterpret_cast<const int32_t*>(wsc + offsetof(BatchHeader, counts)) + cnt_off;
        hdr->counts[cnt_off] = (int32_t)items.size();
        idx_off += (int)items.size();
        pre_off += (int)items.size() + 1;
        ++cnt_off;
        return FBP_OK;
    };
    auto cost = [&](const Item& it) {
        const Plan& p = *plans[(size_t)it.jobs[0]];
        return (int64_t)p.K * (it.sh->WL + 8) * (int64_t)it.jobs.size();
    };
    auto by_cost = [&](const Item& a, const Item& b) {
        const int64_t ca = cost(a), cb = cost(b);
        return ca != cb ? ca > cb : a.jobs[0] < b.jobs[0];
    };
    std::vector<std::vector<Item>> groups(kNumTileConfigs), singles(kNumTileConfigs);
    {
        std::map<const Plan*, std::vector<int32_t>> by_plan;   // job order kept per plan
        std::vector<const Plan*> order;                       // plans in order of first job
        for (int32_t i = 0; i < n; ++i) {
            auto& v = by_plan[plans[(size_t)i]];
            if (v.empty()) order.push_back(plans[(size_t)i]);
            v.push_back(i);
        }
        for (const Plan* pp : order) {
            const Plan& p = *pp;
            const std::vector<int32_t>& v = by_plan[pp];
            const bool stacked = (int)v.size() >= kStackMinSlices;
            const ShapeParams& sh = stacked ? p.stack : p.one;
            const size_t m = stacked ? (size_t)sh.multi : 1;
            const size_t grouped = (m > 1) ? v.size() - v.size() % m : 0;
            for (size_t g = 0; g < grouped; g += m)
                groups[(size_t)sh.cfg].push_back({std::vector<int32_t>(v.begin() + (ptrdiff_t)g,
                                                                       v.begin() + (ptrdiff_t)(g + m)), &sh});
            for (size_t g = grouped; g < v.size(); ++g) singles[(size_t)sh.cfg].push_back({{v[g]}, &sh});
            if (grouped > 0) max_bpm_lds = std::max(max_bpm_lds, bp_lds_bytes(sh.cfg, sh.multi, sh.WL, sh.KBm));
            if (grouped < v.size()) max_bp_lds = std::max(max_bp_lds, bp_lds_bytes(sh.cfg, 1, sh.WL, sh.KB));
        }
    }
    for (int c = 0; c < kNumTileConfigs; ++c) {
        std::stable_sort(groups[(size_t)c].begin(), groups[(size_t)c].end(), by_cost);
        std::stable_sort(singles[(size_t)c].begin(), singles[(size_t)c].end(), by_cost);
        if (!groups[(size_t)c].empty()) mmask |= 1u << c;
        if (!singles[(size_t)c].empty()) mask |= 1u << c;
        rc = add_list(hdr->bpm[c], groups[(size_t)c], true);
        if (rc == FBP_OK) rc = add_list(hdr->bp[c], singles[(size_t)c], false);
        if (rc != FBP_OK) return rc;
    }

    Staging* st = acquire_staging(L.desc_end);
    if (!st) return FBP_ENOMEM;
    std::memcpy(st->host, img.data(), L.desc_end);
    hipError_t e = hipMemcpyAsync(ws, st->host, L.desc_end, hipMemcpyHostToDevice, s);
    if (e == hipSuccess) e = hipEventRecord(st->done, s);
    release_staging(st, e == hipSuccess);
    if (e != hipSuccess) return hip_fail(e, "batch descriptor upload");

    int device = 0;
    FBP_TRY_HIP(hipGetDevice(&device));
    GraphKey key;
    key.device = device;
    key.prec = prec;
    key.ws = reinterpret_cast<uintptr_t>(ws);
    key.cfg_mask = mask;
    key.multi_mask = mmask;
    key.gemm_kinds = gemm_kinds;
    key.gemm_lds = (int)round_up((size_t)gemm_lds_bytes(prec, max_dh, (gemm_kinds & 2) != 0), 8192);
    key.bp_lds = (int)round_up((size_t)max_bp_lds, 4096);
    key.bpm_lds = (int)round_up((size_t)max_bpm_lds, 4096);
    return launch_batch(key, cu_count(device), s);
}

int reconstruct_batch(const fbp_job* jobs, int32_t n, void* ws, size_t ws_bytes, int32_t prec,
                      hipStream_t s) {
    int rc = check_jobs(jobs, n);
    if (rc == FBP_OK) rc = check_prec(prec);
    if (rc != FBP_OK) return rc;
    if (prec == kFFT32) return FBP_EUNSUPPORTED;     // batches filter through grouped GEMMs
    if (n == 0) return FBP_OK;
    const BatchLayout L = batch_layout(jobs, n);
    if (!ws || ws_bytes < L.total) return FBP_EWORKSPACE;
    if ((reinterpret_cast<uintptr_t>(ws) & 255u) != 0) return FBP_EINVAL;
    std::vector<std::pair<uintptr_t, size_t>> imgs((size_t)n);
    for (int32_t i = 0; i < n; ++i) {
        if (overlaps(ws, L.total, jobs[i].sino, sino_bytes(&jobs[i].geom, 1)) ||
            overlaps(ws, L.total, jobs[i].image, image_bytes(&jobs[i].geom, 1)))
            return FBP_EINVAL;
        imgs[(size_t)i] = {reinterpret_cast<uintptr_t>(jobs[i].image), image_bytes(&jobs[i].geom, 1)};
    }
    // images must not overlap each other: in address order each starts at or past
    // the furthest end of those before it
    std::sort(imgs.begin(), imgs.end());
    uintptr_t end = 0;
    for (const auto& iv : imgs) {
        if (iv.first < end) return FBP_EINVAL;
        end = std::max(end, iv.first + iv.second);
    }
    std::vector<fbp_job> par;
    std::vector<int32_t> fan;
    for (int32_t i = 0; i < n; ++i) {
        if (is_fan(&jobs[i].geom)) fan.push_back(i);
        else par.push_back(jobs[i]);
    }
    if (fan.empty()) return reconstruct_batch_parallel(jobs, n, L, ws, prec, s);
    // Fan-beam jobs: after the parallel-beam ones (laid out as a batch of their own
    // at the start of ws, which is no larger than L's descriptors and rows), one by
    // one through the fan-beam filter and backprojection, each with its rows in the
    // space after them; every image is bitwise fbp_reconstruct of the slice alone.
    size_t o = 0;
    if (!par.empty()) {
        const BatchLayout Lp = batch_layout(par.data(), (int32_t)par.size());
        rc = reconstruct_batch_parallel(par.data(), (int32_t)par.size(), Lp, ws, prec, s);
        if (rc != FBP_OK) return rc;
        o = Lp.total;
    }
    char* wsc = static_cast<char*>(ws);
    for (int32_t i : fan) {
        Plan* p = nullptr;
        rc = get_plan(&jobs[i].geom, &p);
        if (rc == FBP_OK) rc = ensure_taps(p, prec);
        if (rc != FBP_OK) return rc;
        float* filt = reinterpret_cast<float*>(wsc + o);
        o = round_up(o + sino_bytes(&jobs[i].geom, 1), 256);
        rc = run_fan_filter(*p, prec, 1, jobs[i].sino, filt, s);
        if (rc == FBP_OK) rc = run_fan_backproject(*p, 1, filt, jobs[i].image, s);
        if (rc != FBP_OK) return rc;
    }
    return FBP_OK;
}

// ------------------------------------------------------------------ autotuning

// Device buffers and events of one tuning run, released on every exit path.
struct TuneScratch {
    float* q = nullptr;
    float* im = nullptr;
    double* dcs = nullptr;
    float* dcs32 = nullptr;
    PartBuffer part;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    hipStream_t s = nullptr;
    ~TuneScratch() {
        (void)hipStreamSynchronize(s);
        if (e0) (void)hipEventDestroy(e0);
        if (e1) (void)hipEventDestroy(e1);
        if (part.free_ev) (void)hipEventDestroy(part.free_ev);
        if (part.ptr) (void)hipFree(part.ptr);
        if (q) (void)hipFree(q);
        if (im) (void)hipFree(im);
        if (dcs) (void)hipFree(dcs);
        if (dcs32) (void)hipFree(dcs32);
    }
};

constexpr int kTuneStackSlices = 16;

// Time every tile shape that supports the geometry, on zero slices (7 runs, minimum
// of the last 5): one slice through the single-slice path, and a stack of
// kTuneStackSlices through the stack path.  Keeps the fastest of each.
int time_tile_shapes(const fbp_geom* g, const std::vector<double>& cs, hipStream_t s, int* best_one,
                     int* best_stack) {
    TuneScratch t;
    t.s = s;
    const size_t qb = sino_bytes(g, kTuneStackSlices), ib = image_bytes(g, kTuneStackSlices);
    const size_t plane = (size_t)g->image_size * (size_t)g->image_size;
    std::vector<float> cs32(cs.size());
    for (size_t i = 0; i < cs.size(); ++i) cs32[i] = (float)cs[i];
    hipError_t e = hipMalloc(&t.q, qb);
    if (e == hipSuccess) e = hipMalloc(&t.im, ib);
    if (e == hipSuccess) e = hipMalloc(&t.dcs, sizeof(double) * cs.size());
    if (e == hipSuccess) e = hipMalloc(&t.dcs32, sizeof(float) * cs32.size());
    if (e == hipSuccess && plane <= (size_t)2048 * 2048) {
        e = hipMalloc(&t.part.ptr, sizeof(float) * plane * kMaxSplit);
        t.part.planes = kMaxSplit;
    }
    if (e != hipSuccess) return hip_fail(e, "hipMalloc (autotune scratch)", FBP_ENOMEM);
    FBP_TRY_HIP(hipEventCreateWithFlags(&t.part.free_ev, hipEventDisableTiming));
    FBP_TRY_HIP(hipMemcpy(t.dcs, cs.data(), sizeof(double) * cs.size(), hipMemcpyHostToDevice));
    FBP_TRY_HIP(hipMemcpy(t.dcs32, cs32.data(), sizeof(float) * cs32.size(), hipMemcpyHostToDevice));
    FBP_TRY_HIP(hipMemsetAsync(t.q, 0, qb, s));
    FBP_TRY_HIP(hipEventCreate(&t.e0));
    FBP_TRY_HIP(hipEventCreate(&t.e1));
    Plan p;   // scratch plan for the timing runs
    p.K = g->n_angles;
    p.D = g->n_det;
    p.N = g->image_size;
    p.dt = g->det_spacing;
    p.cs = cs;
    p.angles.assign(g->angles, g->angles + g->n_angles);
    p.d_cs = t.dcs;
    p.d_cs32 = t.dcs32;
    int device = 0;
    FBP_TRY_HIP(hipGetDevice(&device));
    const int cus = cu_count(device);
    auto time_ms = [&](auto&& run, float* out) -> int {
        float ms_min = 1e30f;
        for (int rep = 0; rep < 7; ++rep) {
            FBP_TRY_HIP(hipEventRecord(t.e0, s));
            const int rc = run();
            if (rc != FBP_OK) return rc;
            FBP_TRY_HIP(hipEventRecord(t.e1, s));
            FBP_TRY_HIP(hipEventSynchronize(t.e1));
            float ms = 0.0f;
            FBP_TRY_HIP(hipEventElapsedTime(&ms, t.e0, t.e1));
            if (rep >= 2) ms_min = std::min(ms_min, ms);   // first two runs warm up
        }
        *out = ms_min;
        return FBP_OK;
    };
    *best_one = *best_stack = -1;
    float one_ms = 0.0f, stack_ms = 0.0f;
    // where a chunked quarter-turn shape fits, only its window pitches are timed:
    // they give the same bits, so the choice moves time but never the result
    bool qt_fits = false;
    for (int c : {kQtCfg32, kQtCfg64}) {
        ShapeParams sp;
        qt_fits = qt_fits || shape_params(c, cs, p.angles, p.N, cus, &sp);
    }
    for (int c = 0; c < kNumTileConfigs; ++c) {
        ShapeParams sp;
        if (qt_fits != qt_family(c)) continue;
        if (!shape_params(c, cs, p.angles, p.N, cus, &sp)) continue;
        float ms = 0.0f;
        int rc = time_ms([&] { return run_single(p, sp, &t.part, t.q, t.im, s); }, &ms);
        if (rc != FBP_OK) return rc;
        if (*best_one < 0 || ms < one_ms) {
            *best_one = c;
            one_ms = ms;
        }
        rc = time_ms([&] { return run_stack(p, sp, kTuneStackSlices, t.q, t.im, s); }, &ms);
        if (rc != FBP_OK) return rc;
        if (*best_stack < 0 || ms < stack_ms) {
            *best_stack = c;
            stack_ms = ms;
        }
    }
    return FBP_OK;
}

int autotune(const fbp_geom* g, hipStream_t s, int32_t* out_cfg) {
    int rc = check_geom(g);
    if (rc != FBP_OK) return rc;
    if (is_fan(g)) {   // one fan-beam kernel: nothing to tune
        if (out_cfg) *out_cfg = -1;
        return FBP_OK;
    }
    int device = 0;
    FBP_TRY_HIP(hipGetDevice(&device));
    std::vector<double> cs(2 * (size_t)g->n_angles);
    for (int k = 0; k < g->n_angles; ++k) {
        cs[2 * k] = std::cos(g->angles[k]) / g->det_spacing;
        cs[2 * k + 1] = std::sin(g->angles[k]) / g->det_spacing;
    }
    int one = -1, stack = -1;
    rc = time_tile_shapes(g, cs, s, &one, &stack);
    if (rc != FBP_OK) return rc;
    if (one < 0 || stack < 0) return FBP_EUNSUPPORTED;
    {
        Registry& R = registry();
        std::lock_guard<std::mutex> lock(R.mu);
        const GeomKey key = make_key(device, g);
        R.tuned[key] = {one, stack};
        const std::string path = tune_cache_path();
        if (!path.empty()) {
            std::ofstream out(path, std::ios::app);
            if (out)
                out << arch_name(device) << ' ' << key.K << ' ' << key.D << ' ' << key.N << ' '
                    << (unsigned long long)key.dt_bits << ' ' << (unsigned long long)key.angle_hash << ' '
                    << one << ' ' << stack << ' ' << key.filter << ' ' << key.weighting << '\n';
        }
    }
    if (out_cfg) *out_cfg = one;
    return FBP_OK;
}

// ------------------------------------------------------------------ cone beam (FDK)

int check_cone_geom(const fbp_cone_geom* g) {
    if (!g) return FBP_EINVAL;
    if (g->n_views < 1 || g->n_det_u < 1 || g->n_det_v < 1 || g->volume_size < 1 || g->volume_depth < 1)
        return FBP_EINVAL;
    if (!std::isfinite(g->det_spacing_u) || !(g->det_spacing_u > 0.0)) return FBP_EINVAL;
    if (!std::isfinite(g->det_spacing_v) || !(g->det_spacing_v > 0.0)) return FBP_EINVAL;
    if (!g->angles) return FBP_EINVAL;
    for (int32_t k = 0; k < g->n_views; ++k)
        if (!std::isfinite(g->angles[k])) return FBP_EINVAL;
    if (g->filter < FBP_FILTER_RAMLAK || g->filter > FBP_FILTER_HANN) return FBP_EINVAL;
    const double R = g->source_distance;
    if (!std::isfinite(R) || !(R > 0.70710678118654752 * (double)g->volume_size)) return FBP_EINVAL;
    if (g->n_det_u > kMaxDet || g->n_det_v > kMaxDet || g->volume_size > kMaxImage ||
        g->volume_depth > kMaxImage || g->n_views > kMaxAngles)
        return FBP_EUNSUPPORTED;
    if ((int64_t)g->n_views * g->n_det_v > INT32_MAX) return FBP_EUNSUPPORTED;
    return FBP_OK;
}

size_t cone_proj_bytes(const fbp_cone_geom* g) {
    return sizeof(float) * (size_t)g->n_views * (size_t)g->n_det_v * (size_t)g->n_det_u;
}
size_t cone_vol_bytes(const fbp_cone_geom* g) {
    return sizeof(float) * (size_t)g->volume_depth * (size_t)g->volume_size * (size_t)g->volume_size;
}

struct ConeKey {
    int device, K, Du, Dv, N, Nz, filter;
    uint64_t du_bits, dv_bits, r_bits, angle_hash;
    bool operator<(const ConeKey& o) const {
        return std::tie(device, K, Du, Dv, N, Nz, filter, du_bits, dv_bits, r_bits, angle_hash) <
               std::tie(o.device, o.K, o.Du, o.Dv, o.N, o.Nz, o.filter, o.du_bits, o.dv_bits, o.r_bits, o.angle_hash);
    }
};

// Plan of one cone-beam geometry: the row filter's taps (a one-angle parallel-beam
// plan over the Du columns), FP64 (cos b, sin b), FP32 pre-weights
// R / sqrt(R^2 + s^2 + z^2) per detector cell, the staged window bounds and a
// scratch buffer for the pre-weighted views.
struct ConePlan {
    int K = 0, Du = 0, Dv = 0, N = 0, Nz = 0, filter = 0;
    double du = 1.0, dv = 1.0, R = 0.0;
    std::vector<double> angles;
    Plan* taps = nullptr;
    double* d_cs = nullptr;
    float* d_pw = nullptr;
    int WL = 0, WV = 0, KB = 0, pitch = 0, cap = 0;
    bool staged = true;
    double half_span = 0.0;
    RowScratch rows;
};

struct ConeRegistry {
    std::mutex mu;
    std::map<ConeKey, std::unique_ptr<ConePlan>> plans;
};

ConeRegistry& cone_registry() {
    static ConeRegistry* r = new ConeRegistry();   // never destroyed: plans live until process exit
    return *r;
}

// Window bounds.  Columns: as the fan beam (a 16 x 16 column tile's shadow is at
// most (kConeTile-1) sqrt(2) max|grad s| / du columns wide).  Rows: over a block of
// kConeZB slices and a tile, v = z rho / dv + (Dv-1)/2 with rho = R/L in
// [rho_lo, rho_hi]; the span is at most ((kConeZB-1) rho_max + max|z| drho) / dv,
// rho_max = R/(R - r) and drho <= (tile diagonal) R/(R - r)^2 (|grad L| = 1,
// |grad rho| = R/L^2).  The kernel's per-view windows (floors, a cell of margin on
// each side, the bilinear neighbour and one spare row) then stay within WL + 1
// columns and WV + 1 rows.  A workgroup's LDS holds cap floats of windows packed
// by their row counts; the windows go through LDS when the largest one fits.
int make_cone_plan(ConePlan* c) {
    const double r = 0.70710678118654752 * (double)(c->N - 1);
    const double diag = (double)(kConeTile - 1) * 1.4142135623730951;
    c->half_span = 0.5 * diag * fan_max_gradient(c->R, r) / c->du;
    const double rho_max = c->R / (c->R - r);
    const double drho = diag * c->R / ((c->R - r) * (c->R - r));
    const double span_v = ((double)(kConeZB - 1) * rho_max + 0.5 * (double)(c->Nz - 1) * drho) / c->dv;
    if (!(c->half_span < 1e6) || !(span_v < 1e6)) return FBP_EUNSUPPORTED;
    c->WL = (int)std::ceil(2.0 * c->half_span) + 4;
    c->WV = (int)std::ceil(span_v) + 5;
    c->pitch = cone_pitch(c->Du % 4 == 0 ? c->WL + 6 : c->WL);   // room for windows aligned to four columns
    c->KB = 16;
    c->cap = (int)((kConeLdsBudget - cone_lds_bytes(c->KB, 0, false)) / sizeof(float));
    c->staged = (int64_t)(c->WV + 1) * c->pitch <= c->cap;   // windows through LDS, else direct reads
    std::vector<double> cs(2 * (size_t)c->K);
    for (int k = 0; k < c->K; ++k) {
        cs[2 * k] = std::cos(c->angles[k]);
        cs[2 * k + 1] = std::sin(c->angles[k]);
    }
    std::vector<float> pw((size_t)c->Dv * c->Du);
    for (int j = 0; j < c->Dv; ++j) {
        const double zj = ((double)j - 0.5 * (double)(c->Dv - 1)) * c->dv;
        for (int i = 0; i < c->Du; ++i) {
            const double si = ((double)i - 0.5 * (double)(c->Du - 1)) * c->du;
            pw[(size_t)j * c->Du + i] = (float)(c->R / std::sqrt(c->R * c->R + si * si + zj * zj));
        }
    }
    hipError_t e = hipMalloc(&c->d_cs, sizeof(double) * cs.size());
    if (e == hipSuccess) e = hipMalloc(&c->d_pw, sizeof(float) * pw.size());
    if (e == hipSuccess) e = hipMemcpy(c->d_cs, cs.data(), sizeof(double) * cs.size(), hipMemcpyHostToDevice);
    if (e == hipSuccess) e = hipMemcpy(c->d_pw, pw.data(), sizeof(float) * pw.size(), hipMemcpyHostToDevice);
    if (e == hipSuccess) e = hipEventCreateWithFlags(&c->rows.free_ev, hipEventDisableTiming);
    if (e != hipSuccess) {
        if (c->d_cs) (void)hipFree(c->d_cs);
        if (c->d_pw) (void)hipFree(c->d_pw);
        c->d_cs = nullptr;
        c->d_pw = nullptr;
        return hip_fail(e, "cone-beam tables", FBP_ENOMEM);
    }
    return FBP_OK;
}

int get_cone_plan(const fbp_cone_geom* g, ConePlan** out) {
    // the taps come from a one-angle parallel-beam plan over the detector columns
    const double zero = 0.0;
    fbp_geom pg{};
    pg.n_angles = 1;
    pg.n_det = g->n_det_u;
    pg.image_size = 1;
    pg.det_spacing = g->det_spacing_u;
    pg.angles = &zero;
    pg.filter = g->filter;
    Plan* taps = nullptr;
    int rc = get_plan(&pg, &taps);
    if (rc == FBP_OK) rc = ensure_taps(taps, kFP32);
    if (rc != FBP_OK) return rc;
    int device = 0;
    FBP_TRY_HIP(hipGetDevice(&device));
    ConeKey key{device, g->n_views, g->n_det_u, g->n_det_v, g->volume_size, g->volume_depth, g->filter, 0, 0, 0,
                hash_angles(g->angles, g->n_views)};
    std::memcpy(&key.du_bits, &g->det_spacing_u, 8);
    std::memcpy(&key.dv_bits, &g->det_spacing_v, 8);
    std::memcpy(&key.r_bits, &g->source_distance, 8);
    ConeRegistry& CR = cone_registry();
    std::lock_guard<std::mutex> lock(CR.mu);
    auto it = CR.plans.find(key);
    if (it != CR.plans.end()) {
        if ((int)it->second->angles.size() != g->n_views ||
            std::memcmp(it->second->angles.data(), g->angles, sizeof(double) * (size_t)g->n_views) != 0)
            return FBP_EUNSUPPORTED;   // 64-bit hash collision: refuse, never mix
        *out = it->second.get();
        return FBP_OK;
    }
    auto c = std::make_unique<ConePlan>();
    c->K = g->n_views;
    c->Du = g->n_det_u;
    c->Dv = g->n_det_v;
    c->N = g->volume_size;
    c->Nz = g->volume_depth;
    c->filter = g->filter;
    c->du = g->det_spacing_u;
    c->dv = g->det_spacing_v;
    c->R = g->source_distance;
    c->angles.assign(g->angles, g->angles + g->n_views);
    c->taps = taps;
    rc = make_cone_plan(c.get());
    if (rc != FBP_OK) return rc;
    *out = c.get();
    CR.plans[key] = std::move(c);
    return FBP_OK;
}

// Pre-weight (through the plan's scratch, at most 64 MiB of views at a time) and
// filter every detector row with half the kernel.
int run_cone_filter(ConePlan& c, const float* proj, float* filt, hipStream_t s) {
    RowScratch& rs = c.rows;
    std::lock_guard<std::mutex> lock(rs.mu);
    const int64_t per_view = (int64_t)c.Dv * c.Du;
    if (!rs.ptr) {
        const int64_t views = std::max<int64_t>(1, std::min<int64_t>(c.K, ((int64_t)64 << 20) / (4 * per_view)));
        const hipError_t e = hipMalloc(&rs.ptr, sizeof(float) * (size_t)(views * per_view));
        if (e != hipSuccess) {
            rs.ptr = nullptr;
            return hip_fail(e, "hipMalloc (cone-beam scratch)", FBP_ENOMEM);
        }
        rs.rows = views;
    }
    if (rs.recorded) FBP_TRY_HIP(hipStreamWaitEvent(s, rs.free_ev, 0));
    bool queued = false;
    for (int64_t k0 = 0; k0 < c.K; k0 += rs.rows) {
        const int64_t m = std::min<int64_t>(rs.rows, c.K - k0);
        const size_t off = (size_t)(k0 * per_view);
        hipError_t e = launch_preweight(proj + off, rs.ptr, c.d_pw, m, (int)per_view, s);
        if (e == hipSuccess) {
            queued = true;
            GemmJob j = gemm_job(*c.taps, kFP32, rs.ptr, filt + off, (int)(m * c.Dv));
            j.out_scale *= 0.5f;                                       // half the kernel
            e = launch_gemm_grid(kFP32, j, s);
        }
        if (e != hipSuccess) {
            const int rc = hip_status(e, "cone-beam filter launch");
            return queued ? fail_after_queued(rc, rs.free_ev, &rs.recorded, s) : rc;
        }
    }
    FBP_TRY_HIP(hipEventRecord(rs.free_ev, s));
    rs.recorded = true;
    return FBP_OK;
}

int run_cone_backproject(const ConePlan& c, const float* filt, float* vol, hipStream_t s) {
    ConeJob j{};
    j.q = filt;
    j.vol = vol;
    j.cs = c.d_cs;
    j.R = c.R;
    j.du = c.du;
    j.dv = c.dv;
    j.inv_R = 1.0 / c.R;
    j.inv_duR = 1.0 / (c.du * c.R);
    j.half_span = c.half_span;
    j.cu = 0.5 * (double)(c.Du - 1);
    j.cv = 0.5 * (double)(c.Dv - 1);
    j.half_pix = 0.5 * (double)(c.N - 1);
    j.half_z = 0.5 * (double)(c.Nz - 1);
    j.N = c.N;
    j.Nz = c.Nz;
    j.K = c.K;
    j.Du = c.Du;
    j.Dv = c.Dv;
    j.WL = c.WL;
    j.WV = c.WV;
    j.pitch = c.pitch;
    j.KB = c.KB;
    j.cap = c.cap;
    j.vec4 = c.staged && c.Du % 4 == 0 && c.pitch % 4 == 0 && c.pitch >= c.WL + 7 &&
             reinterpret_cast<uintptr_t>(filt) % 16 == 0;
    j.tiles_x = (c.N + kConeTile - 1) / kConeTile;
    j.scale = (float)(2.0 * kPi / (double)c.K);
    const hipError_t e = launch_cone_bp(j, c.staged, s);
    return e == hipErrorInvalidValue ? FBP_EUNSUPPORTED : hip_status(e, "cone-beam backprojection launch");
}

}  // namespace

int current_device_cus() {
    int device = 0;
    if (hipGetDevice(&device) != hipSuccess) return 256;
    return cu_count(device);
}

}  // namespace fbp

// ====================================================================== C ABI

using namespace fbp;

extern "C" {

const char* fbp_status_string(int status) {
    switch (status) {
        case FBP_OK: return "ok";
        case FBP_EINVAL: return "invalid argument";
        case FBP_ENOMEM: return "out of memory";
        case FBP_EHIP: return "HIP runtime error";
        case FBP_EUNSUPPORTED: return "unsupported geometry or size";
        case FBP_EWORKSPACE: return "workspace missing or too small";
        case FBP_ENOTREADY: return "no plan or filter taps for this geometry and precision yet";
        default: return "unknown status";
    }
}

const char* fbp_version(void) { return "fbp-mi355x 0.1 (gfx950)"; }

const char* fbp_last_error(void) { return t_last_error; }

int32_t fbp_num_tile_configs(void) { return kNumTileConfigs; }

const char* fbp_tile_config_name(int32_t id) {
    if (id < 0 || id >= kNumTileConfigs) return "invalid tile id";
    return tile_shape(id).name;
}

size_t fbp_workspace_bytes(const fbp_geom* geom, int32_t n_slices, int32_t precision) {
    if (check_geom(geom) != FBP_OK || check_prec(precision) != FBP_OK ||
        check_slices(geom, n_slices) != FBP_OK)
        return 0;
    return round_up(sino_bytes(geom, n_slices), 256);
}

size_t fbp_batch_workspace_bytes(const fbp_job* jobs, int32_t n_jobs, int32_t precision) {
    if (check_prec(precision) != FBP_OK || precision == kFFT32 || n_jobs < 0 || (n_jobs > 0 && !jobs)) return 0;
    const std::vector<int32_t> first = first_of_geometry(jobs, n_jobs);
    for (int32_t i = 0; i < n_jobs; ++i)
        if (first[(size_t)i] == i && check_geom(&jobs[i].geom) != FBP_OK) return 0;
    return batch_layout(jobs, n_jobs).total;
}

int fbp_filter(const fbp_geom* geom, int32_t n_slices, const float* d_sino, float* d_filtered,
               int32_t precision, void* hip_stream) {
    int rc = check_geom(geom);
    if (rc == FBP_OK) rc = check_prec(precision);
    if (rc == FBP_OK) rc = check_slices(geom, n_slices);
    if (rc != FBP_OK) return rc;
    if (n_slices == 0) return FBP_OK;
    if (!d_sino || !d_filtered || !aligned4(d_sino) || !aligned4(d_filtered)) return FBP_EINVAL;
    const size_t nb = sino_bytes(geom, n_slices);
    if (overlaps(d_sino, nb, d_filtered, nb)) return FBP_EINVAL;
    Plan* p = nullptr;
    rc = get_plan(geom, &p);
    if (rc == FBP_OK) rc = ensure_taps(p, precision);
    if (rc != FBP_OK) return rc;
    return run_filter(*p, precision, n_slices, d_sino, d_filtered, (hipStream_t)hip_stream);
}

int fbp_backproject(const fbp_geom* geom, int32_t n_slices, const float* d_filtered, float* d_image,
                    void* hip_stream) {
    int rc = check_geom(geom);
    if (rc == FBP_OK) rc = check_slices(geom, n_slices);
    if (rc != FBP_OK) return rc;
    if (n_slices == 0) return FBP_OK;
    if (!d_filtered || !d_image || !aligned4(d_filtered) || !aligned4(d_image)) return FBP_EINVAL;
    if (overlaps(d_filtered, sino_bytes(geom, n_slices), d_image, image_bytes(geom, n_slices)))
        return FBP_EINVAL;
    Plan* p = nullptr;
    rc = get_plan(geom, &p);
    if (rc != FBP_OK) return rc;
    return run_backproject(*p, p->one, p->stack, n_slices, d_filtered, d_image, (hipStream_t)hip_stream);
}

int fbp_reconstruct(const fbp_geom* geom, int32_t n_slices, const float* d_sino, float* d_image,
                    void* d_workspace, size_t workspace_bytes, int32_t precision, void* hip_stream) {
    int rc = check_geom(geom);
    if (rc == FBP_OK) rc = check_prec(precision);
    if (rc == FBP_OK) rc = check_slices(geom, n_slices);
    if (rc != FBP_OK) return rc;
    if (n_slices == 0) return FBP_OK;
    if (!d_sino || !d_image || !aligned4(d_sino) || !aligned4(d_image)) return FBP_EINVAL;
    const size_t sb = sino_bytes(geom, n_slices), ib = image_bytes(geom, n_slices);
    if (overlaps(d_sino, sb, d_image, ib)) return FBP_EINVAL;
    if (!d_workspace || workspace_bytes < sb) return FBP_EWORKSPACE;
    if ((reinterpret_cast<uintptr_t>(d_workspace) & 255u) != 0) return FBP_EINVAL;
    if (overlaps(d_workspace, sb, d_sino, sb) || overlaps(d_workspace, sb, d_image, ib))
        return FBP_EINVAL;
    Plan* p = nullptr;
    rc = get_plan(geom, &p);
    if (rc == FBP_OK) rc = ensure_taps(p, precision);
    if (rc != FBP_OK) return rc;
    float* filt = static_cast<float*>(d_workspace);
    const hipStream_t s = (hipStream_t)hip_stream;
    rc = run_filter(*p, precision, n_slices, d_sino, filt, s);
    if (rc == FBP_OK) rc = run_backproject(*p, p->one, p->stack, n_slices, filt, d_image, s);
    return rc;
}

int fbp_reconstruct_noalloc(const fbp_geom* geom, int32_t n_slices, const float* d_sino, float* d_image,
                            int32_t precision, void* hip_stream) {
    int rc = check_geom(geom);
    if (rc == FBP_OK) rc = check_prec(precision);
    if (rc == FBP_OK) rc = check_slices(geom, n_slices);
    if (rc != FBP_OK) return rc;
    if (n_slices == 0) return FBP_OK;
    if (!d_sino || !d_image || !aligned4(d_sino) || !aligned4(d_image)) return FBP_EINVAL;
    const size_t sb = sino_bytes(geom, n_slices), ib = image_bytes(geom, n_slices);
    if (overlaps(d_sino, sb, d_image, ib)) return FBP_EINVAL;
    if (sb > FBP_NOALLOC_WORKSPACE_BYTES) return FBP_EWORKSPACE;
    Plan* p = nullptr;
    rc = find_plan(geom, &p);
    if (rc != FBP_OK) return rc;
    if (!taps_ready(p, precision)) return FBP_ENOTREADY;
    void* ws = nullptr;
    size_t ws_bytes = 0;
    const hipError_t e = noalloc_workspace(&ws, &ws_bytes);
    if (e != hipSuccess) return hip_fail(e, "hipGetSymbolAddress (static workspace)");
    if (ws_bytes < sb) return FBP_EWORKSPACE;
    float* filt = static_cast<float*>(ws);
    const hipStream_t s = (hipStream_t)hip_stream;
    rc = run_filter(*p, precision, n_slices, d_sino, filt, s);
    if (rc == FBP_OK) rc = run_backproject(*p, p->one, p->stack, n_slices, filt, d_image, s);
    return rc;
}

int fbp_project(const fbp_geom* geom, int32_t n_slices, const float* d_image, float* d_sino, void* hip_stream) {
    int rc = check_geom(geom);
    if (rc == FBP_OK) rc = check_slices(geom, n_slices);
    if (rc != FBP_OK) return rc;
    if (n_slices == 0) return FBP_OK;
    if (!d_image || !d_sino || !aligned4(d_image) || !aligned4(d_sino)) return FBP_EINVAL;
    if (overlaps(d_image, image_bytes(geom, n_slices), d_sino, sino_bytes(geom, n_slices))) return FBP_EINVAL;
    Plan* p = nullptr;
    rc = get_plan(geom, &p);
    if (rc != FBP_OK) return rc;
    const bool fan = p->R > 0.0;
    ProjScratch& ps = p->proj;
    std::lock_guard<std::mutex> lock(ps.mu);
    if (!ps.ptr) {
        ps.layout = fan ? fan_project_layout(*p) : project_layout(p->cs.data(), p->K, p->N);
        if (ps.layout.T == 0) return FBP_EUNSUPPORTED;
        const size_t slice_bytes = sizeof(float) * ps.layout.slice_floats;
        const int slices = (int)std::max<size_t>(1, std::min<size_t>(16, ((size_t)256 << 20) / slice_bytes));
        hipError_t e = hipMalloc(&ps.ptr, slice_bytes * (size_t)slices);
        if (e == hipSuccess) e = hipEventCreateWithFlags(&ps.free_ev, hipEventDisableTiming);
        if (e != hipSuccess) {
            if (ps.ptr) (void)hipFree(ps.ptr);
            ps.ptr = nullptr;
            return hip_fail(e, "hipMalloc (projector copies)", FBP_ENOMEM);
        }
        ps.slices = slices;
    }
    const hipStream_t s = (hipStream_t)hip_stream;
    const ProjLayout& L = ps.layout;
    ProjJob j{};
    FanProjJob fj{};
    if (fan) {
        fj.pimg = ps.ptr;
        fj.cs = p->d_fcs;
        fj.R = p->R;
        fj.ds = p->dt;
        fj.half_pix = 0.5 * (double)(p->N - 1);
        fj.centre_det = 0.5 * (double)(p->D - 1);
        fj.margin = L.margin;
        fj.N = p->N;
        fj.K = p->K;
        fj.D = p->D;
        fj.pad = L.pad;
        fj.pitch = L.pitch;
        fj.scale = (float)(2.0 * kPi / (double)p->K);
    } else {
        j.pimg = ps.ptr;
        j.cs = p->d_cs;
        j.wscale = p->d_wscale;
        j.half_pix = 0.5 * (double)(p->N - 1);
        j.centre_det = 0.5 * (double)(p->D - 1);
        j.N = p->N;
        j.K = p->K;
        j.D = p->D;
        j.scale = (float)(kPi / (double)p->K);
        j.T = L.T;
        j.fast3 = L.fast3 ? 1 : 0;
        j.pad = L.pad;
        j.pitch = L.pitch;
    }
    const size_t is = (size_t)p->N * p->N, qs = (size_t)p->K * p->D;
    if (ps.recorded) FBP_TRY_HIP(hipStreamWaitEvent(s, ps.free_ev, 0));
    for (int32_t i0 = 0; i0 < n_slices; i0 += ps.slices) {
        const int n = std::min<int32_t>(ps.slices, n_slices - i0);
        hipError_t e = launch_pad(d_image + (size_t)i0 * is, ps.ptr, p->N, L.pad, L.pitch, n, s);
        if (e == hipSuccess) {
            if (fan) {
                fj.sino = d_sino + (size_t)i0 * qs;
                e = launch_fan_project(fj, n, s);
            } else {
                j.sino = d_sino + (size_t)i0 * qs;
                e = launch_project(j, n, s);
            }
        }
        if (e != hipSuccess) {
            const int frc = e == hipErrorInvalidValue ? FBP_EUNSUPPORTED : hip_status(e, "projector kernel launch");
            // work queued by earlier rounds still reads the copies: later users wait for it
            return i0 > 0 ? fail_after_queued(frc, ps.free_ev, &ps.recorded, s) : frc;
        }
    }
    FBP_TRY_HIP(hipEventRecord(ps.free_ev, s));
    ps.recorded = true;
    return FBP_OK;
}

int fbp_reconstruct_batch(const fbp_job* jobs, int32_t n_jobs, void* d_workspace,
                          size_t workspace_bytes, int32_t precision, void* hip_stream) {
    return reconstruct_batch(jobs, n_jobs, d_workspace, workspace_bytes, precision,
                             (hipStream_t)hip_stream);
}

int fbp_autotune(const fbp_geom* geom, void* hip_stream, int32_t* out_config) {
    return autotune(geom, (hipStream_t)hip_stream, out_config);
}

int fbp_plan_config(const fbp_geom* geom) {
    const int rc = check_geom(geom);
    if (rc != FBP_OK) return rc;
    if (is_fan(geom)) return FBP_EUNSUPPORTED;
    Plan* p = nullptr;
    const int prc = get_plan(geom, &p);
    return prc == FBP_OK ? p->one.cfg : prc;
}

int fbp_plan_stack_config(const fbp_geom* geom) {
    const int rc = check_geom(geom);
    if (rc != FBP_OK) return rc;
    if (is_fan(geom)) return FBP_EUNSUPPORTED;
    Plan* p = nullptr;
    const int prc = get_plan(geom, &p);
    return prc == FBP_OK ? p->stack.cfg : prc;
}

int fbp_backproject_with_config(const fbp_geom* geom, int32_t n_slices, const float* d_filtered,
                                float* d_image, int32_t config, void* hip_stream) {
    int rc = check_geom(geom);
    if (rc == FBP_OK) rc = check_slices(geom, n_slices);
    if (rc != FBP_OK) return rc;
    if (is_fan(geom)) return FBP_EUNSUPPORTED;
    if (config < 0 || config >= kNumTileConfigs) return FBP_EINVAL;
    if (n_slices == 0) return FBP_OK;
    if (!d_filtered || !d_image || !aligned4(d_filtered) || !aligned4(d_image)) return FBP_EINVAL;
    if (overlaps(d_filtered, sino_bytes(geom, n_slices), d_image, image_bytes(geom, n_slices)))
        return FBP_EINVAL;
    Plan* p = nullptr;
    rc = get_plan(geom, &p);
    if (rc != FBP_OK) return rc;
    ShapeParams sp;   // the plan's geometry with the given shape in both roles
    if (!shape_params(config, p->cs, p->angles, p->N, cu_count(p->device), &sp)) return FBP_EUNSUPPORTED;
    return run_backproject(*p, sp, sp, n_slices, d_filtered, d_image, (hipStream_t)hip_stream);
}

size_t fbp_cone_workspace_bytes(const fbp_cone_geom* geom) {
    if (check_cone_geom(geom) != FBP_OK) return 0;
    return round_up(cone_proj_bytes(geom), 256);
}

int fbp_cone_filter(const fbp_cone_geom* geom, const float* d_proj, float* d_filtered, void* hip_stream) {
    int rc = check_cone_geom(geom);
    if (rc != FBP_OK) return rc;
    if (!d_proj || !d_filtered || !aligned4(d_proj) || !aligned4(d_filtered)) return FBP_EINVAL;
    const size_t pb = cone_proj_bytes(geom);
    if (overlaps(d_proj, pb, d_filtered, pb)) return FBP_EINVAL;
    ConePlan* c = nullptr;
    rc = get_cone_plan(geom, &c);
    if (rc != FBP_OK) return rc;
    return run_cone_filter(*c, d_proj, d_filtered, (hipStream_t)hip_stream);
}

int fbp_cone_backproject(const fbp_cone_geom* geom, const float* d_filtered, float* d_volume, void* hip_stream) {
    int rc = check_cone_geom(geom);
    if (rc != FBP_OK) return rc;
    if (!d_filtered || !d_volume || !aligned4(d_filtered) || !aligned4(d_volume)) return FBP_EINVAL;
    if (overlaps(d_filtered, cone_proj_bytes(geom), d_volume, cone_vol_bytes(geom))) return FBP_EINVAL;
    ConePlan* c = nullptr;
    rc = get_cone_plan(geom, &c);
    if (rc != FBP_OK) return rc;
    return run_cone_backproject(*c, d_filtered, d_volume, (hipStream_t)hip_stream);
}

int fbp_cone_reconstruct(const fbp_cone_geom* geom, const float* d_proj, float* d_volume, void* d_workspace,
                         size_t workspace_bytes, void* hip_stream) {
    int rc = check_cone_geom(geom);
    if (rc != FBP_OK) return rc;
    if (!d_proj || !d_volume || !aligned4(d_proj) || !aligned4(d_volume)) return FBP_EINVAL;
    const size_t pb = cone_proj_bytes(geom), vb = cone_vol_bytes(geom);
    if (overlaps(d_proj, pb, d_volume, vb)) return FBP_EINVAL;
    if (!d_workspace || workspace_bytes < pb) return FBP_EWORKSPACE;
    if ((reinterpret_cast<uintptr_t>(d_workspace) & 255u) != 0) return FBP_EINVAL;
    if (overlaps(d_workspace, pb, d_proj, pb) || overlaps(d_workspace, pb, d_volume, vb)) return FBP_EINVAL;
    ConePlan* c = nullptr;
    rc = get_cone_plan(geom, &c);
    if (rc != FBP_OK) return rc;
    float* filt = static_cast<float*>(d_workspace);
    const hipStream_t s = (hipStream_t)hip_stream;
    rc = run_cone_filter(*c, d_proj, filt, s);
    if (rc == FBP_OK) rc = run_cone_backproject(*c, filt, d_volume, s);
    return rc;
}

}  // extern "C"
