// Host side of libfastsum: FP64 precompute, plan/workspace management and the
// C ABI declared in include/fastsum.h.
#include "fastsum.h"
#include "fastsum_impl.h"

#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <complex>
#include <cstdint>
#include <cstring>
#include <new>
#include <vector>

#include "host_common.h"

using namespace fastsum;
using namespace fastsum::host;

namespace fastsum {
namespace host {

// ---------------------------------------------------------------------------
// FP64 numerics
// ---------------------------------------------------------------------------

// log of the d-dimensional Fourier transform of F(||.||) at radius w
// (Table 'tab:kernels', column 3, transform convention of eq. Fourier).
double matern_nu(int kernel) {
    return kernel == FASTSUM_MATERN32 ? 1.5 : kernel == FASTSUM_MATERN52 ? 2.5 : 3.5;
}

double log_ft_d(int kernel, double w, int d, double scale) {
    if (kernel == FASTSUM_GAUSS) {
        const double s2 = scale * scale;
        return 0.5 * d * std::log(2.0 * kPi * s2) - 2.0 * kPi * kPi * s2 * w * w;
    }
    if (kernel >= FASTSUM_MATERN32) {
        // Gamma(nu + d/2) 2^{d/2} pi^{d/2} beta^d / (Gamma(nu) nu^{d/2})
        //   * (1 + 2 pi^2 beta^2 w^2 / nu)^{-(nu + d/2)}
        const double nu = matern_nu(kernel), hd = 0.5 * d;
        return std::lgamma(nu + hd) + hd * std::log(2.0 * kPi) + d * std::log(scale) -
               std::lgamma(nu) - hd * std::log(nu) -
               (nu + hd) * std::log1p(2.0 * kPi * kPi * scale * scale * w * w / nu);
    }
    const double alpha = 1.0 / scale;   // Laplace
    return std::lgamma(0.5 * (d + 1)) + d * std::log(2.0) + 0.5 * (d - 1) * std::log(kPi) -
           d * std::log(alpha) -
           0.5 * (d + 1) * std::log1p(4.0 * kPi * kPi * w * w / (alpha * alpha));
}

// One-dimensional Fourier transform of t -> f(|t|) through
// F_1[f(|.|)](w) = pi^{d/2}/Gamma(d/2) |w|^{d-1} F_d[F](|w|)  (App. A).
double sliced_ft(int kernel, double w, int d, double scale) {
    w = std::fabs(w);
    const double lf = log_ft_d(kernel, w, d, scale);
    if (d == 1) return std::exp(lf);
    if (w == 0.0) return 0.0;
    return std::exp(0.5 * d * std::log(kPi) - std::lgamma(0.5 * d) + (d - 1) * std::log(w) + lf);
}

double energy_cd(int d) {
    return std::exp(0.5 * std::log(kPi) + std::lgamma(0.5 * (d + 1)) - std::lgamma(0.5 * d));
}

// c_k, k = 0..K, of the 1-periodic rescaled kernel (App. I Step 2; for the
// energy kernel the triangle-wave extension of -(c_d/tau)|x|).
void fourier_coefficients(int kernel, int d, double scale, double tau, int n_ft,
                          std::vector<double>& c) {
    fourier_coefficients_upto(kernel, d, scale, tau, n_ft / 2, c);
}

void fourier_coefficients_upto(int kernel, int d, double scale, double tau, int K,
                               std::vector<double>& c) {
    c.assign(K + 1, 0.0);
    if (kernel == FASTSUM_ENERGY) {
        const double cd = energy_cd(d);
        c[0] = -cd / (4.0 * tau);
        for (int k = 1; k <= K; k += 2) c[k] = cd / (tau * kPi * kPi * double(k) * double(k));
        return;
    }
    for (int k = 0; k <= K; ++k) c[k] = tau * sliced_ft(kernel, tau * k, d, scale);
}

// Gauss-Legendre nodes/weights on [-1, 1] by Newton iteration on P_m.
void gauss_legendre(int m, std::vector<double>& x, std::vector<double>& w) {
    x.resize(m);
    w.resize(m);
    for (int i = 0; i < (m + 1) / 2; ++i) {
        double z = std::cos(kPi * (i + 0.75) / (m + 0.5));
        double dp = 0.0;
        for (int it = 0; it < 100; ++it) {
            double p0 = 1.0, p1 = 0.0;
            for (int j = 1; j <= m; ++j) {
                const double p2 = p1;
                p1 = p0;
                p0 = ((2.0 * j - 1.0) * z * p1 - (j - 1.0) * p2) / j;
            }
            dp = m * (z * p0 - p1) / (z * z - 1.0);
            const double dz = p0 / dp;
            z -= dz;
            if (std::fabs(dz) < 1e-16) break;
        }
        x[i] = -z;
        x[m - 1 - i] = z;
        w[i] = w[m - 1 - i] = 2.0 / ((1.0 - z * z) * dp * dp);
    }
}

// Solve the small dense system V a = b (partial pivoting), in place.
bool solve_dense(std::vector<double>& V, std::vector<double>& b, int n) {
    for (int c = 0; c < n; ++c) {
        int piv = c;
        for (int r = c + 1; r < n; ++r)
            if (std::fabs(V[r * n + c]) > std::fabs(V[piv * n + c])) piv = r;
        if (V[piv * n + c] == 0.0) return false;
        if (piv != c) {
            for (int k = 0; k < n; ++k) std::swap(V[c * n + k], V[piv * n + k]);
            std::swap(b[c], b[piv]);
        }
        for (int r = c + 1; r < n; ++r) {
            const double f = V[r * n + c] / V[c * n + c];
            for (int k = c; k < n; ++k) V[r * n + k] -= f * V[c * n + k];
            b[r] -= f * b[c];
        }
    }
    for (int c = n - 1; c >= 0; --c) {
        double acc = b[c];
        for (int k = c + 1; k < n; ++k) acc -= V[c * n + k] * b[k];
        b[c] = acc / V[c * n + c];
    }
    return true;
}

bool build_window(int W, WindowPoly& win) {
    win.W = W;
    win.D = (W == 4) ? 4 : (W == 6 ? 5 : 7);
    win.beta = 2.6 * W;
    const int nc = win.D + 1;
    win.coef.assign(W * nc, 0.0);
    std::vector<double> nodes(nc);
    for (int i = 0; i < nc; ++i) nodes[i] = 0.5 * std::cos(kPi * (i + 0.5) / nc);
    for (int t = 0; t < W / 2; ++t) {
        std::vector<double> V(nc * nc), b(nc);
        for (int i = 0; i < nc; ++i) {
            const double sp = nodes[i];
            const double z = (t + 0.5 - 0.5 * W - sp) / (0.5 * W);
            b[i] = std::fabs(z) < 1.0 ? std::exp(win.beta * (std::sqrt(1.0 - z * z) - 1.0)) : 0.0;
            double pw = 1.0;
            for (int k = 0; k < nc; ++k) { V[i * nc + k] = pw; pw *= sp; }
        }
        if (!solve_dense(V, b, nc)) return false;
        for (int k = 0; k < nc; ++k) {
            win.coef[t * nc + k] = b[k];
            // mirror tap: weight_{W-1-t}(sp) = weight_t(-sp)
            win.coef[(W - 1 - t) * nc + k] = (k % 2) ? -b[k] : b[k];
        }
    }
    return true;
}

// phihat(k) = integral of the piecewise-polynomial window against
// exp(-2 pi i k x), x in units of the unit period, for k = 0..kmax.
// A point at u and the cells it touches are (t + 1/2 - W/2 - sp)/n apart.
void window_transform(const WindowPoly& win, int n, int kmax, std::vector<double>& out) {
    std::vector<double> gx, gw;
    gauss_legendre(48, gx, gw);
    out.assign(kmax + 1, 0.0);
    for (int k = 0; k <= kmax; ++k) {
        double acc = 0.0;
        for (int t = 0; t < win.W; ++t)
            for (size_t q = 0; q < gx.size(); ++q) {
                const double sp = 0.5 * gx[q];             // sp in [-1/2, 1/2]
                const double dist = (t + 0.5 - 0.5 * win.W - sp) / n;
                acc += 0.5 * gw[q] * win.eval(t, sp) * std::cos(2.0 * kPi * k * dist);
            }
        out[k] = acc / n;
    }
}

// ---------------------------------------------------------------------------
// parameters
// ---------------------------------------------------------------------------

bool is_pow2(int v) { return v > 0 && (v & (v - 1)) == 0; }

fastsum_status resolve_params(const fastsum_params* in, Resolved& r) {
    if (!in) return FASTSUM_EINVAL;
    fastsum_params p = *in;
    if (p.kernel < FASTSUM_GAUSS || p.kernel > FASTSUM_MATERN72) return FASTSUM_EINVAL;
    if (p.d < 1 || p.d > 4096 || p.P < 1 || p.P > 65536) return FASTSUM_EINVAL;
    if (p.n_ft < 16 || p.n_ft > 4096 || (p.n_ft % 2)) return FASTSUM_EINVAL;
    // Laplace keeps a k^-2 spectrum up to N_ft/2, where the width-4 window's
    // aliasing error reaches ~1e-4; width 6 brings it to ~4e-6.
    if (p.window_w == 0) p.window_w = (p.kernel == FASTSUM_LAPLACE) ? 6 : 4;
    if (p.window_w != 4 && p.window_w != 6 && p.window_w != 8) return FASTSUM_EINVAL;
    if (p.oversample == 0) p.oversample = 2;
    if (p.oversample != 2 && p.oversample != 4) return FASTSUM_EINVAL;
    if (p.proj != FASTSUM_PROJ_FP32 && p.proj != FASTSUM_PROJ_BF16) return FASTSUM_EINVAL;
    if (p.flags & ~(FASTSUM_FLAG_GRAD | FASTSUM_FLAG_MATERIALIZE | FASTSUM_FLAG_SORTED))
        return FASTSUM_EINVAL;
    // exact 1-D sums by sorting exist for the energy kernel only
    if ((p.flags & FASTSUM_FLAG_SORTED) && p.kernel != FASTSUM_ENERGY) return FASTSUM_EINVAL;
    // App. I: T = 0.3 (Gauss), 0.1 (Laplace), 0.2 (Matern); 0.45 for the
    // energy kernel's periodic extension
    if (p.T == 0.0)
        p.T = p.kernel == FASTSUM_GAUSS ? 0.3 : p.kernel == FASTSUM_LAPLACE ? 0.1
              : p.kernel == FASTSUM_ENERGY ? 0.45 : 0.2;
    if (p.gmax_factor == 0.0) p.gmax_factor = 5.0;
    if (!(p.R > 0.0) || !std::isfinite(p.R)) return FASTSUM_EINVAL;
    if (p.kernel != FASTSUM_ENERGY && (!(p.scale > 0.0) || !std::isfinite(p.scale)))
        return FASTSUM_EINVAL;
    if (!(p.gmax_factor > 0.0)) return FASTSUM_EINVAL;
    const int n = p.oversample * p.n_ft;
    if (n > 2048 || !is_pow2(n)) return FASTSUM_EINVAL;
    // every tap of a point with |x~| <= T must stay inside one period
    if (!(p.T > 0.0) || p.T > 0.5 - (p.window_w / 2 + 2.0) / n) return FASTSUM_EINVAL;
    r.p = p;
    r.n = n;
    r.tau = (p.kernel == FASTSUM_ENERGY) ? p.T / p.R
                                         : std::min(p.T / p.R, 1.0 / (2.0 * p.gmax_factor * p.scale));
    return FASTSUM_OK;
}

GridGeom make_geom(int n, int W, double tauR) {
    GridGeom g;
    g.n = n;
    const int half = (int)std::ceil(tauR * n) + W / 2 + 1;
    int lo = std::max(0, n / 2 - half);
    lo &= ~3;
    g.lo = lo;
    g.nr = n - 2 * lo;
    return g;
}

WindowArgs pack_window(const WindowPoly& win) {
    WindowArgs a;
    std::memset(&a, 0, sizeof(a));
    const int nc = win.D + 1;
    for (int t = 0; t < win.W / 2; ++t)
        for (int k = 0; k < nc; ++k) {
            if (k % 2 == 0) a.even[t][k / 2] = (float)win.coef[t * nc + k];
            else a.odd[t][k / 2] = (float)win.coef[t * nc + k];
        }
    return a;
}

uint16_t f32_to_bf16_host(float f) {
    uint32_t u;
    std::memcpy(&u, &f, 4);
    if ((u & 0x7f800000u) == 0x7f800000u) return (uint16_t)((u >> 16) | ((u & 0xffffu) ? 0x40u : 0u));
    u += 0x7fffu + ((u >> 16) & 1u);
    return (uint16_t)(u >> 16);
}

void build_tables(int kernel, int d, double scale, double tau, int n_ft, int n,
                  const WindowPoly& win, std::vector<float2>& mult,
                  std::vector<float2>& mult_d, std::vector<float2>& tw) {
    std::vector<double> c;
    fourier_coefficients(kernel, d, scale, tau, n_ft, c);
    std::vector<double> ph;
    window_transform(win, n, n / 2, ph);
    const int K = n_ft / 2;
    mult.assign(n, make_float2(0.f, 0.f));
    mult_d.assign(n, make_float2(0.f, 0.f));
    tw.assign(n, make_float2(0.f, 0.f));
    for (int k = 0; k < n; ++k) {
        const int ks = (k <= n / 2) ? k : k - n;
        const int a = std::abs(ks);
        double m = 0.0;
        if (a <= K) {
            const double cp = (a == K) ? 0.5 * c[a] : c[a];
            const double den = n * ph[a];
            m = cp / (den * den);
        }
        mult[k] = make_float2((float)m, 0.f);
        mult_d[k] = make_float2(0.f, (float)(2.0 * kPi * ks * m));
        tw[k] = make_float2((float)std::cos(2.0 * kPi * k / n), (float)-std::sin(2.0 * kPi * k / n));
    }
}

int spread_chunks(int64_t N, int P) {
    // aim for >= 2048 workgroups, chunks of >= 4096 sources, <= 2^20 sources
    int64_t want = (2048 + P - 1) / P;
    int64_t maxc = std::max<int64_t>(1, (N + 4095) / 4096);
    int64_t c = std::max<int64_t>(1, std::min<int64_t>(want, std::min<int64_t>(maxc, 64)));
    return (int)std::max<int64_t>(c, (N + kMaxChunk - 1) / kMaxChunk);
}

int64_t spread_chunk_len(int64_t N, int nchunk) {
    return round_up((N + nchunk - 1) / nchunk, kChunkAlign);
}

// Fraction of the last round of workgroups that is busy when `blocks`
// workgroups run `slots` at a time (1 = every round full).
static double round_efficiency(int64_t blocks, int64_t slots) {
    const int64_t rounds = (blocks + slots - 1) / slots;
    return (double)blocks / (double)(rounds * slots);
}

int64_t fused_chunk_len(int64_t N, int nchunk) {
    return round_up((N + nchunk - 1) / nchunk, 16);
}

int fused_chunks(int64_t N, int P, int64_t slots, int nr) {
    // Every workgroup spreads one chunk of sources on 16 directions, so the
    // spread takes ceil(groups * nc / slots) rounds of N / nc sources, and
    // the FFT convolution reads nc partial grids of P * nr cells.  The chunk
    // count minimises the sum of the two, with a source costing 9.6 ns per
    // resident workgroup and a partial cell 4 B at 3.2 TB/s (both measured
    // on MI355X at N = 60000, P = 3500, W = 4); fewer chunks among near ties.
    constexpr double kSrc = 9.6e-9, kCell = 4.0 / 3.2e12;
    const int64_t groups = (P + kFuseDirs - 1) / kFuseDirs;
    const int64_t cmin = std::max<int64_t>(1, (N + kMaxChunk - 1) / kMaxChunk);
    const int64_t cmax = std::max(cmin, std::min<int64_t>(kFusedMaxChunks, (N + 255) / 256));
    int64_t best = cmin;
    double best_t = 1e300;
    for (int64_t nc = cmin; nc <= cmax; ++nc) {
        const int64_t len = fused_chunk_len(N, (int)nc);
        const int64_t actual = (N + len - 1) / len;
        const int64_t rounds = (groups * actual + slots - 1) / slots;
        const double t = (double)rounds * (double)len * kSrc + (double)actual * P * nr * kCell;
        if (t < best_t * 0.98) { best_t = t; best = actual; }
    }
    return (int)best;
}

int fused_dir_range(int64_t M, int P, int64_t slots, int nr, int W) {
    // ranges of whole 16-direction groups; at least three rounds of
    // workgroups when P allows, then the fullest rounds (fewest ranges
    // among near ties: each range re-reads the targets)
    const int64_t tiles = (M + fused_gather_tile(nr, W) - 1) / fused_gather_tile(nr, W);
    const int64_t groups = (P + kFuseDirs - 1) / kFuseDirs;
    int64_t best_pr = groups * kFuseDirs;
    double best_eff = -1.0;
    for (int64_t r = 1; r <= groups; ++r) {
        const int64_t pr = round_up((P + r - 1) / r, kFuseDirs);
        const int64_t ranges = (P + pr - 1) / pr;
        if (ranges != r) continue;
        const int64_t blocks = tiles * ranges;
        if (blocks < 3 * slots && r < groups) continue;
        const double eff = round_efficiency(blocks, slots);
        if (eff > best_eff + 0.02) { best_eff = eff; best_pr = pr; }
    }
    return (int)best_pr;
}

int gather_group(int64_t M, int P, int pstage) {
    // aim for about 1024 workgroups; group size a multiple of pstage, <= 128
    const int64_t tiles = (M + kGatherTile - 1) / kGatherTile;
    int64_t groups = std::max<int64_t>(1, (1024 + tiles - 1) / tiles);
    int64_t pg = (P + groups - 1) / groups;
    pg = round_up(std::max<int64_t>(pg, 1), pstage);
    pg = std::min<int64_t>(pg, 128);
    pg = std::max<int64_t>(pg, pstage);
    return (int)pg;
}

int64_t round_up(int64_t v, int64_t m) { return (v + m - 1) / m * m; }

// Split-f16 tiles of the directions (rows p = xi[:, p], d x P row-major on
// the host), layout as the device's split_points_kernel; directions past P
// and coordinates past d are zero.
void split_dirs_host(const float* xi, int d, int P, std::vector<uint16_t>& out) {
    const int KB = split_kblocks(d);
    const int64_t groups = (P + kFuseDirs - 1) / kFuseDirs;
    out.assign((size_t)(groups * KB * 2 * kSplitTileBytes / 2), 0);
    for (int64_t t = 0; t < groups; ++t)
        for (int kb = 0; kb < KB; ++kb)
            for (int lane = 0; lane < 64; ++lane)
                for (int e = 0; e < 8; ++e) {
                    const int64_t p = 16 * t + (lane & 15);
                    const int i = 32 * kb + 8 * (lane >> 4) + e;
                    const float v = (p < P && i < d) ? xi[(size_t)i * P + p] : 0.f;
                    const _Float16 hi = (_Float16)v;
                    const _Float16 lo = (_Float16)(v - (float)hi);
                    const size_t base = (size_t)((t * KB + kb) * 2) * (kSplitTileBytes / 2) + 8 * lane + e;
                    std::memcpy(&out[base], &hi, 2);
                    std::memcpy(&out[base + kSplitTileBytes / 2], &lo, 2);
                }
}

// BF16 tiles of tau xi (A: P x dpad, tau xi_p in row p), same layout with
// one part per k-block; rounded to nearest even.
void bf16_dirs_host(const std::vector<float>& A, int dpad, int d, int P,
                    std::vector<uint16_t>& out) {
    const int KB = split_kblocks(d);
    const int64_t groups = (P + kFuseDirs - 1) / kFuseDirs;
    out.assign((size_t)(groups * KB * kSplitTileBytes / 2), 0);
    for (int64_t t = 0; t < groups; ++t)
        for (int kb = 0; kb < KB; ++kb)
            for (int lane = 0; lane < 64; ++lane)
                for (int e = 0; e < 8; ++e) {
                    const int64_t p = 16 * t + (lane & 15);
                    const int i = 32 * kb + 8 * (lane >> 4) + e;
                    const float v = (p < P && i < d) ? A[(size_t)p * dpad + i] : 0.f;
                    out[(size_t)(t * KB + kb) * (kSplitTileBytes / 2) + 8 * lane + e] = f32_to_bf16_host(v);
                }
}

// Split tiles of xi^T for the back-projection GEMM: rows i (coordinates),
// columns p (directions), same layout as split_dirs_host.
void split_xit_host(const float* xi, int d, int P, std::vector<uint16_t>& out) {
    const int KB = split_kblocks(P);
    const int64_t tiles = (d + 15) / 16;
    out.assign((size_t)(tiles * KB * 2 * kSplitTileBytes / 2), 0);
    for (int64_t t = 0; t < tiles; ++t)
        for (int kb = 0; kb < KB; ++kb)
            for (int lane = 0; lane < 64; ++lane)
                for (int e = 0; e < 8; ++e) {
                    const int64_t i = 16 * t + (lane & 15);
                    const int p = 32 * kb + 8 * (lane >> 4) + e;
                    const float v = (i < d && p < P) ? xi[(size_t)i * P + p] : 0.f;
                    const _Float16 hi = (_Float16)v;
                    const _Float16 lo = (_Float16)(v - (float)hi);
                    const size_t base = (size_t)((t * KB + kb) * 2) * (kSplitTileBytes / 2) + 8 * lane + e;
                    std::memcpy(&out[base], &hi, 2);
                    std::memcpy(&out[base + kSplitTileBytes / 2], &lo, 2);
                }
}

fastsum_status status_of(hipError_t e) {
    if (e == hipSuccess) return FASTSUM_OK;
    if (e == hipErrorOutOfMemory) return FASTSUM_ENOMEM;
    return FASTSUM_EDEVICE;
}

}  // namespace host
}  // namespace fastsum

// ---------------------------------------------------------------------------
// plan object
// ---------------------------------------------------------------------------

struct fastsum_plan_s {
    Resolved r;
    WindowPoly win;
    WindowArgs win_args;
    GridGeom geom;
    int d = 0, P = 0, dpad = 0, dpad64 = 0, W = 4;
    int64_t n_max = 0, m_max = 0, ld_x = 0, ld_y = 0, ldm = 0;
    int nchunk_cap = 1, pstage = 8, ngroup_cap = 1;
    bool fused = false;               // projections inside spread / gather
    bool sorted = false;              // exact energy sums by sorting, no Fourier buffers
    bool have_proj = false;           // last exec stored its projections
    int64_t tune_chunk_len = 0;       // fastsum_set_launch overrides (0: rule)
    int64_t spread_slots = 1, gather_slots = 1;   // resident fused workgroups on the device
    int tune_dir_range = 0;
    float bound = 0.f;
    int device = 0;
    // device buffers
    float* A = nullptr;            // tau * Xi^T, P x dpad
    float* A64 = nullptr;          // the same, zero-padded to round_up(P, 64) x 64 (d <= 64)
    uint16_t* at = nullptr;        // split-f16 tiles of the directions (fused plans)
    uint16_t* xt = nullptr;        // split-f16 tiles of the sources / targets (fused plans)
    uint16_t* yt = nullptr;
    double xi_norm_max = 1.0;      // max_p |xi_p| (range check of the fused path)
    float* ab = nullptr;           // back-projection operands of the fused adjoint
    float* gpart = nullptr;        // its per-range partial sums, kGradMaxRanges x ldg x 16 DC
    int64_t ldg = 0;
    // stored projections by the tile GEMM (BF16, or FP32 with d > 64):
    // direction tiles (BF16 tau xi, or f16 hi / lo of xi) and a point-tile
    // buffer for one point set at a time
    bool tile_gemm = false;
    uint16_t* gdt = nullptr;
    uint16_t* gpt = nullptr;
    float* xproj = nullptr;
    float* yproj = nullptr;
    float* partial = nullptr;
    float* grid = nullptr;
    float* grid_d = nullptr;
    float* grid_w = nullptr;       // grids of the transposed sum (weight and source adjoints)
    float* grid_wd = nullptr;      // its derivative grids (source adjoint)
    float* tout = nullptr;         // output of the transposed sum when grad_w is not wanted
    double* spart = nullptr;
    float* tprime = nullptr;
    float2* mult = nullptr;
    float2* mult_d = nullptr;
    float2* tw = nullptr;
    int* flag = nullptr;
    unsigned* norms = nullptr;     // bound check slots (kNormUints): largest |x / R|^2, |y / R|^2
    bool norms_dirty = false;      // an exec stopped before its check cleared them
    float norm_lim = 1.f;          // (1 + 1e-5) / max_p |xi_p|
    float* slice_max = nullptr;    // per-slice max |w| (fixed-point scaling)
    // sorted plans: rows of stride sort_L, sources at 0, targets at sort_yoff
    float* keys = nullptr;
    float* keys_out = nullptr;
    unsigned int* vals = nullptr;
    void* sort_temp = nullptr;
    size_t sort_temp_bytes = 0;
    float* sv = nullptr;           // per-direction exact sums, P x ldm (bucketed, see sti)
    unsigned short* sti = nullptr; // each staged sum's target offset in its 4096-target bucket
    float* sty = nullptr;          // sorted adjoint: d/dy~ and d/dx~ per direction, P x ldm
    float* stx = nullptr;
    float* styb = nullptr;         // the same, staged by bucket (values, offsets)
    unsigned short* styo = nullptr;
    float* stxb = nullptr;
    unsigned short* stxo = nullptr;
    int64_t sort_L = 0, sort_yoff = 0;
    // back-projection on the tile GEMM (d above the fused range): split
    // tiles of xi^T, the derivative matrix as tiles, abs-max slots
    uint16_t* xit = nullptr;
    uint16_t* bp_tiles = nullptr;
    unsigned* bp_scratch = nullptr;
    // last exec
    bool have_exec = false, last_same = false;
    const float* last_x = nullptr;
    const float* last_w = nullptr;
    const float* last_y = nullptr;
    int64_t last_N = 0, last_M = 0;
    int last_nchunk = 0, last_ngroup = 0;
    hipStream_t last_stream = nullptr;
    // profiling
    struct Rec { int phase; hipEvent_t a, b; };
    bool prof = false;
    std::vector<Rec> recs;
    std::vector<hipEvent_t> pool;
};

namespace {

void free_plan(fastsum_plan_s* p) {
    if (!p) return;
    for (auto& r : p->recs) { (void)hipEventDestroy(r.a); (void)hipEventDestroy(r.b); }
    for (auto e : p->pool) (void)hipEventDestroy(e);
    void* bufs[] = {p->A, p->A64, p->at, p->xt, p->yt, p->gdt, p->gpt, p->xproj, p->yproj, p->partial, p->grid, p->grid_d,
                    p->grid_w, p->spart, p->tprime, p->mult, p->mult_d, p->tw, p->flag,
                    p->slice_max, p->ab, p->gpart, p->grid_wd, p->tout, p->keys,
                    p->keys_out, p->vals, p->sort_temp, p->sv, p->sty, p->stx, p->norms,
                    p->xit, p->bp_tiles, p->bp_scratch,
                    p->sti, p->styb, p->styo, p->stxb, p->stxo};
    for (void* b : bufs)
        if (b) (void)hipFree(b);
    delete p;
}

template <typename T>
bool dev_alloc(T** ptr, size_t count) {
    if (count == 0) count = 1;
    return hipMalloc((void**)ptr, count * sizeof(T)) == hipSuccess;
}

hipEvent_t take_event(fastsum_plan_s* p) {
    if (!p->pool.empty()) {
        hipEvent_t e = p->pool.back();
        p->pool.pop_back();
        return e;
    }
    hipEvent_t e = nullptr;
    if (hipEventCreate(&e) != hipSuccess) return nullptr;
    return e;
}

// Records HIP events around one kernel launch when profiling is enabled.
struct PhaseTimer {
    fastsum_plan_s* p;
    int phase;
    hipStream_t st;
    hipEvent_t a = nullptr;
    PhaseTimer(fastsum_plan_s* pl, int ph, hipStream_t s) : p(pl), phase(ph), st(s) {
        if (p->prof && (a = take_event(p)) != nullptr) (void)hipEventRecord(a, st);
    }
    ~PhaseTimer() {
        if (!a) return;
        hipEvent_t b = take_event(p);
        if (!b) { p->pool.push_back(a); return; }
        (void)hipEventRecord(b, st);
        p->recs.push_back({phase, a, b});
    }
};

fastsum_status check(hipError_t e) { return status_of(e); }

#define FS_TRY(expr)                                  \
    do {                                              \
        fastsum_status _st = check(expr);             \
        if (_st != FASTSUM_OK) return _st;            \
    } while (0)

// Spreading chunks: the plan's rule (rule_chunks) unless fastsum_set_launch
// gave a chunk length; never more chunks than the workspace holds.  Chunks
// of the stored-projection spread start on fixed-point slices (multiples of
// kChunkAlign), those of the fused spread on batches of 16 sources.
int chunk_plan(const fastsum_plan_s* pl, int64_t N, int rule_chunks, bool fused,
               int64_t& chunk_len) {
    auto len_of = [&](int nc) { return fused ? fused_chunk_len(N, nc) : spread_chunk_len(N, nc); };
    chunk_len = pl->tune_chunk_len > 0
                    ? round_up(pl->tune_chunk_len, fused ? 16 : kChunkAlign)
                    : len_of(rule_chunks);
    chunk_len = std::max(chunk_len, len_of(pl->nchunk_cap));
    return (int)((N + chunk_len - 1) / chunk_len);
}

// One 1-D Fourier summation pass for every direction:
// spread (sources) -> fftconv -> gather (targets) into s.
fastsum_status sum_pass(fastsum_plan_s* pl, const float* src_proj, int64_t ld_src,
                        const float* wts, int64_t Nsrc, const float* tgt_proj,
                        int64_t ld_tgt, int64_t Mtgt, float* out, float* grid,
                        float* grid_d, const BoundCheck& bc, hipStream_t st) {
    const int P = pl->P;
    int64_t chunk_len = 0;
    const int nchunk = chunk_plan(pl, Nsrc, spread_chunks(Nsrc, P), false, chunk_len);
    {
        PhaseTimer t(pl, FASTSUM_PHASE_SPREAD, st);
        FS_TRY(launch_spread(pl->W, src_proj, ld_src, wts, Nsrc, P, pl->geom, nchunk, chunk_len,
                             pl->slice_max, pl->win_args, pl->partial, st));
    }
    {
        PhaseTimer t(pl, FASTSUM_PHASE_FFTCONV, st);
        FS_TRY(launch_fftconv(pl->partial, nchunk, P, pl->geom, pl->tw, pl->mult, pl->mult_d,
                              grid, grid_d, st));
    }
    const int pg = gather_group(Mtgt, P, pl->pstage);
    const int ng = (P + pg - 1) / pg;
    pl->last_nchunk = nchunk;
    pl->last_ngroup = ng;
    {
        PhaseTimer t(pl, FASTSUM_PHASE_GATHER, st);
        FS_TRY(launch_gather(pl->W, tgt_proj, ld_tgt, Mtgt, P, pl->geom, grid, pg, pl->pstage,
                             pl->win_args, pl->spart, pl->ldm, nullptr, 0, st));
    }
    PhaseTimer t(pl, FASTSUM_PHASE_REDUCE, st);
    FS_TRY(launch_reduce(pl->spart, ng, pl->ldm, Mtgt, 1.0 / P, out, bc, st));
    return FASTSUM_OK;
}

// Fused path (d <= 64): the points are split into f16 operand tiles
// (scaled by 1/R), then the projections tau R <xi, x / R> are computed inside
// the spreading and gathering kernels.
//   split(x), split(y) -> spread(x, w) -> fftconv -> gather(y) -> reduce
// Spread (sources xt, weights w), FFT convolution (and the derivative grids
// when grid_d is given), gather at the targets yt and reduction into out:
// one sliced Fourier sum on split operand tiles.
fastsum_status fused_sum(fastsum_plan_s* pl, const uint16_t* xt, const float* w, int64_t N,
                         const uint16_t* yt, int64_t M, float* out, float* grid, float* grid_d,
                         const BoundCheck& bc, hipStream_t st) {
    const int P = pl->P;
    const float pscale = (float)(pl->r.tau * pl->r.p.R);
    int64_t chunk_len = 0;
    const int nchunk = chunk_plan(pl, N, fused_chunks(N, P, pl->spread_slots, pl->geom.nr), true,
                                  chunk_len);
    {
        PhaseTimer t(pl, FASTSUM_PHASE_SPREAD, st);
        FS_TRY(launch_spread_fused(pl->W, xt, N, pl->d, pl->at, w, P, pl->geom, pscale, nchunk,
                                   chunk_len, pl->slice_max, pl->win_args, pl->partial, st));
    }
    {
        PhaseTimer t(pl, FASTSUM_PHASE_FFTCONV, st);
        FS_TRY(launch_fftconv(pl->partial, nchunk, P, pl->geom, pl->tw, pl->mult,
                              grid_d ? pl->mult_d : nullptr, grid, grid_d, st));
    }
    const int prange = pl->tune_dir_range > 0 ? pl->tune_dir_range
                                              : fused_dir_range(M, P, pl->gather_slots, pl->geom.nr, pl->W);
    const int nrange = (P + prange - 1) / prange;
    pl->last_nchunk = nchunk;
    pl->last_ngroup = nrange;
    {
        PhaseTimer t(pl, FASTSUM_PHASE_GATHER, st);
        FS_TRY(launch_gather_fused(pl->W, yt, M, pl->d, pl->at, P, pl->geom, pscale, grid,
                                   prange, pl->win_args, pl->spart, pl->ldm, st));
    }
    PhaseTimer t(pl, FASTSUM_PHASE_REDUCE, st);
    FS_TRY(launch_reduce(pl->spart, nrange, pl->ldm, M, 1.0 / P, out, bc, st));
    return FASTSUM_OK;
}

fastsum_status fused_pass(fastsum_plan_s* pl, const float* x, const float* w, int64_t N,
                          const float* y, int64_t M, float* out, const BoundCheck& bc,
                          hipStream_t st) {
    const float inv_r = (float)(1.0 / pl->r.p.R);
    // |x~| <= tau R for every direction when |x| max|xi| <= R (same slack as
    // the stored path's check of each projection)
    const double lim = (1.0 + 1e-5) / pl->xi_norm_max;
    const float norm2_max = (float)(lim * lim);
    const uint16_t* yt = pl->xt;
    {
        PhaseTimer t(pl, FASTSUM_PHASE_PROJECT, st);
        FS_TRY(launch_split_points(x, N, pl->d, inv_r, pl->xt, norm2_max, pl->flag, pl->norms,
                                   st));
        if (y != x) {
            FS_TRY(launch_split_points(y, M, pl->d, inv_r, pl->yt, norm2_max, pl->flag,
                                       pl->norms + kNormRoleUints, st));
            yt = pl->yt;
        }
    }
    return fused_sum(pl, pl->xt, w, N, yt, M, out, pl->grid,
                     (pl->r.p.flags & FASTSUM_FLAG_GRAD) ? pl->grid_d : nullptr, bc, st);
}

// direction ranges of the fused adjoint gather: at least three rounds of
// workgroups when P allows, at most kGradMaxRanges ranges
constexpr int kGradMaxRanges = 4;

int fused_grad_range(int64_t M, int P, int64_t slots) {
    const int64_t tiles = (M + fused_grad_tile() - 1) / fused_grad_tile();
    const int64_t groups = (P + kFuseDirs - 1) / kFuseDirs;
    const int64_t want = std::min<int64_t>(kGradMaxRanges, (3 * slots + tiles - 1) / tiles);
    const int64_t ranges = std::max<int64_t>(1, std::min(groups, want));
    return (int)round_up((P + ranges - 1) / ranges, kFuseDirs);
}

// Stored projections of X into out (row stride ld); norm_slot (nullable)
// receives the rows' largest |x / R|^2 for the bound check.
fastsum_status project(fastsum_plan_s* pl, const float* X, int64_t N, float* out, int64_t ld,
                       unsigned* norm_slot, hipStream_t st) {
    PhaseTimer t(pl, FASTSUM_PHASE_PROJECT, st);
    const float inv_r = (float)(1.0 / pl->r.p.R);
    if (pl->tile_gemm) {
        // BF16: bf16(x) . bf16(tau xi); FP32: (x / R) . xi split into f16
        // hi + lo, times tau R
        const bool bf16 = pl->r.p.proj == FASTSUM_PROJ_BF16;
        return check(launch_project_tiles(X, N, pl->d, bf16, pl->gdt, pl->P, inv_r,
                                          bf16 ? 1.f : (float)(pl->r.tau * pl->r.p.R), pl->gpt,
                                          out, ld, pl->bound, pl->flag, norm_slot, st));
    }
    return check(launch_project_f32(X, N, pl->d, pl->A64, pl->P, out, ld, pl->bound, pl->flag,
                                    norm_slot, inv_r, st));
}

// grad[m * d + i] = coef v[m] sum_p T[p * ld + m] tau xi_p[i]: on the tile
// GEMM above the fused range, else the FP32-MFMA back-projection kernel
fastsum_status backproject(fastsum_plan_s* pl, const float* T, int64_t ld, int64_t M, float coef,
                           const float* v, float* grad, hipStream_t st) {
    if (pl->xit)
        return check(launch_backproject_tiles(T, ld, M, pl->P, pl->d, pl->xit, (float)pl->r.tau,
                                              coef, v, grad, pl->bp_tiles, pl->bp_scratch, st));
    return check(launch_backproject(T, ld, M, pl->P, pl->d, pl->A, pl->dpad, coef, v, grad, st));
}

// Sorted plans (energy kernel): project x and y into the rows of the sort,
// then per direction sort + FP64 prefix sums give
// -(c_d / tau) sum_n w_n |x~_n - y~_m| = sum_n w_n f(<xi_p, x_n - y_m>)
// exactly, and the FP64 mean over the directions finishes s.
fastsum_status sorted_pass(fastsum_plan_s* pl, const float* x, const float* w, int64_t N,
                           const float* y, int64_t M, float* out, bool same,
                           const BoundCheck& bc, hipStream_t st) {
    const int64_t L = pl->sort_L, yoff = pl->sort_yoff;
    fastsum_status r = project(pl, x, N, pl->keys, L, pl->norms, st);
    if (r != FASTSUM_OK) return r;
    if (!same) {
        r = project(pl, y, M, pl->keys + yoff, L, pl->norms + kNormRoleUints, st);
        if (r != FASTSUM_OK) return r;
    }
    const double coef = -energy_cd(pl->d) / pl->r.tau;
    {
        PhaseTimer t(pl, FASTSUM_PHASE_SORT, st);
        FS_TRY(launch_sorted_energy(pl->keys, pl->keys_out, pl->vals, pl->sort_temp,
                                    pl->sort_temp_bytes, L, pl->P, (int)N, (int)yoff, (int)M,
                                    same ? 1 : 0, w, coef, pl->sv, pl->sti, pl->ldm, st));
    }
    pl->last_nchunk = 0;
    pl->last_ngroup = pl->P;
    PhaseTimer t(pl, FASTSUM_PHASE_REDUCE, st);
    FS_TRY(launch_sorted_bucket_reduce(pl->sv, pl->sti, pl->P, pl->ldm, (int)M, pl->spart,
                                       1.0 / pl->P, out, bc, st));
    return FASTSUM_OK;
}

// Adjoint of a sorted exec from the rows that exec sorted (sources x,
// targets y, or one copy of the points when they were both): per
// direction the weight sums over strictly smaller and larger keys give the
// derivatives at every point; back-projection with tau Xi and the weights
// v or w gives grad_y and grad_x, the FP64 mean of the transposed sums
// grad_w.
fastsum_status sorted_grad(fastsum_plan_s* pl, const float* v, float* grad_x, float* grad_y,
                           float* grad_w, hipStream_t st) {
    const int64_t L = pl->sort_L, yoff = pl->sort_yoff, N = pl->last_N, M = pl->last_M;
    const int P = pl->P;
    if (!grad_x && !grad_y && !grad_w) return FASTSUM_OK;
    const double coef = -energy_cd(pl->d) / pl->r.tau;
    {
        PhaseTimer t(pl, FASTSUM_PHASE_SORT, st);
        FS_TRY(launch_sorted_grad(pl->keys, pl->keys_out, pl->vals, L, P, (int)N, (int)yoff,
                                  (int)M, pl->last_same ? 1 : 0, pl->last_w, v, coef, pl->styb,
                                  pl->styo, pl->stxb, pl->stxo, pl->sv, pl->sti, pl->ldm,
                                  (grad_y ? 1 : 0) | (grad_x ? 2 : 0) | (grad_w ? 4 : 0), st));
        if (grad_y) FS_TRY(launch_sorted_place(pl->styb, pl->styo, P, pl->ldm, (int)M, pl->sty, st));
        if (grad_x) FS_TRY(launch_sorted_place(pl->stxb, pl->stxo, P, pl->ldm, (int)N, pl->stx, st));
    }
    const float inv_p = (float)(1.0 / P);
    if (grad_y) {
        PhaseTimer t(pl, FASTSUM_PHASE_BACKPROJECT, st);
        fastsum_status r = backproject(pl, pl->sty, pl->ldm, M, inv_p, v, grad_y, st);
        if (r != FASTSUM_OK) return r;
    }
    if (grad_x) {
        PhaseTimer t(pl, FASTSUM_PHASE_BACKPROJECT, st);
        fastsum_status r = backproject(pl, pl->stx, pl->ldm, N, inv_p, pl->last_w, grad_x, st);
        if (r != FASTSUM_OK) return r;
    }
    if (grad_w) {
        PhaseTimer t(pl, FASTSUM_PHASE_REDUCE, st);
        FS_TRY(launch_sorted_bucket_reduce(pl->sv, pl->sti, P, pl->ldm, (int)N, pl->spart,
                                           1.0 / P, grad_w, BoundCheck{}, st));
    }
    return FASTSUM_OK;
}

}  // namespace

// ---------------------------------------------------------------------------
// C ABI
// ---------------------------------------------------------------------------

extern "C" {

const char* fastsum_status_string(fastsum_status s) {
    switch (s) {
        case FASTSUM_OK: return "ok";
        case FASTSUM_EINVAL: return "invalid argument";
        case FASTSUM_ENOMEM: return "out of memory";
        case FASTSUM_EDEVICE: return "HIP runtime error";
        case FASTSUM_ERANGE: return "point outside the bound R";
        case FASTSUM_EUNSUPPORTED: return "unsupported";
        case FASTSUM_ESTATE: return "invalid call order";
    }
    return "unknown status";
}

fastsum_status fastsum_host_tables(const fastsum_params* prm, double* tau_out, double* ck_out,
                                   double* phihat_out) {
    Resolved r;
    fastsum_status st = resolve_params(prm, r);
    if (st != FASTSUM_OK) return st;
    if (tau_out) *tau_out = r.tau;
    if (ck_out) {
        std::vector<double> c;
        fourier_coefficients(r.p.kernel, r.p.d, r.p.scale, r.tau, r.p.n_ft, c);
        std::copy(c.begin(), c.end(), ck_out);
    }
    if (phihat_out) {
        WindowPoly win;
        if (!build_window(r.p.window_w, win)) return FASTSUM_EINVAL;
        std::vector<double> ph;
        window_transform(win, r.n, r.n / 2, ph);
        std::copy(ph.begin(), ph.end(), phihat_out);
    }
    return FASTSUM_OK;
}

fastsum_status fastsum_plan_create(const fastsum_params* prm, const float* xi, int64_t n_max,
                                   int64_t m_max, void* stream, fastsum_plan* out) {
    if (!prm || !xi || !out || n_max < 1 || m_max < 1) return FASTSUM_EINVAL;
    Resolved r;
    fastsum_status st = resolve_params(prm, r);
    if (st != FASTSUM_OK) return st;
    hipStream_t hs = (hipStream_t)stream;

    fastsum_plan_s* pl = new (std::nothrow) fastsum_plan_s();
    if (!pl) return FASTSUM_ENOMEM;
    pl->r = r;
    pl->d = r.p.d;
    pl->P = r.p.P;
    pl->W = r.p.window_w;
    pl->dpad = (int)round_up(pl->d, 4);
    pl->dpad64 = (int)round_up(pl->d, 64);
    pl->n_max = n_max;
    pl->m_max = m_max;
    if (!build_window(pl->W, pl->win)) { delete pl; return FASTSUM_EINVAL; }
    pl->win_args = pack_window(pl->win);
    const double tauR = r.tau * r.p.R;
    pl->geom = make_geom(r.n, pl->W, tauR);
    pl->bound = (float)(tauR * (1.0 + 1e-5) + 1e-7);
    if (hipGetDevice(&pl->device) != hipSuccess) { delete pl; return FASTSUM_EDEVICE; }

    const int P = pl->P, n = r.n, nr = pl->geom.nr;
    const int64_t cap = std::max(n_max, m_max);
    pl->ld_x = round_up(n_max, 64);
    pl->ld_y = round_up(m_max, 64);
    pl->ldm = round_up(cap, 64);
    pl->pstage = std::max(1, std::min(8, 12288 / nr));
    pl->ngroup_cap = (P + pl->pstage - 1) / pl->pstage;
    // spread_chunks grows with the source count, and the weight adjoint
    // spreads the targets: size for the larger of the two roles
    pl->nchunk_cap = spread_chunks(cap, P);
    const bool grad = (r.p.flags & FASTSUM_FLAG_GRAD) != 0;
    pl->fused = !(r.p.flags & (FASTSUM_FLAG_MATERIALIZE | FASTSUM_FLAG_SORTED)) &&
                r.p.proj == FASTSUM_PROJ_FP32 &&
                fused_supported(pl->d, nr);
    if (pl->fused) {
        int ncu = 0, sb = 1, gb = 1;
        if (hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, pl->device) != hipSuccess || ncu < 1)
            ncu = 1;
        fused_occupancy(pl->W, pl->d, nr, &sb, &gb);
        pl->spread_slots = (int64_t)ncu * sb;
        pl->gather_slots = (int64_t)ncu * gb;
        // the rule never takes more than kFusedMaxChunks (or N / 2^20) chunks
        pl->nchunk_cap = std::max<int>(pl->nchunk_cap, (int)std::max<int64_t>(
                                           kFusedMaxChunks, (cap + kMaxChunk - 1) / kMaxChunk));
    }

    pl->sorted = (r.p.flags & FASTSUM_FLAG_SORTED) != 0;
    if (pl->sorted) {
        pl->sort_yoff = pl->ld_x;
        pl->sort_L = pl->ld_x + pl->ld_y;
        // the bucket counters of the scans live in LDS: at most 2^12 buckets of 4096
        if (pl->sort_L > INT32_MAX / 2 || (int64_t)P * pl->sort_L >= ((int64_t)1 << 32) ||
            pl->ldm > ((int64_t)1 << 24)) {
            delete pl;
            return FASTSUM_EINVAL;
        }
        pl->sort_temp_bytes = sorted_energy_temp_bytes(pl->sort_L, P);
        if (pl->sort_temp_bytes == 0) { delete pl; return FASTSUM_EDEVICE; }
    }

    // fused plans store no projections; they keep split operand tiles.
    // Sorted plans keep the projections in their sort rows and have no grids.
    const int64_t gtiles = (P + kFuseDirs - 1) / kFuseDirs;
    const size_t PL = (size_t)P * pl->sort_L;
    bool ok = pl->sorted
        ? dev_alloc(&pl->A, (size_t)P * pl->dpad) && dev_alloc(&pl->keys, PL) &&
              dev_alloc(&pl->keys_out, PL) && dev_alloc(&pl->vals, PL) &&
              dev_alloc((char**)&pl->sort_temp, pl->sort_temp_bytes) &&
              dev_alloc(&pl->sv, (size_t)P * pl->ldm) && dev_alloc(&pl->sti, (size_t)P * pl->ldm) &&
              dev_alloc(&pl->spart, (size_t)kSortMaxRanges * pl->ldm) &&
              dev_alloc(&pl->flag, 1) && dev_alloc(&pl->norms, kNormUints)
        : dev_alloc(&pl->A, (size_t)P * pl->dpad) && dev_alloc(&pl->norms, kNormUints) &&
              (pl->fused ? dev_alloc(&pl->xt, (size_t)split_tiles_bytes(n_max, pl->d) / 2) &&
                               dev_alloc(&pl->yt, (size_t)split_tiles_bytes(m_max, pl->d) / 2) &&
                               dev_alloc(&pl->at, (size_t)split_tiles_bytes(gtiles * kFuseDirs, pl->d) / 2)
                         : dev_alloc(&pl->xproj, (size_t)P * pl->ld_x) &&
                               dev_alloc(&pl->yproj, (size_t)P * pl->ld_y)) &&
              dev_alloc(&pl->partial, (size_t)pl->nchunk_cap * P * nr) &&
              dev_alloc(&pl->grid, (size_t)P * nr) &&
              dev_alloc(&pl->spart, (size_t)pl->ngroup_cap * pl->ldm) &&
              dev_alloc(&pl->mult, (size_t)n) && dev_alloc(&pl->tw, (size_t)n) &&
              dev_alloc(&pl->flag, 1) && dev_alloc(&pl->slice_max, (size_t)((cap + kSliceLen - 1) / kSliceLen));
    const int64_t p64 = round_up(P, 64);
    if (ok && pl->d <= kA64Cols) ok = dev_alloc(&pl->A64, (size_t)p64 * kA64Cols);
    pl->tile_gemm = !pl->fused && (pl->d > kA64Cols || r.p.proj == FASTSUM_PROJ_BF16);
    if (ok && pl->tile_gemm) {
        const bool bf16 = r.p.proj == FASTSUM_PROJ_BF16;
        ok = dev_alloc(&pl->gdt, project_tiles_bytes(gtiles * kFuseDirs, pl->d, bf16) / 2) &&
             dev_alloc(&pl->gpt, project_tiles_bytes(cap, pl->d, bf16) / 2);
    }
    const int DC = (pl->d + 15) / 16;
    pl->ldg = cap;       // the source adjoint back-projects at the sources
    if (ok && grad && pl->sorted)
        ok = dev_alloc(&pl->sty, (size_t)P * pl->ldm) && dev_alloc(&pl->stx, (size_t)P * pl->ldm) &&
             dev_alloc(&pl->styb, (size_t)P * pl->ldm) && dev_alloc(&pl->styo, (size_t)P * pl->ldm) &&
             dev_alloc(&pl->stxb, (size_t)P * pl->ldm) && dev_alloc(&pl->stxo, (size_t)P * pl->ldm);
    if (ok && grad && !pl->sorted)
        ok = dev_alloc(&pl->grid_d, (size_t)P * nr) && dev_alloc(&pl->grid_w, (size_t)P * nr) &&
             dev_alloc(&pl->grid_wd, (size_t)P * nr) && dev_alloc(&pl->tout, (size_t)cap) &&
             dev_alloc(&pl->mult_d, (size_t)n) &&
             (pl->fused ? dev_alloc(&pl->ab, (size_t)gtiles * 4 * DC * 64) &&
                              dev_alloc(&pl->gpart, (size_t)kGradMaxRanges * pl->ldg * 16 * DC)
                        : dev_alloc(&pl->tprime, (size_t)P * std::max(pl->ld_x, pl->ld_y)));
    if (ok && grad && pl->d > kSplitMaxD) {
        const int64_t rows = pl->sorted ? pl->ldm : std::max(pl->ld_x, pl->ld_y);
        ok = dev_alloc(&pl->xit, backproject_tiles_bytes(pl->d, P) / 2) &&
             dev_alloc(&pl->bp_tiles, backproject_tiles_bytes(rows, P) / 2) &&
             dev_alloc(&pl->bp_scratch, backproject_scratch_bytes() / sizeof(unsigned));
    }
    if (!ok) { free_plan(pl); return FASTSUM_ENOMEM; }
    // the padding between a sorted row's sources and targets is sorted
    // along with zero weight: keep its keys finite (0 * key must be 0 in the
    // prefix sums), once, since no projection writes there
    if (pl->sorted && hipMemset(pl->keys, 0, PL * sizeof(float)) != hipSuccess) {
        free_plan(pl);
        return FASTSUM_EDEVICE;
    }

    // tables
    std::vector<float2> mult, mult_d, tw;
    build_tables(r.p.kernel, pl->d, r.p.scale, r.tau, r.p.n_ft, n, pl->win, mult, mult_d, tw);
    std::vector<float> A((size_t)P * pl->dpad, 0.f);
    for (int p = 0; p < P; ++p)
        for (int i = 0; i < pl->d; ++i) A[(size_t)p * pl->dpad + i] = (float)(r.tau * (double)xi[(size_t)i * P + p]);
    std::vector<float> A64;
    if (pl->A64) {
        A64.assign((size_t)p64 * kA64Cols, 0.f);
        for (int p = 0; p < P; ++p)
            for (int i = 0; i < pl->d; ++i) A64[(size_t)p * kA64Cols + i] = A[(size_t)p * pl->dpad + i];
    }
    std::vector<uint16_t> at, gdt, xit;
    if (pl->xit) split_xit_host(xi, pl->d, P, xit);
    if (pl->at) split_dirs_host(xi, pl->d, P, at);
    if (pl->gdt) {
        if (r.p.proj == FASTSUM_PROJ_BF16) bf16_dirs_host(A, pl->dpad, pl->d, P, gdt);
        else split_dirs_host(xi, pl->d, P, gdt);
    }
    // back-projection operands: group g, MFMA i, chunk q, lane k*16 + m
    std::vector<float> ab;
    if (pl->ab) {
        ab.assign((size_t)gtiles * 4 * DC * 64, 0.f);
        for (int64_t g = 0; g < gtiles; ++g)
            for (int i = 0; i < 4; ++i)
                for (int q = 0; q < DC; ++q)
                    for (int k = 0; k < 4; ++k)
                        for (int m = 0; m < 16; ++m) {
                            const int64_t p = 16 * g + 4 * k + i;
                            const int col = 16 * q + m;
                            if (p < P && col < pl->d)
                                ab[(((size_t)g * 4 + i) * DC + q) * 64 + k * 16 + m] =
                                    A[(size_t)p * pl->dpad + col];
                        }
    }
    pl->xi_norm_max = 0.0;
    for (int p = 0; p < P; ++p) {
        double ss = 0.0;
        for (int i = 0; i < pl->d; ++i) ss += (double)xi[(size_t)i * P + p] * xi[(size_t)i * P + p];
        pl->xi_norm_max = std::max(pl->xi_norm_max, std::sqrt(ss));
    }
    if (!(pl->xi_norm_max > 0.0)) pl->xi_norm_max = 1.0;
    // |x~ - y~| <= tau max|xi| (|x| + |y|) <= tau R when the bound holds
    pl->norm_lim = (float)((1.0 + 1e-5) / pl->xi_norm_max);
    hipError_t e = hipMemcpyAsync(pl->A, A.data(), A.size() * sizeof(float), hipMemcpyHostToDevice, hs);
    if (e == hipSuccess && pl->at)
        e = hipMemcpyAsync(pl->at, at.data(), at.size() * sizeof(uint16_t), hipMemcpyHostToDevice, hs);
    if (e == hipSuccess && pl->ab)
        e = hipMemcpyAsync(pl->ab, ab.data(), ab.size() * sizeof(float), hipMemcpyHostToDevice, hs);
    if (e == hipSuccess && pl->gdt)
        e = hipMemcpyAsync(pl->gdt, gdt.data(), gdt.size() * 2, hipMemcpyHostToDevice, hs);
    if (e == hipSuccess && pl->xit)
        e = hipMemcpyAsync(pl->xit, xit.data(), xit.size() * 2, hipMemcpyHostToDevice, hs);
    if (e == hipSuccess && pl->A64)
        e = hipMemcpyAsync(pl->A64, A64.data(), A64.size() * sizeof(float), hipMemcpyHostToDevice, hs);
    if (e == hipSuccess && pl->mult)
        e = hipMemcpyAsync(pl->mult, mult.data(), n * sizeof(float2), hipMemcpyHostToDevice, hs);
    if (e == hipSuccess && pl->tw)
        e = hipMemcpyAsync(pl->tw, tw.data(), n * sizeof(float2), hipMemcpyHostToDevice, hs);
    if (e == hipSuccess && pl->mult_d)
        e = hipMemcpyAsync(pl->mult_d, mult_d.data(), n * sizeof(float2), hipMemcpyHostToDevice, hs);
    if (e == hipSuccess) e = hipMemsetAsync(pl->flag, 0, sizeof(int), hs);
    if (e == hipSuccess) e = hipMemsetAsync(pl->norms, 0, kNormUints * sizeof(unsigned), hs);
    if (e == hipSuccess) e = hipStreamSynchronize(hs);
    if (e != hipSuccess) { free_plan(pl); return FASTSUM_EDEVICE; }
    *out = pl;
    return FASTSUM_OK;
}

fastsum_status fastsum_bound(const float* x, int64_t N, const float* y, int64_t M, int32_t d,
                             void* stream, double* bound_out) {
    if (!x || !y || !bound_out || N < 1 || M < 1 || d < 1) return FASTSUM_EINVAL;
    hipStream_t st = (hipStream_t)stream;
    unsigned* slots = nullptr;
    if (!dev_alloc(&slots, kNormUints)) return FASTSUM_ENOMEM;
    std::vector<unsigned> h(kNormUints, 0u);
    hipError_t e = hipMemsetAsync(slots, 0, kNormUints * sizeof(unsigned), st);
    if (e == hipSuccess) e = launch_point_norms(x, N, d, 1.f, slots, st);
    if (e == hipSuccess) e = launch_point_norms(y, M, d, 1.f, slots + kNormRoleUints, st);
    if (e == hipSuccess)
        e = hipMemcpyAsync(h.data(), slots, kNormUints * sizeof(unsigned), hipMemcpyDeviceToHost, st);
    if (e == hipSuccess) e = hipStreamSynchronize(st);
    (void)hipFree(slots);
    if (e != hipSuccess) return FASTSUM_EDEVICE;
    // float bits of non-negative values (and +inf / NaN) order as integers
    unsigned u[2] = {0u, 0u};
    for (int r = 0; r < 2; ++r)
        for (int k = 0; k < kNormRoleUints; k += kNormStride) u[r] = std::max(u[r], h[r * kNormRoleUints + k]);
    float n2[2];
    std::memcpy(n2, u, sizeof(n2));
    const double b = std::sqrt((double)n2[0]) + std::sqrt((double)n2[1]);
    *bound_out = b;
    return std::isfinite(b) ? FASTSUM_OK : FASTSUM_ERANGE;
}

void fastsum_destroy(fastsum_plan plan) {
    if (!plan) return;
    (void)hipDeviceSynchronize();
    free_plan(plan);
}

fastsum_status fastsum_exec(fastsum_plan pl, const float* x, int64_t N, const float* w,
                            const float* y, int64_t M, float* s, void* stream) {
    if (!pl || !x || !w || !y || !s) return FASTSUM_EINVAL;
    if (N < 1 || M < 1 || N > pl->n_max || M > pl->m_max) return FASTSUM_EINVAL;
    // y == x: the targets are the first M <= N sources, whose projections
    // (or operand tiles) serve both roles
    const bool same = (x == y);
    if (same && M > N) return FASTSUM_EINVAL;
    const bool prefix = same && M < N;
    hipStream_t st = (hipStream_t)stream;
    // the exec's last kernel checks max |x| + max |y| <= R and clears the
    // norm slots; an exec that stopped early left them set
    if (pl->norms_dirty) FS_TRY(launch_clear_norms(pl->norms, st));
    pl->norms_dirty = true;
    const BoundCheck bc{pl->norms, pl->flag, pl->norm_lim, (same && !prefix) ? 1 : 0};
    // a sorted plan keeps the targets in rows of their own
    const bool shared = same && !(prefix && pl->sorted);
    if (prefix && !pl->sorted)
        FS_TRY(launch_point_norms(y, M, pl->d, (float)(1.0 / pl->r.p.R),
                                  pl->norms + kNormRoleUints, st));
    fastsum_status r = FASTSUM_OK;
    if (pl->sorted) {
        r = sorted_pass(pl, x, w, N, y, M, s, shared, bc, st);
    } else if (pl->fused) {
        r = fused_pass(pl, x, w, N, y, M, s, bc, st);
    } else {
        r = project(pl, x, N, pl->xproj, pl->ld_x, pl->norms, st);
        const float* yp = pl->xproj;
        int64_t ldy = pl->ld_x;
        if (r == FASTSUM_OK && !same) {
            r = project(pl, y, M, pl->yproj, pl->ld_y, pl->norms + kNormRoleUints, st);
            yp = pl->yproj;
            ldy = pl->ld_y;
        }
        if (r == FASTSUM_OK)
            r = sum_pass(pl, pl->xproj, pl->ld_x, w, N, yp, ldy, M, s, pl->grid,
                         (pl->r.p.flags & FASTSUM_FLAG_GRAD) ? pl->grid_d : nullptr, bc, st);
    }
    if (r != FASTSUM_OK) return r;
    pl->norms_dirty = false;
    pl->have_exec = true;
    pl->have_proj = !pl->fused;
    pl->last_same = shared;
    pl->last_x = x;
    pl->last_w = w;
    pl->last_y = y;
    pl->last_N = N;
    pl->last_M = M;
    pl->last_stream = st;
    return FASTSUM_OK;
}

fastsum_status fastsum_grad_xyw(fastsum_plan pl, const float* grad_s, float* grad_x, float* grad_y,
                                float* grad_w, void* stream) {
    if (!pl || !grad_s) return FASTSUM_EINVAL;
    if (!(pl->r.p.flags & FASTSUM_FLAG_GRAD) || !pl->have_exec) return FASTSUM_ESTATE;
    hipStream_t st = (hipStream_t)stream;
    const int P = pl->P;
    const int64_t M = pl->last_M, N = pl->last_N;
    const float coef = (float)(1.0 / P);
    // The transposed sum u(x) = sum_m v_m K(x, y_m) (sources y with weights
    // v = grad_s, targets x) gives grad_w = u(x) and, through its
    // derivative grids, grad_x[n] = w_n du/dx(x_n).
    float* uout = grad_w ? grad_w : pl->tout;
    if (pl->sorted) return sorted_grad(pl, grad_s, grad_x, grad_y, grad_w, st);
    if (pl->fused) {
        const uint16_t* yt = pl->last_same ? pl->xt : pl->yt;
        const float pscale = (float)(pl->r.tau * pl->r.p.R);
        if (grad_y) {
            PhaseTimer t(pl, FASTSUM_PHASE_BACKPROJECT, st);
            FS_TRY(launch_grad_fused(pl->W, yt, M, pl->d, pl->at, pl->ab, P, pl->geom, pscale,
                                     pl->grid_d, fused_grad_range(M, P, pl->gather_slots),
                                     pl->win_args, pl->gpart, pl->ldg, coef, grad_s, grad_y, st));
        }
        if (grad_w || grad_x) {
            fastsum_status r = fused_sum(pl, yt, grad_s, M, pl->xt, N, uout, pl->grid_w,
                                         grad_x ? pl->grid_wd : nullptr, BoundCheck{}, st);
            if (r != FASTSUM_OK) return r;
        }
        if (grad_x) {
            PhaseTimer t(pl, FASTSUM_PHASE_BACKPROJECT, st);
            FS_TRY(launch_grad_fused(pl->W, pl->xt, N, pl->d, pl->at, pl->ab, P, pl->geom, pscale,
                                     pl->grid_wd, fused_grad_range(N, P, pl->gather_slots),
                                     pl->win_args, pl->gpart, pl->ldg, coef, pl->last_w, grad_x,
                                     st));
        }
        return FASTSUM_OK;
    }
    const float* yp = pl->last_same ? pl->xproj : pl->yproj;
    const int64_t ldy = pl->last_same ? pl->ld_x : pl->ld_y;
    if (grad_y) {
        // t'_{m,p}: interpolate the derivative grids of the last exec
        const int pg = gather_group(M, P, pl->pstage);
        {
            PhaseTimer t(pl, FASTSUM_PHASE_GATHER, st);
            FS_TRY(launch_gather(pl->W, yp, ldy, M, P, pl->geom, pl->grid_d, pg, pl->pstage,
                                 pl->win_args, nullptr, 0, pl->tprime, pl->ld_y, st));
        }
        PhaseTimer t(pl, FASTSUM_PHASE_BACKPROJECT, st);
        fastsum_status r = backproject(pl, pl->tprime, pl->ld_y, M, coef, grad_s, grad_y, st);
        if (r != FASTSUM_OK) return r;
    }
    if (grad_w || grad_x) {
        fastsum_status r = sum_pass(pl, yp, ldy, grad_s, M, pl->xproj, pl->ld_x, N, uout,
                                    pl->grid_w, grad_x ? pl->grid_wd : nullptr, BoundCheck{}, st);
        if (r != FASTSUM_OK) return r;
    }
    if (grad_x) {
        const int pg = gather_group(N, P, pl->pstage);
        {
            PhaseTimer t(pl, FASTSUM_PHASE_GATHER, st);
            FS_TRY(launch_gather(pl->W, pl->xproj, pl->ld_x, N, P, pl->geom, pl->grid_wd, pg,
                                 pl->pstage, pl->win_args, nullptr, 0, pl->tprime, pl->ld_x, st));
        }
        PhaseTimer t(pl, FASTSUM_PHASE_BACKPROJECT, st);
        fastsum_status r = backproject(pl, pl->tprime, pl->ld_x, N, coef, pl->last_w, grad_x, st);
        if (r != FASTSUM_OK) return r;
    }
    return FASTSUM_OK;
}

fastsum_status fastsum_grad(fastsum_plan pl, const float* grad_s, float* grad_y, float* grad_w,
                            void* stream) {
    return fastsum_grad_xyw(pl, grad_s, nullptr, grad_y, grad_w, stream);
}

fastsum_status fastsum_check(fastsum_plan pl) {
    if (!pl) return FASTSUM_EINVAL;
    int h = 0;
    hipError_t e = hipStreamSynchronize(pl->last_stream);
    if (e == hipSuccess) e = hipMemcpy(&h, pl->flag, sizeof(int), hipMemcpyDeviceToHost);
    if (e == hipSuccess && h) e = hipMemset(pl->flag, 0, sizeof(int));
    if (e != hipSuccess) return FASTSUM_EDEVICE;
    return h ? FASTSUM_ERANGE : FASTSUM_OK;
}

fastsum_status fastsum_get_info(fastsum_plan pl, fastsum_plan_info* info) {
    if (!pl || !info) return FASTSUM_EINVAL;
    info->tau = pl->r.tau;
    info->beta = pl->win.beta;
    info->n_grid = pl->r.n;
    info->window_w = pl->W;
    info->poly_degree = pl->win.D;
    info->n_ft = pl->r.p.n_ft;
    info->n_max = pl->n_max;
    info->m_max = pl->m_max;
    info->proj = pl->r.p.proj;
    info->flags = pl->r.p.flags;
    info->grid_lo = pl->geom.lo;
    info->grid_nr = pl->geom.nr;
    info->last_spread_chunks = pl->last_nchunk;
    info->last_gather_groups = pl->last_ngroup;
    info->fused = pl->fused ? 1 : 0;
    return FASTSUM_OK;
}

fastsum_status fastsum_debug_read(fastsum_plan pl, int32_t which, float* host_out,
                                  int64_t count) {
    if (!pl || !host_out) return FASTSUM_EINVAL;
    if (!pl->have_exec) return FASTSUM_ESTATE;
    const float* src = nullptr;
    int64_t rows = pl->P, cols = 0, ld = 0;
    if ((which == 0 || which == 1) && !pl->have_proj) return FASTSUM_ESTATE;
    if (pl->sorted && which == 2) return FASTSUM_ESTATE;
    if (pl->sorted && (which == 0 || which == 1)) {
        src = (which == 1 && !pl->last_same) ? pl->keys + pl->sort_yoff : pl->keys;
        cols = which == 0 ? pl->last_N : pl->last_M;
        ld = pl->sort_L;
    } else if (which == 0) { src = pl->xproj; cols = pl->last_N; ld = pl->ld_x; }
    else if (which == 1) {
        src = pl->last_same ? pl->xproj : pl->yproj;
        cols = pl->last_M;
        ld = pl->last_same ? pl->ld_x : pl->ld_y;
    } else if (which == 2) { src = pl->grid; cols = pl->geom.nr; ld = pl->geom.nr; }
    else return FASTSUM_EINVAL;
    if (count != rows * cols) return FASTSUM_EINVAL;
    if (hipStreamSynchronize(pl->last_stream) != hipSuccess) return FASTSUM_EDEVICE;
    if (hipMemcpy2D(host_out, cols * sizeof(float), src, ld * sizeof(float), cols * sizeof(float),
                    rows, hipMemcpyDeviceToHost) != hipSuccess)
        return FASTSUM_EDEVICE;
    return FASTSUM_OK;
}

fastsum_status fastsum_distance_qmc(int32_t d, int32_t P, int32_t iters, double lr, float* xi,
                                    void* stream) {
    if (!xi || d < 1 || d > 64 || P < 1 || iters < 0 || !(lr > 0.0) || !std::isfinite(lr))
        return FASTSUM_EINVAL;
    hipStream_t st = (hipStream_t)stream;
    float *m = nullptr, *v = nullptr, *part = nullptr;
    const size_t n = (size_t)P * d;
    if (!dev_alloc(&m, n) || !dev_alloc(&v, n) || !dev_alloc(&part, distance_qmc_part_floats(P))) {
        for (float* b : {m, v, part})
            if (b) (void)hipFree(b);
        return FASTSUM_ENOMEM;
    }
    hipError_t e = distance_qmc(xi, P, d, iters, lr, m, v, part, st);
    const hipError_t es = hipStreamSynchronize(st);
    for (float* b : {m, v, part}) (void)hipFree(b);
    if (e == hipErrorInvalidValue) return FASTSUM_EINVAL;
    return (e == hipSuccess && es == hipSuccess) ? FASTSUM_OK : FASTSUM_EDEVICE;
}

fastsum_status fastsum_rotate_directions(int32_t d, int32_t P, const float* q, float* xi,
                                         void* stream) {
    if (!q || !xi || d < 1 || d > 64 || P < 1) return FASTSUM_EINVAL;
    hipStream_t st = (hipStream_t)stream;
    if (rotate_directions(q, xi, P, d, st) != hipSuccess) return FASTSUM_EDEVICE;
    return hipStreamSynchronize(st) == hipSuccess ? FASTSUM_OK : FASTSUM_EDEVICE;
}

fastsum_status fastsum_set_launch(fastsum_plan pl, int64_t chunk_len, int32_t dir_range) {
    if (!pl || chunk_len < 0 || chunk_len % 16 != 0 || chunk_len > kMaxChunk ||
        dir_range < 0 || dir_range % kFuseDirs != 0)
        return FASTSUM_EINVAL;
    pl->tune_chunk_len = chunk_len;
    pl->tune_dir_range = dir_range;
    return FASTSUM_OK;
}

fastsum_status fastsum_profile(fastsum_plan pl, int32_t enable) {
    if (!pl) return FASTSUM_EINVAL;
    pl->prof = enable != 0;
    return FASTSUM_OK;
}

fastsum_status fastsum_profile_read(fastsum_plan pl, double* ms_total, int64_t* launches) {
    if (!pl) return FASTSUM_EINVAL;
    if (ms_total) std::fill(ms_total, ms_total + FASTSUM_PHASE_COUNT, 0.0);
    if (launches) std::fill(launches, launches + FASTSUM_PHASE_COUNT, (int64_t)0);
    fastsum_status st = FASTSUM_OK;
    for (auto& r : pl->recs) {
        float ms = 0.f;
        if (hipEventSynchronize(r.b) != hipSuccess || hipEventElapsedTime(&ms, r.a, r.b) != hipSuccess)
            st = FASTSUM_EDEVICE;
        if (ms_total) ms_total[r.phase] += ms;
        if (launches) launches[r.phase] += 1;
        pl->pool.push_back(r.a);
        pl->pool.push_back(r.b);
    }
    pl->recs.clear();
    return st;
}

}  // extern "C"
