// Host-side FP64 precompute shared by single plans (plan.cpp) and batches
// (batch.cpp).  Internal; not part of the public ABI.
#pragma once

#include "fastsum.h"
#include "fastsum_impl.h"

#include <cstdint>
#include <vector>

namespace fastsum {
namespace host {

constexpr double kPi = 3.14159265358979323846264338327950288;
constexpr int64_t kChunkAlign = kSliceLen;       // spread chunks start on fixed-point slices
constexpr int64_t kMaxChunk = (int64_t)1 << 20;   // sources per spreading workgroup, at most
constexpr int64_t kFusedMaxChunks = 16;           // fused spreading: source chunks, at most (rule)

// Exponential-of-semicircle window phi(z) = exp(beta (sqrt(1 - z^2) - 1)),
// |z| <= 1, z = (cell - u) / (W/2).  Tap t of a point with sp = frac(u) - 1/2
// sits at z_t = (t + 1/2 - W/2 - sp) / (W/2).  The weight of tap t is
// replaced by its degree-D interpolant in sp at Chebyshev points; everything
// downstream (phihat, the multipliers) is computed from these polynomials, so
// the deconvolution matches the window the kernels actually apply.
struct WindowPoly {
    int W = 4, D = 4;
    double beta = 0.0;
    std::vector<double> coef;   // W x (D+1), monomial coefficients in sp
    double eval(int t, double sp) const {
        double acc = 0.0;
        for (int i = D; i >= 0; --i) acc = acc * sp + coef[t * (D + 1) + i];
        return acc;
    }
};

struct Resolved {
    fastsum_params p;
    int n = 0;          // grid size
    double tau = 0.0;
};

// c_k, k = 0..K (K = n_ft/2), of the 1-periodic rescaled 1-D kernel.
void fourier_coefficients(int kernel, int d, double scale, double tau, int n_ft,
                          std::vector<double>& c);
// the same for every k in [0, kmax] (kmax need not be tied to a grid)
void fourier_coefficients_upto(int kernel, int d, double scale, double tau, int kmax,
                               std::vector<double>& c);
bool build_window(int W, WindowPoly& win);
void window_transform(const WindowPoly& win, int n, int kmax, std::vector<double>& out);
fastsum_status resolve_params(const fastsum_params* in, Resolved& r);
GridGeom make_geom(int n, int W, double tauR);
WindowArgs pack_window(const WindowPoly& win);
uint16_t f32_to_bf16_host(float f);
// multipliers c'_k / (n phihat_k)^2, derivative multipliers 2 pi i k m_k and
// twiddles exp(-2 pi i k / n), each of length n
void build_tables(int kernel, int d, double scale, double tau, int n_ft, int n,
                  const WindowPoly& win, std::vector<float2>& mult,
                  std::vector<float2>& mult_d, std::vector<float2>& tw);
int spread_chunks(int64_t N, int P);
int64_t spread_chunk_len(int64_t N, int nchunk);
int gather_group(int64_t M, int P, int pstage);
void split_dirs_host(const float* xi, int d, int P, std::vector<uint16_t>& out);
// fused spreading: sources per chunk (a multiple of 16) and the chunk count
// of the plan's rule for grids of nr stored cells
int64_t fused_chunk_len(int64_t N, int nchunk);
int fused_chunks(int64_t N, int P, int64_t slots, int nr);
int fused_dir_range(int64_t M, int P, int64_t slots, int nr, int W);
int64_t round_up(int64_t v, int64_t m);
fastsum_status status_of(hipError_t e);

}  // namespace host
}  // namespace fastsum
