// Distance QMC designs on the GPU (App. H): P unit directions that locally
// maximise sum_{p,q} (|xi_p - xi_q| + |xi_p + xi_q|) (the symmetrised
// distance energy of eq. distance-sym with its sign reversed), by projected
// Adam steps from a given start.  Rows of xi are directions (P x d, FP32).
//
// Gradient of row p:  xi_p sum_q (a_pq + b_pq) + sum_q (b_pq - a_pq) xi_q,
// a_pq = 1/|xi_p - xi_q| (0 for q = p), b_pq = 1/|xi_p + xi_q|, with
// |xi_p -+ xi_q|^2 = 2 -+ 2 <xi_p, xi_q> for unit rows; then its tangent
// part.  In the partial-gradient kernel one thread per row p holds xi_p and
// its accumulator in registers (d <= 64, zero-padded to DMAX) while the rows
// q of one q-chunk stream through LDS in tiles of 64, read as broadcasts;
// a second kernel, one wave per row, sums the chunks in order and takes the
// Adam step.
#include "fastsum.h"
#include "fastsum_impl.h"

#include <algorithm>
#include <cmath>
#include <mutex>

namespace fastsum {

namespace {

constexpr int kQmcBlock = 256;
constexpr int kQmcRows = 64;         // rows p per gradient workgroup (one wave)
constexpr int kQmcTile = 64;         // rows q per LDS tile

// Partial gradient sums of rows p0 .. p0+63 over the rows q of chunk
// blockIdx.y (qlen rows each, a multiple of the tile): part[(chunk P + p)
// (DMAX + 1) + i] = sum_q (b - a) xi_q[i] for i < DMAX, and at i = DMAX
// sum_q (a + b).
template <int DMAX>
__global__ __launch_bounds__(kQmcRows) void qmc_grad_partial_kernel(
    const float* __restrict__ xi, int P, int d, int qlen, float* __restrict__ part) {
    __shared__ float tile[kQmcTile][DMAX];
    const int tid = threadIdx.x;
    const int p = blockIdx.x * kQmcRows + tid;
    const int q_begin = blockIdx.y * qlen, q_end = min(P, q_begin + qlen);
    float xp[DMAX], acc[DMAX];
#pragma unroll
    for (int i = 0; i < DMAX; ++i) {
        xp[i] = (p < P && i < d) ? xi[(int64_t)p * d + i] : 0.f;
        acc[i] = 0.f;
    }
    float s = 0.f;
    for (int q0 = q_begin; q0 < q_end; q0 += kQmcTile) {
        __syncthreads();
        for (int j = tid; j < kQmcTile * DMAX; j += kQmcRows) {
            const int r = j / DMAX, i = j % DMAX;
            tile[r][i] = (q0 + r < q_end && i < d) ? xi[(int64_t)(q0 + r) * d + i] : 0.f;
        }
        __syncthreads();
        const int nq = min(kQmcTile, q_end - q0);
        for (int r = 0; r < nq; ++r) {
            float g = 0.f;
#pragma unroll
            for (int i = 0; i < DMAX; ++i) g = fmaf(xp[i], tile[r][i], g);
            g = fminf(1.f, fmaxf(-1.f, g));
            const float a = (q0 + r == p) ? 0.f : rsqrtf(fmaxf(2.f - 2.f * g, 1e-24f));
            const float b = rsqrtf(fmaxf(2.f + 2.f * g, 1e-24f));
            s += a + b;
            const float c = b - a;
#pragma unroll
            for (int i = 0; i < DMAX; ++i) acc[i] = fmaf(c, tile[r][i], acc[i]);
        }
    }
    if (p >= P) return;
    float* __restrict__ dst = part + ((int64_t)blockIdx.y * P + p) * (DMAX + 1);
#pragma unroll
    for (int i = 0; i < DMAX; ++i) dst[i] = acc[i];
    dst[DMAX] = s;
}

__device__ __forceinline__ float qmc_wave_sum(float v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    return v;
}

// One wave per row p, lane i for coordinate i (d <= 64): the chunk partials
// summed in chunk order give g = tangent part of (s xi_p + acc); then the
// Adam step (moments m, v taken as zero before the first step; bc1, bc2 the
// bias corrections 1 - beta^it) and the renormalisation of the row.
__global__ __launch_bounds__(kQmcBlock) void qmc_step_kernel(
    float* __restrict__ xi, int P, int d, int nchunk, int stride,
    const float* __restrict__ part, float* __restrict__ m, float* __restrict__ v, float step,
    float bc1, float bc2, int first) {
    const int lane = threadIdx.x & 63;
    const int p = blockIdx.x * (kQmcBlock / 64) + (threadIdx.x >> 6);
    if (p >= P) return;                        // whole waves; no barriers below
    constexpr float b1 = 0.9f, b2 = 0.999f, eps = 1e-12f;
    const bool on = lane < d;
    const int64_t k = (int64_t)p * d + lane;
    const float x = on ? xi[k] : 0.f;
    float acc = 0.f, s = 0.f;
    for (int c = 0; c < nchunk; ++c) {
        const float* __restrict__ src = part + ((int64_t)c * P + p) * stride;
        if (on) acc += src[lane];
        s += src[stride - 1];
    }
    float g = fmaf(s, x, acc);
    g -= qmc_wave_sum(g * x) * x;
    float xn = 0.f;
    if (on) {
        const float mi = (first ? 0.f : b1 * m[k]) + (1.f - b1) * g;
        const float vi = (first ? 0.f : b2 * v[k]) + (1.f - b2) * g * g;
        m[k] = mi;
        v[k] = vi;
        xn = x + step * (mi / bc1) / (sqrtf(vi / bc2) + eps);
    }
    const float inv = rsqrtf(qmc_wave_sum(xn * xn));
    if (on) xi[k] = xn * inv;
}

// Randomised design (App. E): row p of xi becomes Q xi_p / |Q xi_p|, Q
// (d x d, row-major) applied as y_i = sum_j Q_ij x_j.  One wave per row,
// lane i for coordinate i; the coordinates of the row reach every lane by
// shuffles, so the row is replaced in place after it has been read whole.
__global__ __launch_bounds__(kQmcBlock) void rotate_rows_kernel(
    const float* __restrict__ q, float* __restrict__ xi, int P, int d) {
    const int lane = threadIdx.x & 63;
    const int p = blockIdx.x * (kQmcBlock / 64) + (threadIdx.x >> 6);
    if (p >= P) return;                        // whole waves; no barriers below
    const bool on = lane < d;
    const int64_t k = (int64_t)p * d + lane;
    const float x = on ? xi[k] : 0.f;
    float y = 0.f;
    for (int j = 0; j < d; ++j) {
        const float xj = __shfl(x, j, 64);
        if (on) y = fmaf(q[(int64_t)lane * d + j], xj, y);
    }
    const float nrm = sqrtf(qmc_wave_sum(y * y));
    if (on) xi[k] = y / nrm;
}

// q-chunks so that the gradient has about 2048 workgroups (at least 8 per
// CU), each chunk a whole number of tiles
int qmc_chunk_len(int P) {
    const int pblocks = (P + kQmcRows - 1) / kQmcRows;
    const int tiles = (P + kQmcTile - 1) / kQmcTile;
    const int want = std::max(1, std::min(tiles, (2048 + pblocks - 1) / pblocks));
    return ((tiles + want - 1) / want) * kQmcTile;
}

template <int DMAX>
int launch_qmc_partial(const float* xi, int P, int d, float* part, hipStream_t st) {
    const int qlen = qmc_chunk_len(P);
    const int nchunk = (P + qlen - 1) / qlen;
    hipLaunchKernelGGL(qmc_grad_partial_kernel<DMAX>,
                       dim3((unsigned)((P + kQmcRows - 1) / kQmcRows), (unsigned)nchunk),
                       dim3(kQmcRows), 0, st, xi, P, d, qlen, part);
    return nchunk;
}

}  // namespace

size_t distance_qmc_part_floats(int P) {
    const int qlen = qmc_chunk_len(P);
    return (size_t)((P + qlen - 1) / qlen) * P * (64 + 1);
}

hipError_t distance_qmc(float* xi, int P, int d, int iters, double lr, float* m, float* v,
                        float* part, hipStream_t st) {
    if (P < 1 || d < 1 || d > 64 || iters < 0) return hipErrorInvalidValue;
    hipError_t e = hipSuccess;
    const dim3 grid((unsigned)((P + kQmcBlock / 64 - 1) / (kQmcBlock / 64)));
    const int dmax = d <= 16 ? 16 : d <= 32 ? 32 : d <= 48 ? 48 : 64;
    double p1 = 1.0, p2 = 1.0;
    for (int it = 1; it <= iters; ++it) {
        int nchunk;
        if (dmax == 16) nchunk = launch_qmc_partial<16>(xi, P, d, part, st);
        else if (dmax == 32) nchunk = launch_qmc_partial<32>(xi, P, d, part, st);
        else if (dmax == 48) nchunk = launch_qmc_partial<48>(xi, P, d, part, st);
        else nchunk = launch_qmc_partial<64>(xi, P, d, part, st);
        p1 *= 0.9;
        p2 *= 0.999;
        const double step = lr * (1.0 - 0.9 * it / iters);
        hipLaunchKernelGGL(qmc_step_kernel, grid, dim3(kQmcBlock), 0, st, xi, P, d, nchunk,
                           dmax + 1, part, m, v, (float)step, (float)(1.0 - p1),
                           (float)(1.0 - p2), it == 1 ? 1 : 0);
        e = hipGetLastError();
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}

hipError_t rotate_directions(const float* q, float* xi, int P, int d, hipStream_t st) {
    if (P < 1 || d < 1 || d > 64) return hipErrorInvalidValue;
    const dim3 grid((unsigned)((P + kQmcBlock / 64 - 1) / (kQmcBlock / 64)));
    hipLaunchKernelGGL(rotate_rows_kernel, grid, dim3(kQmcBlock), 0, st, q, xi, P, d);
    return hipGetLastError();
}

}  // namespace fastsum

// ---------------------------------------------------------------------------
// Allocation-free variant: the Adam moments and the chunk partials live in a
// static device array of fixed size.  Nothing in it needs clearing between
// calls: the first step takes the moments as zero without reading them and
// every step overwrites every partial it reads.
// ---------------------------------------------------------------------------

namespace {

constexpr size_t kQmcScratchFloats = (size_t)5 << 20;    // 20 MiB per device
static __device__ __align__(256) float scratch[kQmcScratchFloats];

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mutex;
float* g_scratch_ptr[kMaxDevices] = {};

// The device address of `scratch` on the current device (looked up once per
// device; the host-side name is not a device address).
hipError_t scratch_on_current_device(float** out) {
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return e;
    if (dev < 0 || dev >= kMaxDevices) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lock(g_scratch_mutex);
    if (g_scratch_ptr[dev] == nullptr) {
        void* ptr = nullptr;
        e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return e;
        if (ptr == nullptr) return hipErrorInvalidSymbol;
        g_scratch_ptr[dev] = static_cast<float*>(ptr);
    }
    *out = g_scratch_ptr[dev];
    return hipSuccess;
}

}  // namespace

extern "C" fastsum_status fastsum_distance_qmc_noalloc(int32_t d, int32_t P, int32_t iters,
                                                       double lr, float* xi, void* stream) {
    if (!xi || d < 1 || d > 64 || P < 1 || iters < 0 || !(lr > 0.0) || !std::isfinite(lr))
        return FASTSUM_EINVAL;
    const size_t n = (size_t)P * d;
    if (2 * n + fastsum::distance_qmc_part_floats(P) > kQmcScratchFloats) return FASTSUM_EINVAL;
    float* base = nullptr;
    if (scratch_on_current_device(&base) != hipSuccess) return FASTSUM_EDEVICE;
    const hipError_t e = fastsum::distance_qmc(xi, P, d, iters, lr, base, base + n, base + 2 * n,
                                               (hipStream_t)stream);
    if (e == hipErrorInvalidValue) return FASTSUM_EINVAL;
    return e == hipSuccess ? FASTSUM_OK : FASTSUM_EDEVICE;
}
