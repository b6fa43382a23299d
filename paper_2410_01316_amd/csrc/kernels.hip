// Device kernels of the QMC-slicing fast summation on gfx950 (MI355X).
//
// Data flow of one summation (App. I Steps 1-3 applied per direction, then
// the average over directions of eq. kernel_sum_sliced):
//   project   x~ = tau <xi_p, x_n>  (P x N, direction-major)   MFMA GEMM
//   spread    u_p[j] = sum_n w_n phi(j - u(x~_{n,p}))             LDS int64 atomics
//   fftconv   g_p = IDFT(mult . DFT(u_p))                         LDS FFT
//   gather    s_m = (1/P) sum_p sum_j g_p[j] phi(j - u(y~_{m,p}))  FP64 sum
// mult_k = c'_k / (n phihat_k)^2 folds the Fourier coefficients of the
// rescaled 1-D kernel and the window deconvolution into one table.
//
// Every phase is a tile function.  The single-problem kernels map
// blockIdx to one tile; the batched kernels are persistent and walk a task
// list of tiles drawn from many problems (one launch per phase).
#include "fastsum_impl.h"
#include "device_common.h"

#include <hip/hip_runtime.h>

#include <algorithm>

namespace fastsum {

// ---------------------------------------------------------------------------
// window weights
// ---------------------------------------------------------------------------

template <int W> struct WinShape;
template <> struct WinShape<4> { static constexpr int NE = 3, NO = 2; };  // degree 4
template <> struct WinShape<6> { static constexpr int NE = 3, NO = 3; };  // degree 5
template <> struct WinShape<8> { static constexpr int NE = 4, NO = 4; };  // degree 7

// Per-thread constants of window evaluation on one grid.  The leading
// Horner coefficients live in VGPRs: a VALU instruction reads at most one
// scalar register and the first Horner step would otherwise need two.
template <int W>
struct WinEval {
    float n, half_n;
    int off;                      // W/2 - 1 + lo: first tap of cell 0, relative to lo
    int maxb;                     // nr - W: largest first tap
    float e_lead[W / 2], o_lead[W / 2];
    // pscale: the kernel's projection values are x~ / pscale
    __device__ __forceinline__ WinEval(const GridGeom& g, const WindowArgs& win,
                                       float pscale = 1.f) {
        constexpr int NE = WinShape<W>::NE, NO = WinShape<W>::NO;
        n = (float)g.n * pscale;
        half_n = 0.5f * (float)g.n;
        off = W / 2 - 1 + g.lo;
        maxb = g.nr - W;
#pragma unroll
        for (int t = 0; t < W / 2; ++t) {
            e_lead[t] = win.even[t][NE - 1];
            o_lead[t] = win.odd[t][NO - 1];
            asm volatile("" : "+v"(e_lead[t]));
            asm volatile("" : "+v"(o_lead[t]));
        }
    }
};

// Even and odd parts of the taps of window pair t at offset sp (q = sp^2).
template <int W>
__device__ __forceinline__ void window_pair(float q, int t, const WindowArgs& win,
                                            const WinEval<W>& ev, float& e, float& o) {
    constexpr int NE = WinShape<W>::NE, NO = WinShape<W>::NO;
    e = ev.e_lead[t];
#pragma unroll
    for (int j = NE - 2; j >= 0; --j) e = fmaf(e, q, win.even[t][j]);
    o = ev.o_lead[t];
#pragma unroll
    for (int j = NO - 2; j >= 0; --j) o = fmaf(o, q, win.odd[t][j]);
}

template <int W>
__device__ __forceinline__ void window_weights(float sp, const WindowArgs& win,
                                               const WinEval<W>& ev, float (&wt)[W]) {
    const float q = sp * sp;
#pragma unroll
    for (int t = 0; t < W / 2; ++t) {
        float e, o;
        window_pair<W>(q, t, win, ev, e, o);
        wt[t] = fmaf(o, sp, e);
        wt[W - 1 - t] = fmaf(-o, sp, e);
    }
}

// Position u = x~ n + n/2 of a rescaled projection in grid cells: returns
// the first tap floor(u) - (W/2 - 1) - lo, clamped to [0, nr - W] so that no
// point (outside the bound, infinite or NaN) addresses a cell outside the
// stored range, and sets sp = frac(u) - 1/2.  Points inside the bound are
// never clamped (the stored range has a margin of a cell on each side).
template <int W>
__device__ __forceinline__ int tap0(float xt, const WinEval<W>& ev, float& sp) {
    const float u = fmaf(xt, ev.n, ev.half_n);
    sp = __builtin_amdgcn_fractf(u) - 0.5f;
    int j;
    asm("v_cvt_flr_i32_f32 %0, %1" : "=v"(j) : "v"(u));
    int b;
    asm("v_med3_i32 %0, %1, 0, %2" : "=v"(b) : "v"(j - ev.off), "v"(ev.maxb));
    return b;
}

// ---------------------------------------------------------------------------
// projection: out[p][j] = sum_i A[p][i] X[j][i]   (MFMA, 64 x 128 tiles)
// ---------------------------------------------------------------------------

constexpr int kProjBM = 64;    // directions per workgroup tile
constexpr int kProjBN = 128;   // points per workgroup tile (32 per wave)
constexpr int kProjKC = 32;    // k-chunk staged in LDS (f32)

struct ProjSmemF32 {
    float As[kProjBM][kProjKC + 1];
    float Xs[kProjBN][kProjKC + 1];
};

// The MFMAs compute C^T: acc[bi][bj] holds rows n = wave*32 + bj*16 +
// 4*(lane/16) + r (r = 0..3) of direction column p = bi*16 + lane%16, i.e.
// four consecutive points of one output row: one 16-byte store each.
__device__ __forceinline__ void project_store(const f32x4 (&acc)[4][2], int p0, int64_t n0,
                                              int P, int64_t N, float* __restrict__ out,
                                              int64_t ld, float bound, int* __restrict__ flag) {
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    float mx = 0.f;
#pragma unroll
    for (int bi = 0; bi < 4; ++bi) {
        const int p = p0 + bi * 16 + (lane & 15);
        if (p >= P) continue;
        float* __restrict__ row = out + (int64_t)p * ld;
#pragma unroll
        for (int bj = 0; bj < 2; ++bj) {
            const int64_t n = n0 + wave * 32 + bj * 16 + 4 * (lane >> 4);
            const f32x4 v = acc[bi][bj];
            if (n + 3 < N) {
                *reinterpret_cast<float4*>(row + n) = make_float4(v[0], v[1], v[2], v[3]);
                mx = fmaxf(mx, fmaxf(fmaxf(fabsf(v[0]), fabsf(v[1])), fmaxf(fabsf(v[2]), fabsf(v[3]))));
            } else {
#pragma unroll
                for (int r = 0; r < 4; ++r)
                    if (n + r < N) {
                        row[n + r] = v[r];
                        mx = fmaxf(mx, fabsf(v[r]));
                    }
            }
            // NaN never compares: catch it separately
            if (v[0] != v[0] || v[1] != v[1] || v[2] != v[2] || v[3] != v[3]) mx = INFINITY;
        }
    }
    if (!(mx <= bound)) atomicOr(flag, 1);
}

__device__ __forceinline__ void project_tile_f32(
    ProjSmemF32& sm, const float* __restrict__ X, int64_t N, int d, int dpad,
    const float* __restrict__ A, int P, float* __restrict__ out, int64_t ld, float bound,
    int* __restrict__ flag, int p0, int64_t n0) {
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    f32x4 acc[4][2];
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j) acc[i][j] = f32x4{0.f, 0.f, 0.f, 0.f};

    // software pipeline: chunk k0 + KC is loaded into registers while the
    // MFMAs of chunk k0 run from LDS, so load latency is not exposed
    constexpr int QA = kProjBM * kProjKC / kBlock, QX = kProjBN * kProjKC / kBlock;
    float va[QA], vx[QX];
    auto load = [&](int k0) {
        const int kc = min(kProjKC, d - k0);
#pragma unroll
        for (int q = 0; q < QA; ++q) {
            const int e = tid + q * kBlock, r = e / kProjKC, k = e % kProjKC;
            va[q] = (k < kc && p0 + r < P) ? A[(int64_t)(p0 + r) * dpad + k0 + k] : 0.f;
        }
#pragma unroll
        for (int q = 0; q < QX; ++q) {
            const int e = tid + q * kBlock, r = e / kProjKC, k = e % kProjKC;
            vx[q] = (k < kc && n0 + r < N) ? X[(n0 + r) * d + k0 + k] : 0.f;
        }
    };
    load(0);
    for (int k0 = 0; k0 < d; k0 += kProjKC) {
        const int kc = min(kProjKC, d - k0);
        __syncthreads();                    // the previous chunk's MFMAs are done with LDS
#pragma unroll
        for (int q = 0; q < QA; ++q) {
            const int e = tid + q * kBlock;
            sm.As[e / kProjKC][e % kProjKC] = va[q];
        }
#pragma unroll
        for (int q = 0; q < QX; ++q) {
            const int e = tid + q * kBlock;
            sm.Xs[e / kProjKC][e % kProjKC] = vx[q];
        }
        __syncthreads();
        if (k0 + kProjKC < d) load(k0 + kProjKC);
        for (int ks = 0; ks < kc; ks += 4) {
            float a[4], b[2];
#pragma unroll
            for (int bi = 0; bi < 4; ++bi) a[bi] = sm.As[bi * 16 + (lane & 15)][ks + (lane >> 4)];
#pragma unroll
            for (int bj = 0; bj < 2; ++bj)
                b[bj] = sm.Xs[wave * 32 + bj * 16 + (lane & 15)][ks + (lane >> 4)];
#pragma unroll
            for (int bi = 0; bi < 4; ++bi)
#pragma unroll
                for (int bj = 0; bj < 2; ++bj)
                    acc[bi][bj] = __builtin_amdgcn_mfma_f32_16x16x4f32(b[bj], a[bi], acc[bi][bj], 0, 0, 0);
        }
    }
    project_store(acc, p0, n0, P, N, out, ld, bound, flag);
}

// d <= 64: the block keeps its 128-point X tile in LDS for its whole life
// and walks a range of 64-direction tiles, so X is read from memory once per
// direction range instead of once per direction tile.  A64 is tau * Xi^T
// zero-padded to 64 columns and to a multiple of 64 rows, so the next A tile
// is fetched with unconditional 16-byte loads into registers while the
// current one feeds the MFMAs.  Full tiles store without branches, which
// lets the wait for the prefetched A tile skip the tile's own stores.
constexpr int kXresMaxD = 64;
constexpr int kXresLd = kXresMaxD + 1;
constexpr int kXresQ4 = kProjBM * kXresMaxD / (4 * kBlock);   // float4 per thread and tile

struct ProjSmemXres {
    float Xs[kProjBN][kXresLd];
    float As[kProjBM][kXresLd];
};

__device__ __forceinline__ void xres_load_a(float4 (&va)[kXresQ4], const float* __restrict__ A64,
                                            int p0) {
    const float4* __restrict__ src = reinterpret_cast<const float4*>(A64 + (int64_t)p0 * kXresMaxD);
#pragma unroll
    for (int q = 0; q < kXresQ4; ++q) va[q] = src[threadIdx.x + q * kBlock];
}

__device__ __forceinline__ void project_store_full(const f32x4 (&acc)[4][2], int p0, int64_t n0,
                                                   float* __restrict__ out, int64_t ld,
                                                   float bound, bool& bad) {
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    float* __restrict__ base = out + (int64_t)(p0 + (lane & 15)) * ld + n0 + wave * 32 + 4 * (lane >> 4);
#pragma unroll
    for (int bi = 0; bi < 4; ++bi)
#pragma unroll
        for (int bj = 0; bj < 2; ++bj) {
            const f32x4 v = acc[bi][bj];
            *reinterpret_cast<float4*>(base + (int64_t)bi * 16 * ld + bj * 16) =
                make_float4(v[0], v[1], v[2], v[3]);
#pragma unroll
            for (int r = 0; r < 4; ++r) bad |= !(fabsf(v[r]) <= bound);
        }
}

template <int KS>   // number of k-steps of 4 (fully unrolled)
__device__ __forceinline__ void xres_mfma(const ProjSmemXres& sm, f32x4 (&acc)[4][2]) {
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j) acc[i][j] = f32x4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
    for (int ks = 0; ks < 4 * KS; ks += 4) {
        float a[4], b[2];
#pragma unroll
        for (int bi = 0; bi < 4; ++bi) a[bi] = sm.As[bi * 16 + (lane & 15)][ks + (lane >> 4)];
#pragma unroll
        for (int bj = 0; bj < 2; ++bj)
            b[bj] = sm.Xs[wave * 32 + bj * 16 + (lane & 15)][ks + (lane >> 4)];
#pragma unroll
        for (int bi = 0; bi < 4; ++bi)
#pragma unroll
            for (int bj = 0; bj < 2; ++bj)
                acc[bi][bj] = __builtin_amdgcn_mfma_f32_16x16x4f32(b[bj], a[bi], acc[bi][bj], 0, 0, 0);
    }
}

__device__ __forceinline__ void xres_put_a(ProjSmemXres& sm, const float4 (&va)[kXresQ4]) {
#pragma unroll
    for (int q = 0; q < kXresQ4; ++q) {
        const int e4 = threadIdx.x + q * kBlock, r = e4 >> 4, c = (e4 & 15) * 4;
        sm.As[r][c] = va[q].x;
        sm.As[r][c + 1] = va[q].y;
        sm.As[r][c + 2] = va[q].z;
        sm.As[r][c + 3] = va[q].w;
    }
}

template <int KS>
__device__ __forceinline__ void project_tile_f32_xres(
    ProjSmemXres& sm, const float* __restrict__ X, int64_t N, int d,
    const float* __restrict__ A64, int P, float* __restrict__ out, int64_t ld, float bound,
    int* __restrict__ flag, int p_begin, int p_end, int64_t n0, unsigned* __restrict__ norm_slot,
    float inv_r) {
    const int tid = threadIdx.x;
    float4 va[kXresQ4];
    xres_load_a(va, A64, p_begin);
    __syncthreads();                                // LDS may still be read by a previous tile
    // X tile: rows n0..n0+127 are contiguous in memory (row length d)
    for (int e = tid; e < kProjBN * kXresLd; e += kBlock) {
        const int r = e / kXresLd, k = e % kXresLd;
        sm.Xs[r][k] = (k < d && n0 + r < N) ? X[(n0 + r) * d + k] : 0.f;
    }
    if (norm_slot != nullptr) {                     // uniform: the bound check's row norms
        __syncthreads();
        const int row = tid >> 1;                   // two threads per row (kBlock = 2 kProjBN)
        float ss = 0.f;
        for (int k = tid & 1; k < d; k += 2) {
            const float v = sm.Xs[row][k] * inv_r;
            ss = fmaf(v, v, ss);
        }
        ss += __shfl_xor(ss, 1);
        record_norm2(norm_slot, ss);
    }
    // steady state: whole 64 x 128 tiles, straight-line code so the wait
    // for the prefetched A tile does not include this tile's stores
    const int p_full = (n0 + kProjBN <= N) ? p_begin + ((p_end - p_begin) / kProjBM) * kProjBM
                                           : p_begin;
    const int p_last = p_begin + ((p_end - p_begin - 1) / kProjBM) * kProjBM;
    bool bad = false;
    f32x4 acc[4][2];
    int p0 = p_begin;
    for (; p0 < p_full; p0 += kProjBM) {
        __syncthreads();                            // previous tile's MFMAs are done with As
        xres_put_a(sm, va);
        __syncthreads();
        xres_load_a(va, A64, min(p0 + kProjBM, p_last));   // prefetch (last tile re-read)
        xres_mfma<KS>(sm, acc);
        project_store_full(acc, p0, n0, out, ld, bound, bad);
    }
    // ragged tail: a partial direction tile and/or the last point tile
    for (; p0 < p_end; p0 += kProjBM) {
        __syncthreads();
        xres_put_a(sm, va);
        __syncthreads();
        if (p0 + kProjBM < p_end) xres_load_a(va, A64, p0 + kProjBM);
        xres_mfma<KS>(sm, acc);
        project_store(acc, p0, n0, P, N, out, ld, bound, flag);
    }
    if (bad) atomicOr(flag, 1);
}

// workgroup (x, y): point tile x, direction range y; the first range also
// records the tile's row norms
template <int KS>
__global__ __launch_bounds__(kBlock) void project_f32_xres_kernel(
    const float* __restrict__ X, int64_t N, int d, const float* __restrict__ A64,
    int P, float* __restrict__ out, int64_t ld, float bound, int* __restrict__ flag,
    int prange, unsigned* __restrict__ norm_slot, float inv_r) {
    __shared__ ProjSmemXres sm;
    const int p_begin = blockIdx.y * prange;
    project_tile_f32_xres<KS>(sm, X, N, d, A64, P, out, ld, bound, flag, p_begin,
                              min(P, p_begin + prange), (int64_t)blockIdx.x * kProjBN,
                              blockIdx.y == 0 ? norm_slot : nullptr, inv_r);
}

template <int KS>
void launch_xres(dim3 grid, hipStream_t stream, const float* X, int64_t N, int d,
                 const float* A64, int P, float* out, int64_t ld, float bound, int* flag,
                 int prange, unsigned* norm_slot, float inv_r) {
    hipLaunchKernelGGL(project_f32_xres_kernel<KS>, grid, dim3(kBlock), 0, stream, X, N, d, A64,
                       P, out, ld, bound, flag, prange, norm_slot, inv_r);
}

int project_xres_range(int64_t N, int P) {
    const int64_t ntiles = (N + kProjBN - 1) / kProjBN;
    const int64_t ranges = std::max<int64_t>(1, (2048 + ntiles - 1) / ntiles);
    const int64_t pr = (P + ranges - 1) / ranges;
    return (int)(((pr + kProjBM - 1) / kProjBM) * kProjBM);
}

hipError_t launch_project_f32(const float* X, int64_t N, int d, const float* A64, int P,
                              float* out, int64_t ld, float bound, int* flag,
                              unsigned* norm_slot, float inv_r, hipStream_t stream) {
    if (d > kXresMaxD || A64 == nullptr) return hipErrorInvalidValue;
    const int prange = project_xres_range(N, P);
    dim3 grid((unsigned)((N + kProjBN - 1) / kProjBN), (unsigned)((P + prange - 1) / prange));
    using L = void (*)(dim3, hipStream_t, const float*, int64_t, int, const float*, int,
                       float*, int64_t, float, int*, int, unsigned*, float);
    static const L table[16] = {
        launch_xres<1>, launch_xres<2>, launch_xres<3>, launch_xres<4>,
        launch_xres<5>, launch_xres<6>, launch_xres<7>, launch_xres<8>,
        launch_xres<9>, launch_xres<10>, launch_xres<11>, launch_xres<12>,
        launch_xres<13>, launch_xres<14>, launch_xres<15>, launch_xres<16>};
    table[(d + 3) / 4 - 1](grid, stream, X, N, d, A64, P, out, ld, bound, flag, prange,
                           norm_slot, inv_r);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// spread: one tile = one direction x one chunk of sources
//
// LDS float atomics are slow on this chip, 32-bit integer ones are fast.
// Sources are taken in slices of kSlice = 4096: within a slice every tap
// w * phi is scaled by 2^k (|w| 2^k < 2^18 for the slice's largest |w|),
// rounded to an integer and added with an integer LDS atomic.  A cell of a
// slice then holds at most 4096 terms below 2^18 * 1.01 in magnitude, so its
// sum is exact in 32 bits.  After each slice the cells are moved into FP32
// accumulators in registers (thread t owns cells t + kBlock q, fixed order).
// Grids are bitwise reproducible.
// ---------------------------------------------------------------------------

constexpr int kSlice = 4096;                       // sources per fixed-point slice
constexpr int kSliceSteps = kSlice / (4 * kBlock); // float4 steps per thread and slice
constexpr int kSpreadAcc = 2048 / kBlock;          // cell accumulators per thread (nr <= 2048)

// slice_max[s] = max |w_i| over sources i of slice s
__device__ __forceinline__ void slice_max_tile(float* red, const float* __restrict__ w,
                                               int64_t N, int s, float* __restrict__ slice_max) {
    const int64_t i0 = (int64_t)s * kSlice;
    float v[kSlice / kBlock];
#pragma unroll
    for (int q = 0; q < kSlice / kBlock; ++q) {
        const int64_t i = i0 + threadIdx.x + (int64_t)q * kBlock;
        v[q] = (i < N) ? fabsf(w[i]) : 0.f;
    }
    float m = 0.f;
#pragma unroll
    for (int q = 0; q < kSlice / kBlock; ++q) m = fmaxf(m, v[q]);
    __syncthreads();               // red may still be read by a previous tile
    red[threadIdx.x] = m;
    __syncthreads();
    for (int k = kBlock / 2; k > 0; k >>= 1) {
        if (threadIdx.x < k) red[threadIdx.x] = fmaxf(red[threadIdx.x], red[threadIdx.x + k]);
        __syncthreads();
    }
    if (threadIdx.x == 0) slice_max[s] = red[0];
}

__global__ __launch_bounds__(kBlock) void slice_max_kernel(
    const float* __restrict__ w, int64_t N, float* __restrict__ slice_max) {
    __shared__ float red[kBlock];
    slice_max_tile(red, w, N, blockIdx.x, slice_max);
}

// exponent k with mx * 2^k < 2^18 (0 for an empty, zero or non-finite slice)
__device__ __forceinline__ int slice_exponent(float mx) {
    int e = 0;
    const bool ok = mx > 0.f && mx <= 3.4e38f;
    if (ok) (void)frexpf(mx, &e);   // mx < 2^e
    return ok ? 18 - e : 0;
}

// Adds ws * weight_t, rounded to the nearest integer (ties to even), to the
// W cells of a point.  The rounding must be unbiased: ws * weight_t has only
// a few fraction bits at the top of the fixed-point range, so exact halves
// are common and rounding them up would add a bias that grows with the
// number of sources.
template <int W>
__device__ __forceinline__ void spread_point(float xt, float ws, const WinEval<W>& ev,
                                             const WindowArgs& win, int* lds32) {
    float sp;
    int* __restrict__ c = lds32 + tap0<W>(xt, ev, sp);
    const float q = sp * sp, spw = sp * ws;
#pragma unroll
    for (int t = 0; t < W / 2; ++t) {
        float e, o;
        window_pair<W>(q, t, win, ev, e, o);
        e *= ws;
        atomicAdd(c + t, __float2int_rn(fmaf(o, spw, e)));
        atomicAdd(c + W - 1 - t, __float2int_rn(fmaf(-o, spw, e)));
    }
}

template <int W>
__device__ __forceinline__ void spread_tile(
    void* lds_raw, const float* __restrict__ proj, int64_t ld,
    const float* __restrict__ w, int64_t N, int P, const GridGeom& g, int64_t chunk_len,
    const float* __restrict__ slice_max, const WindowArgs& win, float* __restrict__ partial,
    int p, int c) {
    int* lds32 = reinterpret_cast<int*>(lds_raw);             // nr ints
    const WinEval<W> ev(g, win);
    float acc[kSpreadAcc];
#pragma unroll
    for (int q = 0; q < kSpreadAcc; ++q) acc[q] = 0.f;
    __syncthreads();               // LDS may still be read by a previous tile
    for (int j = threadIdx.x; j < g.nr; j += kBlock) lds32[j] = 0;
    __syncthreads();
    const int64_t i0 = (int64_t)c * chunk_len;          // multiple of kSlice
    const int64_t i1 = min(N, i0 + chunk_len);
    const float* __restrict__ row = proj + (int64_t)p * ld;
    for (int64_t s0 = i0; s0 < i1; s0 += kSlice) {
        const int k = slice_exponent(slice_max[s0 / kSlice]);
        const float scale = ldexpf(1.f, k);
        // issue all loads of the slice first; rows are padded to 64 floats
        float4 xv[kSliceSteps];
        float wv[kSliceSteps][4];
#pragma unroll
        for (int q = 0; q < kSliceSteps; ++q) {
            const int64_t i = s0 + 4 * threadIdx.x + (int64_t)q * 4 * kBlock;
            xv[q] = (i < i1) ? *reinterpret_cast<const float4*>(row + i) : make_float4(0.f, 0.f, 0.f, 0.f);
#pragma unroll
            for (int r = 0; r < 4; ++r) wv[q][r] = (i + r < i1) ? w[i + r] : 0.f;
        }
#pragma unroll
        for (int q = 0; q < kSliceSteps; ++q) {
            spread_point<W>(xv[q].x, wv[q][0] * scale, ev, win, lds32);
            spread_point<W>(xv[q].y, wv[q][1] * scale, ev, win, lds32);
            spread_point<W>(xv[q].z, wv[q][2] * scale, ev, win, lds32);
            spread_point<W>(xv[q].w, wv[q][3] * scale, ev, win, lds32);
        }
        __syncthreads();
        const float unscale = ldexpf(1.f, -k);
#pragma unroll
        for (int q = 0; q < kSpreadAcc; ++q) {
            const int j = threadIdx.x + q * kBlock;
            if (j < g.nr) {
                acc[q] = fmaf((float)lds32[j], unscale, acc[q]);
                lds32[j] = 0;
            }
        }
        __syncthreads();
    }
    float* __restrict__ dst = partial + ((int64_t)c * P + p) * g.nr;
#pragma unroll
    for (int q = 0; q < kSpreadAcc; ++q) {
        const int j = threadIdx.x + q * kBlock;
        if (j < g.nr) dst[j] = acc[q];
    }
}

template <int W>
__global__ __launch_bounds__(kBlock) void spread_kernel(
    const float* __restrict__ proj, int64_t ld, const float* __restrict__ w,
    int64_t N, int P, GridGeom g, int64_t chunk_len, const float* __restrict__ slice_max,
    WindowArgs win, float* __restrict__ partial) {
    extern __shared__ int lds_spread[];
    spread_tile<W>(lds_spread, proj, ld, w, N, P, g, chunk_len, slice_max, win, partial,
                   blockIdx.x, blockIdx.y);
}

hipError_t launch_spread(int W, const float* proj, int64_t ld, const float* w,
                         int64_t N, int P, GridGeom g, int nchunk,
                         int64_t chunk_len, float* slice_max, const WindowArgs& win,
                         float* partial, hipStream_t stream) {
    hipLaunchKernelGGL(slice_max_kernel, dim3((unsigned)((N + kSlice - 1) / kSlice)), dim3(kBlock),
                       0, stream, w, N, slice_max);
    dim3 grid((unsigned)P, (unsigned)nchunk);
    const size_t lds = stored_spread_lds(g.nr);
    switch (W) {
        case 4: hipLaunchKernelGGL(spread_kernel<4>, grid, dim3(kBlock), lds, stream, proj, ld, w, N, P, g, chunk_len, slice_max, win, partial); break;
        case 6: hipLaunchKernelGGL(spread_kernel<6>, grid, dim3(kBlock), lds, stream, proj, ld, w, N, P, g, chunk_len, slice_max, win, partial); break;
        case 8: hipLaunchKernelGGL(spread_kernel<8>, grid, dim3(kBlock), lds, stream, proj, ld, w, N, P, g, chunk_len, slice_max, win, partial); break;
        default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// FFT convolution: two real grids packed as one complex sequence
// ---------------------------------------------------------------------------

__device__ __forceinline__ float2 cmul(float2 a, float2 b) {
    return make_float2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}
__device__ __forceinline__ float2 cadd(float2 a, float2 b) { return make_float2(a.x + b.x, a.y + b.y); }
__device__ __forceinline__ float2 csub(float2 a, float2 b) { return make_float2(a.x - b.x, a.y - b.y); }

// Mixed-radix Stockham autosort FFT of length n (a power of two, 32..2048) in
// LDS: radix-8 passes while n / L >= 8, then one radix-4 or radix-2 pass
// (n = 2048: 8, 8, 8, 4).  Each thread keeps its R values in registers
// through the twiddle and the butterfly.  tw[m] = exp(-2 pi i m / n) is the
// LDS copy of the table; sgn = +1 forward, -1 inverse (exp(+2 pi i ...), no
// 1/n: the multiplier table carries the normalisation).

__device__ __forceinline__ void dft4(float2 (&c)[4], float sgn) {
    const float2 t0 = cadd(c[0], c[2]), t1 = csub(c[0], c[2]), t2 = cadd(c[1], c[3]);
    const float2 d13 = csub(c[1], c[3]);
    const float2 t3 = make_float2(sgn * d13.y, -sgn * d13.x);     // d13 * (-i sgn)
    c[0] = cadd(t0, t2);
    c[1] = cadd(t1, t3);
    c[2] = csub(t0, t2);
    c[3] = csub(t1, t3);
}

__device__ __forceinline__ void dft8(float2 (&a)[8], float sgn) {
    constexpr float s2 = 0.70710678118654752f;
    float2 u[4], v[4];
#pragma unroll
    for (int j = 0; j < 4; ++j) {
        u[j] = cadd(a[j], a[j + 4]);
        v[j] = csub(a[j], a[j + 4]);
    }
    // v_j * exp(-2 pi i j sgn / 8)
    v[1] = make_float2(s2 * (v[1].x + sgn * v[1].y), s2 * (v[1].y - sgn * v[1].x));
    v[2] = make_float2(sgn * v[2].y, -sgn * v[2].x);
    v[3] = make_float2(s2 * (-v[3].x + sgn * v[3].y), s2 * (-v[3].y - sgn * v[3].x));
    dft4(u, sgn);
    dft4(v, sgn);
#pragma unroll
    for (int m = 0; m < 4; ++m) {
        a[2 * m] = u[m];
        a[2 * m + 1] = v[m];
    }
}

template <int R>
__device__ __forceinline__ void fft_pass(const float2* a, float2* b, int n, int L,
                                         const float2* tw, float sgn) {
    const int nb = n / R;
    const int tstep = n / (R * L);
    for (int t = threadIdx.x; t < nb; t += kBlock) {
        const int k = t & (L - 1);
        float2 v[R];
#pragma unroll
        for (int j = 0; j < R; ++j) v[j] = a[t + j * nb];
        if (k) {
#pragma unroll
            for (int j = 1; j < R; ++j) {
                float2 w = tw[j * k * tstep];
                w.y *= sgn;
                v[j] = cmul(v[j], w);
            }
        }
        if constexpr (R == 8) {
            dft8(v, sgn);
        } else if constexpr (R == 4) {
            dft4(v, sgn);
        } else {
            const float2 s = cadd(v[0], v[1]);
            v[1] = csub(v[0], v[1]);
            v[0] = s;
        }
        const int base = (t - k) * R + k;
#pragma unroll
        for (int q = 0; q < R; ++q) b[base + q * L] = v[q];
    }
}

// returns the buffer (a or b) that holds the transform
__device__ float2* fft_lds(float2* a, float2* b, int n, const float2* tw, bool inverse) {
    const float sgn = inverse ? -1.f : 1.f;
    for (int L = 1; L < n;) {
        const int rest = n / L;
        int R;
        if (rest >= 8) {
            fft_pass<8>(a, b, n, L, tw, sgn);
            R = 8;
        } else if (rest == 4) {
            fft_pass<4>(a, b, n, L, tw, sgn);
            R = 4;
        } else {
            fft_pass<2>(a, b, n, L, tw, sgn);
            R = 2;
        }
        __syncthreads();
        float2* t = a;
        a = b;
        b = t;
        L *= R;
    }
    return a;
}

// LDS of one fftconv tile: the twiddle table and two (three with the
// derivative grids) buffers of n complex values
size_t fftconv_lds_bytes(int n, bool grad) { return (size_t)(grad ? 4 : 3) * n * sizeof(float2); }

__device__ __forceinline__ void fftconv_tile(
    float2* cbuf, const float* __restrict__ partial, int nchunk, int P, const GridGeom& g,
    const float2* __restrict__ tw, const float2* __restrict__ mult,
    const float2* __restrict__ mult_d, float* __restrict__ grid, float* __restrict__ grid_d,
    int pair) {
    constexpr int kPer = 2048 / kBlock;   // table entries per thread (n <= 2048)
    constexpr int kInFlight = 8;          // chunk partials per direction loaded at once
    const int n = g.n;
    const int tid = threadIdx.x;
    float2* twl = cbuf;
    float2* b0 = cbuf + n;
    float2* b1 = cbuf + 2 * n;
    float2* b2 = cbuf + 3 * n;            // only with derivative grids
    const int pa = 2 * pair, pb = pa + 1;
    const bool has_b = pb < P;
    // the twiddles and multipliers (tables shared by every pair) are loaded
    // into registers first, so their latency overlaps the partials'
    float2 twv[kPer], mv[kPer], mdv[kPer];
#pragma unroll
    for (int q = 0; q < kPer; ++q) {
        const int j = tid + q * kBlock;
        if (j < n) {
            twv[q] = tw[j];
            mv[q] = mult[j];
            if (grid_d != nullptr) mdv[q] = mult_d[j];
        }
    }
    __syncthreads();               // LDS may still be read by a previous tile
    // inside [lo, lo + nr): the sum of the chunk partials of both directions
    // (in chunk order), read as float4 (nr is a multiple of 4) with up to
    // kInFlight chunks of both directions in flight
    const float4* __restrict__ pa4 = reinterpret_cast<const float4*>(partial + (int64_t)pa * g.nr);
    const float4* __restrict__ pb4 = reinterpret_cast<const float4*>(partial + (int64_t)(has_b ? pb : pa) * g.nr);
    const int64_t cstride4 = (int64_t)P * g.nr / 4;
    for (int r4 = tid; r4 < g.nr / 4; r4 += kBlock) {
        float4 sa = make_float4(0.f, 0.f, 0.f, 0.f), sb = sa;
        for (int c0 = 0; c0 < nchunk; c0 += kInFlight) {
            float4 va[kInFlight], vb[kInFlight];
#pragma unroll
            for (int q = 0; q < kInFlight; ++q) {
                if (c0 + q < nchunk) {
                    va[q] = pa4[(c0 + q) * cstride4 + r4];
                    vb[q] = pb4[(c0 + q) * cstride4 + r4];
                }
            }
#pragma unroll
            for (int q = 0; q < kInFlight; ++q) {
                if (c0 + q < nchunk) {
                    sa.x += va[q].x; sa.y += va[q].y; sa.z += va[q].z; sa.w += va[q].w;
                    sb.x += vb[q].x; sb.y += vb[q].y; sb.z += vb[q].z; sb.w += vb[q].w;
                }
            }
        }
        if (!has_b) sb = make_float4(0.f, 0.f, 0.f, 0.f);
        const int j0 = g.lo + 4 * r4;
        b0[j0] = make_float2(sa.x, sb.x);
        b0[j0 + 1] = make_float2(sa.y, sb.y);
        b0[j0 + 2] = make_float2(sa.z, sb.z);
        b0[j0 + 3] = make_float2(sa.w, sb.w);
    }
    // cells outside [lo, lo + nr) are zero
#pragma unroll
    for (int q = 0; q < kPer; ++q) {
        const int j = tid + q * kBlock;
        if (j < n) {
            twl[j] = twv[q];
            if (j < g.lo || j >= g.lo + g.nr) b0[j] = make_float2(0.f, 0.f);
        }
    }
    __syncthreads();
    float2* spec = fft_lds(b0, b1, n, twl, false);
    float2* other = (spec == b0) ? b1 : b0;
    const int passes = grid_d ? 2 : 1;
    for (int pass = 0; pass < passes; ++pass) {
        float* __restrict__ out = pass ? grid_d : grid;
        // with one pass the spectrum is multiplied in place; with two it is
        // kept for the second multiplier
        float2* wa = (passes == 1) ? spec : (pass == 0 ? other : spec);
        float2* wb = (passes == 1) ? other : b2;
#pragma unroll
        for (int q = 0; q < kPer; ++q) {
            const int j = tid + q * kBlock;
            if (j < n) wa[j] = cmul(spec[j], pass ? mdv[q] : mv[q]);
        }
        __syncthreads();
        const float2* res = fft_lds(wa, wb, n, twl, true);
        for (int r = tid; r < g.nr; r += kBlock) {
            const float2 v = res[g.lo + r];
            out[(int64_t)pa * g.nr + r] = v.x;
            if (has_b) out[(int64_t)pb * g.nr + r] = v.y;
        }
        __syncthreads();
    }
}

__global__ __launch_bounds__(kBlock) void fftconv_kernel(
    const float* __restrict__ partial, int nchunk, int P, GridGeom g,
    const float2* __restrict__ tw, const float2* __restrict__ mult,
    const float2* __restrict__ mult_d, float* __restrict__ grid,
    float* __restrict__ grid_d) {
    extern __shared__ float2 cbuf[];
    fftconv_tile(cbuf, partial, nchunk, P, g, tw, mult, mult_d, grid, grid_d, blockIdx.x);
}

hipError_t launch_fftconv(const float* partial, int nchunk, int P, GridGeom g,
                          const float2* tw, const float2* mult,
                          const float2* mult_d, float* grid, float* grid_d,
                          hipStream_t stream) {
    dim3 grid_dim((unsigned)((P + 1) / 2));
    const size_t lds = fftconv_lds_bytes(g.n, grid_d != nullptr);
    hipLaunchKernelGGL(fftconv_kernel, grid_dim, dim3(kBlock), lds, stream, partial,
                       nchunk, P, g, tw, mult, mult_d, grid, grid_d);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// gather: one tile = 1024 targets x a group of directions
// ---------------------------------------------------------------------------

constexpr int kGatherTPT = 4;   // consecutive targets per thread (one float4)

template <int W>
__device__ __forceinline__ float interp(float xt, const float* gl, const WinEval<W>& ev,
                                        const WindowArgs& win) {
    float sp;
    const float* __restrict__ c = gl + tap0<W>(xt, ev, sp);
    float wt[W];
    window_weights<W>(sp, win, ev, wt);
    float t = 0.f;
#pragma unroll
    for (int k = 0; k < W; ++k) t = fmaf(c[k], wt[k], t);
    return t;
}

template <int W, bool WRITE_T>
__device__ __forceinline__ void gather_tile(
    float* lds, const float* __restrict__ proj, int64_t ld, int64_t M, int P,
    const GridGeom& g, const float* __restrict__ grid, int pg, int pstage,
    const WindowArgs& win, double* __restrict__ spart, int64_t ldm, float* __restrict__ tout,
    int64_t ld_t, int mtile, int group) {
    const int tid = threadIdx.x;
    const int64_t m = (int64_t)mtile * (kBlock * kGatherTPT) + kGatherTPT * tid;
    const bool active = m < M;
    const int p_begin = group * pg;
    const int p_end = min(P, p_begin + pg);
    const WinEval<W> ev(g, win);
    double a0 = 0.0, a1 = 0.0, a2 = 0.0, a3 = 0.0;
    for (int ps = p_begin; ps < p_end; ps += pstage) {
        const int np = min(pstage, p_end - ps);
        __syncthreads();
        {   // stage np grids (np * nr floats, nr a multiple of 4)
            const float4* __restrict__ src4 = reinterpret_cast<const float4*>(grid + (int64_t)ps * g.nr);
            float4* dst4 = reinterpret_cast<float4*>(lds);
            const int n4 = np * g.nr / 4;
            int j = tid;
            for (; j + 3 * kBlock < n4; j += 4 * kBlock) {
                const float4 v0 = src4[j], v1 = src4[j + kBlock], v2 = src4[j + 2 * kBlock],
                             v3 = src4[j + 3 * kBlock];
                dst4[j] = v0;
                dst4[j + kBlock] = v1;
                dst4[j + 2 * kBlock] = v2;
                dst4[j + 3 * kBlock] = v3;
            }
            for (; j < n4; j += kBlock) dst4[j] = src4[j];
        }
        __syncthreads();
        if (active) {
            // rows are padded to a multiple of 64 floats: the float4 at m is in bounds
            const float* __restrict__ rowp = proj + (int64_t)ps * ld + m;
            float4 cur = *reinterpret_cast<const float4*>(rowp);
            for (int pp = 0; pp < np; ++pp) {
                float4 nxt = cur;
                if (pp + 1 < np) nxt = *reinterpret_cast<const float4*>(rowp + (int64_t)(pp + 1) * ld);
                const float* gl = lds + pp * g.nr;
                const float t0 = interp<W>(cur.x, gl, ev, win);
                const float t1 = interp<W>(cur.y, gl, ev, win);
                const float t2 = interp<W>(cur.z, gl, ev, win);
                const float t3 = interp<W>(cur.w, gl, ev, win);
                if (WRITE_T) {
                    *reinterpret_cast<float4*>(tout + (int64_t)(ps + pp) * ld_t + m) =
                        make_float4(t0, t1, t2, t3);
                } else {
                    a0 += (double)t0;
                    a1 += (double)t1;
                    a2 += (double)t2;
                    a3 += (double)t3;
                }
                cur = nxt;
            }
        }
    }
    if (!WRITE_T && active) {
        double* __restrict__ dst = spart + (int64_t)group * ldm + m;
        dst[0] = a0;
        if (m + 1 < M) dst[1] = a1;
        if (m + 2 < M) dst[2] = a2;
        if (m + 3 < M) dst[3] = a3;
    }
}

template <int W, bool WRITE_T>
__global__ __launch_bounds__(kBlock) void gather_kernel(
    const float* __restrict__ proj, int64_t ld, int64_t M, int P, GridGeom g,
    const float* __restrict__ grid, int pg, int pstage, WindowArgs win,
    double* __restrict__ spart, int64_t ldm, float* __restrict__ tout,
    int64_t ld_t) {
    extern __shared__ float lds[];
    gather_tile<W, WRITE_T>(lds, proj, ld, M, P, g, grid, pg, pstage, win, spart, ldm, tout,
                            ld_t, blockIdx.x, blockIdx.y);
}

hipError_t launch_gather(int W, const float* proj, int64_t ld, int64_t M,
                         int P, GridGeom g, const float* grid, int pg,
                         int pstage, const WindowArgs& win, double* spart,
                         int64_t ldm, float* tout, int64_t ld_t,
                         hipStream_t stream) {
    dim3 grid_dim((unsigned)((M + kBlock * kGatherTPT - 1) / (kBlock * kGatherTPT)),
                  (unsigned)((P + pg - 1) / pg));
    const size_t lds = (size_t)pstage * g.nr * sizeof(float);
#define FS_GATHER(WW, WT)                                                                     \
    hipLaunchKernelGGL((gather_kernel<WW, WT>), grid_dim, dim3(kBlock), lds, stream, proj, ld, \
                       M, P, g, grid, pg, pstage, win, spart, ldm, tout, ld_t)
    const bool wt = tout != nullptr;
    switch (W) {
        case 4: if (wt) FS_GATHER(4, true); else FS_GATHER(4, false); break;
        case 6: if (wt) FS_GATHER(6, true); else FS_GATHER(6, false); break;
        case 8: if (wt) FS_GATHER(8, true); else FS_GATHER(8, false); break;
        default: return hipErrorInvalidValue;
    }
#undef FS_GATHER
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// reduction over direction groups (FP64) and back-projection
// ---------------------------------------------------------------------------

__device__ __forceinline__ void reduce_tile(const double* __restrict__ spart, int nb,
                                            int64_t ldm, int64_t M, double scale,
                                            float* __restrict__ s, int64_t m) {
    if (m >= M) return;
    double acc = 0.0;
    for (int b = 0; b < nb; ++b) acc += spart[(int64_t)b * ldm + m];
    s[m] = (float)(acc * scale);
}

__global__ __launch_bounds__(kBlock) void reduce_kernel(
    const double* __restrict__ spart, int nb, int64_t ldm, int64_t M,
    double scale, float* __restrict__ s, BoundCheck bc) {
    reduce_tile(spart, nb, ldm, M, scale, s, (int64_t)blockIdx.x * kBlock + threadIdx.x);
    if (blockIdx.x == 0 && threadIdx.x < 64) finish_bound_check(bc);
}

hipError_t launch_reduce(const double* spart, int nb, int64_t ldm, int64_t M,
                         double scale, float* s, const BoundCheck& bc, hipStream_t stream) {
    dim3 grid((unsigned)((M + kBlock - 1) / kBlock));
    hipLaunchKernelGGL(reduce_kernel, grid, dim3(kBlock), 0, stream, spart, nb, ldm, M, scale, s,
                       bc);
    return hipGetLastError();
}

// grad_y[m][i] = v[m] * coef * sum_p tprime[p][m] * A[p][i]   (A = tau Xi^T)
// on the matrix cores: a wave owns 64 targets (four 16-target tiles) x 32
// coordinates (two 16-coordinate chunks) and steps over the directions four
// at a time with v_mfma_f32_16x16x4f32 (A operand: t' of target 16 t + c,
// direction p + k at lane c + 16 k, so each direction row is read as 256
// contiguous bytes; B operand: A[p + k][16 q + c]).  Lane (c, r) ends with
// targets 16 t + 4r .. +3 of coordinate 16 q + c.
constexpr int kBpTiles = 4;     // 16-target tiles per wave
constexpr int kBpChunks = 2;    // 16-coordinate chunks per wave pass
constexpr int kBpUnroll = 2;    // direction steps of 4 per loop iteration

__global__ __launch_bounds__(kBlock) void backproject_kernel(
    const float* __restrict__ tprime, int64_t ld, int64_t M, int P, int d,
    const float* __restrict__ A, int dpad, float coef,
    const float* __restrict__ v, float* __restrict__ grad_y) {
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int c = lane & 15, k = lane >> 4;
    const int64_t m0 = ((int64_t)blockIdx.x * (kBlock / 64) + wave) * (16 * kBpTiles);
    if (m0 >= M) return;                       // whole waves; no barriers below
    const int i0 = blockIdx.y * (16 * kBpChunks);
    const int nq = min(kBpChunks, (d - i0 + 15) / 16);
    f32x4 acc[kBpTiles][kBpChunks];
#pragma unroll
    for (int t = 0; t < kBpTiles; ++t)
#pragma unroll
        for (int q = 0; q < kBpChunks; ++q) acc[t][q] = f32x4{0.f, 0.f, 0.f, 0.f};
    for (int p0 = 0; p0 < P; p0 += 4 * kBpUnroll) {
        float a[kBpUnroll][kBpTiles], b[kBpUnroll][kBpChunks];
#pragma unroll
        for (int u = 0; u < kBpUnroll; ++u) {
            const int p = p0 + 4 * u + k;
            const float* __restrict__ row = tprime + (int64_t)p * ld + m0 + c;
#pragma unroll
            for (int t = 0; t < kBpTiles; ++t)
                a[u][t] = (p < P && m0 + 16 * t + c < M) ? row[16 * t] : 0.f;
#pragma unroll
            for (int q = 0; q < kBpChunks; ++q) {
                const int col = i0 + 16 * q + c;
                b[u][q] = (p < P && col < d) ? A[(int64_t)p * dpad + col] : 0.f;
            }
        }
#pragma unroll
        for (int u = 0; u < kBpUnroll; ++u)
#pragma unroll
            for (int q = 0; q < kBpChunks; ++q)
                if (q < nq)
#pragma unroll
                    for (int t = 0; t < kBpTiles; ++t)
                        acc[t][q] = __builtin_amdgcn_mfma_f32_16x16x4f32(a[u][t], b[u][q], acc[t][q], 0, 0, 0);
    }
#pragma unroll
    for (int t = 0; t < kBpTiles; ++t)
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            const int64_t m = m0 + 16 * t + 4 * k + j;
            if (m >= M) continue;
            const float sv = v[m] * coef;
#pragma unroll
            for (int q = 0; q < kBpChunks; ++q) {
                const int col = i0 + 16 * q + c;
                if (q < nq && col < d) grad_y[m * d + col] = sv * acc[t][q][j];
            }
        }
}

hipError_t launch_backproject(const float* tprime, int64_t ld, int64_t M,
                              int P, int d, const float* A, int dpad, float coef,
                              const float* v, float* grad_y, hipStream_t stream) {
    const int64_t waves = (M + 16 * kBpTiles - 1) / (16 * kBpTiles);
    dim3 grid((unsigned)((waves + kBlock / 64 - 1) / (kBlock / 64)),
              (unsigned)((d + 16 * kBpChunks - 1) / (16 * kBpChunks)));
    hipLaunchKernelGGL(backproject_kernel, grid, dim3(kBlock), 0, stream, tprime, ld, M,
                       P, d, A, dpad, coef, v, grad_y);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// fused projection + spread / gather (d <= 64)
//
// The projections x~ = tau <xi_p, x_n> never reach memory: a workgroup owns
// 16 directions, computes 16 x 16 projection blocks of its points with
// v_mfma_f32_16x16x32_f16 on split-f16 operands and spreads or interpolates
// them from registers.  This removes the write and re-read of the P x N
// projection matrices, the dominant memory traffic for small d.
//
// Split-f16 operands: a value v (points scaled by 1/R, directions as they
// are, so |v| <= 1) is held as hi = f16(v) and lo = f16(v - hi); then
// |v - hi - lo| <= 2^-22 |v| (lo may be subnormal: the MFMA keeps f16
// subnormals), and hi_a hi_b + hi_a lo_b + lo_a hi_b, each product exact in
// the FP32 accumulation, misses a.b by about 2^-21 |a||b| per term: FP32
// accuracy at three f16 MFMAs per 32 columns instead of eight FP32 MFMAs.
// Operand tiles (split_points_kernel, and on the host for directions): tile t
// (16 rows), k-block kb (32 columns), part q (0 hi, 1 lo) is 64 lanes x 8
// halves, lane l = c + 16 j holding row 16t + c, columns 32kb + 8j .. +7 —
// exactly the MFMA operand layout, so each operand load is one contiguous
// 1 KB wave access.
// ---------------------------------------------------------------------------

constexpr int kSpreadBlock = 512;                          // 8 waves
constexpr int kSpreadWaves = kSpreadBlock / 64;
constexpr int kFuseAcc = 32;                               // FP32 cell accumulators per thread
constexpr int kFuseMaxCells = kFuseAcc * kSpreadBlock;     // kFuseDirs * nr <= this
// wide grids (kFuseDirs * nr up to 16 x 2048, e.g. the energy kernel at
// T = 0.45): twice the accumulators, one workgroup per CU, and the gathers
// stage one group's grids at a time (two would not fit in LDS)
constexpr int kFuseAccWide = 64;
constexpr int kFuseMaxCellsWide = kFuseAccWide * kSpreadBlock;
constexpr int kGatherBlock = 512;                          // 8 waves, one workgroup per CU
constexpr int kGatherWaves = kGatherBlock / 64;
constexpr int kGatherNB = 8;                               // 16-target batches per wave
// wide grids: fewer batches (registers; W = 8 takes three)
constexpr int gather_nb(bool wide, int W) { return !wide ? kGatherNB : (W >= 8 ? 3 : 4); }
constexpr int kDmaBytes = 64 * 16;                         // one wave's 16-byte LDS-direct loads

// split_points_kernel: one thread per (tile, lane), all k-blocks; rows >= N
// and columns >= d are zero.  Also the range check of the fused path: a
// row with |z * scale|^2 > norm2_max sets *flag (z * scale is x / R, and
// |<xi, x / R>| <= max|xi| |x| / R bounds every projection of the row), and
// the row norms of the bound check (BoundCheck) when norm_slot is given.
// Called by whole waves (one tile per wave).
__device__ __forceinline__ void split_points_lane(const float* __restrict__ Z, int64_t N, int d,
                                                  float scale, int KB, int64_t t, int lane,
                                                  u32x4* __restrict__ tiles, float norm2_max,
                                                  int* __restrict__ flag,
                                                  unsigned* __restrict__ norm_slot) {
    // The tile's rows as a buffer: a lane reads its eight columns with two
    // 16-byte loads; rows past N read as zero and columns >= d (the next
    // row's values) are masked.
    const int64_t r0 = 16 * t;
    const int64_t nrows = N - r0 < 16 ? N - r0 : 16;
    const __amdgpu_buffer_rsrc_t zs =
        buffer_rsrc(Z + r0 * d, (nrows > 0 ? nrows : 0) * (int64_t)d * 4);
    float ss = 0.f;
    for (int kb = 0; kb < KB; ++kb) {
        const int col0 = 32 * kb + 8 * (lane >> 4);
        const int off = ((lane & 15) * d + col0) * 4;
        const u32x4 va = __builtin_amdgcn_raw_buffer_load_b128(zs, off, 0, 0);
        const u32x4 vb = __builtin_amdgcn_raw_buffer_load_b128(zs, off + 16, 0, 0);
        h8 hi, lo;
#pragma unroll
        for (int e = 0; e < 8; ++e) {
            const unsigned raw = e < 4 ? va[e] : vb[e - 4];
            const float v = col0 + e < d ? __uint_as_float(raw) * scale : 0.f;
            ss = fmaf(v, v, ss);
            const _Float16 h = (_Float16)v;
            hi[e] = h;
            lo[e] = (_Float16)(v - (float)h);
        }
        const int64_t base = (t * KB + kb) * 2 * 64 + lane;   // in 16-byte units
        tiles[base] = __builtin_bit_cast(u32x4, hi);
        tiles[base + 64] = __builtin_bit_cast(u32x4, lo);
    }
    // the row's columns are spread over lanes c, c+16, c+32, c+48
    ss += __shfl_xor(ss, 16);
    ss += __shfl_xor(ss, 32);
    if (!(ss <= norm2_max) && lane < 16) atomicOr(flag, 1);   // NaN also flags
    if (norm_slot != nullptr) record_norm2(norm_slot, ss);
}

__global__ __launch_bounds__(kBlock) void split_points_kernel(
    const float* __restrict__ Z, int64_t N, int d, float scale, int KB, int64_t ntiles,
    u32x4* __restrict__ tiles, float norm2_max, int* __restrict__ flag,
    unsigned* __restrict__ norm_slot) {
    const int64_t id = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (id >= ntiles * 64) return;                    // whole waves
    split_points_lane(Z, N, d, scale, KB, id >> 6, (int)(id & 63), tiles, norm2_max, flag,
                      norm_slot);
}

// One wave per row of X: the largest |x_n * scale|^2 into *slot (bound
// helper, scale 1; targets shared with the sources, scale 1 / R).
__global__ __launch_bounds__(kBlock) void point_norms_kernel(const float* __restrict__ X,
                                                             int64_t N, int d, float scale,
                                                             unsigned* __restrict__ slot) {
    const int lane = threadIdx.x & 63;
    const int64_t wave = ((int64_t)blockIdx.x * kBlock + threadIdx.x) >> 6;
    const int64_t nwaves = ((int64_t)gridDim.x * kBlock) >> 6;
    float mx = 0.f;
    for (int64_t n = wave; n < N; n += nwaves) {      // uniform over the wave
        const float* __restrict__ row = X + n * d;
        float ss = 0.f;
        for (int k = lane; k < d; k += 64) {
            const float v = row[k] * scale;
            ss = fmaf(v, v, ss);
        }
#pragma unroll
        for (int o = 32; o > 0; o >>= 1) ss += __shfl_xor(ss, o);
        mx = (ss <= 3.4e38f) ? fmaxf(mx, ss) : __builtin_inff();   // NaN -> inf
    }
    record_norm2(slot, mx);
}

__global__ void clear_norms_kernel(unsigned* __restrict__ norms) {
    for (int i = threadIdx.x; i < kNormUints; i += kBlock) norms[i] = 0u;
}

hipError_t launch_clear_norms(unsigned* norms, hipStream_t stream) {
    hipLaunchKernelGGL(clear_norms_kernel, dim3(1), dim3(kBlock), 0, stream, norms);
    return hipGetLastError();
}

hipError_t launch_point_norms(const float* X, int64_t N, int d, float scale, unsigned* slot,
                              hipStream_t stream) {
    const int64_t waves = std::min<int64_t>(N, (int64_t)32768);   // 128 per CU
    hipLaunchKernelGGL(point_norms_kernel, dim3((unsigned)((waves * 64 + kBlock - 1) / kBlock)),
                       dim3(kBlock), 0, stream, X, N, d, scale, slot);
    return hipGetLastError();
}

// operand of one tile: hi and lo parts of each k-block
template <int KB>
struct SplitOp {
    h8 hi[KB], lo[KB];
};

template <int KB>
__device__ __forceinline__ void load_split(SplitOp<KB>& op, __amdgpu_buffer_rsrc_t rs,
                                           int64_t tile_rel, int lane) {
#pragma unroll
    for (int kb = 0; kb < KB; ++kb) {
        const int off = (int)(((tile_rel * KB + kb) * 2) * kSplitTileBytes) + 16 * lane;
        op.hi[kb] = buffer_load_h8(rs, off);
        op.lo[kb] = buffer_load_h8(rs, off + kSplitTileBytes);
    }
}

template <int KB>
__device__ __forceinline__ void load_split(SplitOp<KB>& op, const uint16_t* __restrict__ tiles,
                                           int64_t tile, int lane) {
    const h8* __restrict__ src = reinterpret_cast<const h8*>(tiles);
#pragma unroll
    for (int kb = 0; kb < KB; ++kb) {
        const int64_t base = (tile * KB + kb) * 2 * 64 + lane;
        op.hi[kb] = src[base];
        op.lo[kb] = src[base + 64];
    }
}

// C += A B^T over the tile's columns: the two small cross terms first
template <int KB>
__device__ __forceinline__ f32x4 split_mfma(const SplitOp<KB>& a, const SplitOp<KB>& b, f32x4 acc) {
#pragma unroll
    for (int kb = 0; kb < KB; ++kb) {
        acc = __builtin_amdgcn_mfma_f32_16x16x32_f16(a.hi[kb], b.lo[kb], acc, 0, 0, 0);
        acc = __builtin_amdgcn_mfma_f32_16x16x32_f16(a.lo[kb], b.hi[kb], acc, 0, 0, 0);
    }
#pragma unroll
    for (int kb = 0; kb < KB; ++kb)
        acc = __builtin_amdgcn_mfma_f32_16x16x32_f16(a.hi[kb], b.hi[kb], acc, 0, 0, 0);
    return acc;
}

// Spread with projections computed in registers.  A workgroup owns the 16
// directions 16 dgroup .. 16 dgroup + 15 and the sources of chunk `chunk`; grids are
// kFuseDirs x nr int32 cells in LDS (fixed point per slice as in
// spread_tile) flushed after every slice into per-thread FP32 accumulators.
// v = <xi_p, x_n / R>; x~ = pscale v with pscale = tau R.  The range check
// of these points was done when they were split.
template <int W, int KB, int ACC>
__device__ __forceinline__ void spread_fused_body(
    int* cells, const uint16_t* __restrict__ Xt, int64_t N, const uint16_t* __restrict__ At,
    const float* __restrict__ w, int P, const GridGeom& g, float pscale, int64_t chunk_len,
    const float* __restrict__ slice_max, const WindowArgs& win, float* __restrict__ partial,
    int dgroup, int chunk) {
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int c = lane & 15, r = lane >> 4;
    const int p0 = dgroup * kFuseDirs;
    const int ncell = kFuseDirs * g.nr;
    SplitOp<KB> dop;
    load_split<KB>(dop, At, dgroup, lane);
    float acc[ACC];
#pragma unroll
    for (int q = 0; q < ACC; ++q) acc[q] = 0.f;
    for (int j = tid; j < ncell; j += kSpreadBlock) cells[j] = 0;
    __syncthreads();
    int* gcol = cells + c * g.nr;                     // grid of direction p0 + c
    const WinEval<W> ev(g, win, pscale);
    const int64_t i0 = (int64_t)chunk * chunk_len;   // multiple of 16
    const int len = (int)min(N - i0, chunk_len);           // <= 2^20 sources
    // the chunk's tiles and a few beyond (prefetch), within the tile array;
    // the weights of the chunk only, so sources past it spread nothing
    const int64_t t0 = i0 / 16;
    const int64_t ntiles = (N + 15) / 16;
    const int64_t trange = min(ntiles - t0, (int64_t)(len + 15) / 16 + 2 * kSpreadWaves);
    const __amdgpu_buffer_rsrc_t xs =
        buffer_rsrc(Xt + t0 * KB * 2 * (kSplitTileBytes / 2), trange * KB * 2 * kSplitTileBytes);
    const __amdgpu_buffer_rsrc_t ws = buffer_rsrc(w + i0, (int64_t)len * 4);
    // projects one batch of 16 sources on the 16 directions and spreads it
    auto batch = [&](const SplitOp<KB>& xo, const float (&wv)[4], float scale) {
        // C[point][dir]: lane holds points 4r + i of direction c
        const f32x4 pr = split_mfma<KB>(xo, dop, f32x4{0.f, 0.f, 0.f, 0.f});
#pragma unroll
        for (int i = 0; i < 4; ++i) spread_point<W>(pr[i], wv[i] * scale, ev, win, gcol);
    };
    auto load = [&](SplitOp<KB>& xo, float (&wv)[4], int n0) {
#pragma unroll
        for (int i = 0; i < 4; ++i) wv[i] = buffer_load_f32(ws, (n0 + 4 * r + i) * 4);
        load_split<KB>(xo, xs, n0 / 16, lane);
    };
    // the chunk's pieces inside fixed-point slices, [s0, s1) relative to i0
    // (chunks need not start on a slice; every piece starts on a batch of 16)
    for (int s0 = 0; s0 < len;) {
        const int64_t slice = (i0 + s0) / kSlice;
        const int k = slice_exponent(slice_max[slice]);
        const float scale = ldexpf(1.f, k);
        const int s1 = (int)min((int64_t)len, (slice + 1) * kSlice - i0);
        // batches of 16 sources, wave-strided, two in flight: while one is
        // spread the other's operands load.  Each buffer is reloaded only
        // after its batch is done, so loads land in place (no copies that
        // would wait on them).  The last loads of a slice fetch the next
        // slice's first tiles, harmlessly (loaded again at its start).
        constexpr int stride = kSpreadWaves * 16;
        int n0 = s0 + wave * 16;
        SplitOp<KB> xa, xb;
        float wa[4], wb[4];
        load(xa, wa, n0);
        for (; n0 < s1; n0 += 2 * stride) {
            load(xb, wb, n0 + stride);
            batch(xa, wa, scale);
            load(xa, wa, n0 + 2 * stride);
            if (n0 + stride < s1) batch(xb, wb, scale);
        }
        __syncthreads();
        const float unscale = ldexpf(1.f, -k);
#pragma unroll
        for (int q = 0; q < ACC; ++q) {
            const int j = tid + q * kSpreadBlock;
            if (j < ncell) {
                acc[q] = fmaf((float)cells[j], unscale, acc[q]);
                cells[j] = 0;
            }
        }
        __syncthreads();
        s0 = s1;
    }
    // cells j = dir * nr + (cell - lo): the block's rows of partial are contiguous
    const int nvalid = min(kFuseDirs, P - p0) * g.nr;
    float* __restrict__ dst = partial + ((int64_t)chunk * P + p0) * g.nr;
#pragma unroll
    for (int q = 0; q < ACC; ++q) {
        const int j = tid + q * kSpreadBlock;
        if (j < nvalid) dst[j] = acc[q];
    }
}

// workgroup (x, y): direction group x, source chunk y
template <int W, int KB, int ACC>
__global__ __launch_bounds__(kSpreadBlock) void spread_fused_kernel(
    const uint16_t* __restrict__ Xt, int64_t N, const uint16_t* __restrict__ At,
    const float* __restrict__ w, int P, GridGeom g, float pscale, int64_t chunk_len,
    const float* __restrict__ slice_max, WindowArgs win, float* __restrict__ partial) {
    extern __shared__ int cells[];
    spread_fused_body<W, KB, ACC>(cells, Xt, N, At, w, P, g, pscale, chunk_len, slice_max, win,
                             partial, blockIdx.x, blockIdx.y);
}

// Copies the grids of directions p0 .. p0+np-1 (contiguous, np * nr floats)
// into LDS with 16-byte LDS-direct loads, 1 KB per wave instruction.  Lanes
// past the end re-read the group's first bytes (in bounds) and write into
// the buffer's padding.  Completion is tracked by vmcnt.
__device__ __forceinline__ void gather_stage(const float* __restrict__ grid, int p0, int np,
                                             int nr, float* buf, int wave, int lane) {
    const int nbytes = np * nr * 4;
    const char* src = reinterpret_cast<const char*>(grid + (int64_t)p0 * nr);
    for (int piece = wave; piece * kDmaBytes < nbytes; piece += kGatherWaves) {
        int off = piece * kDmaBytes + lane * 16;
        off = off < nbytes ? off : 0;
        __builtin_amdgcn_global_load_lds(src + off, (lds_void*)(buf + piece * (kDmaBytes / 4)),
                                         16, 0, 0);
    }
}

// Gather with projections computed in registers.  A workgroup owns the
// TGT = 128 NB targets of tile `tile` (NB = gather_nb(WIDE, W)) and
// the direction range `range`
// (prange directions, a multiple of kFuseDirs).  The grids of each group of 16
// directions are staged in one of two LDS buffers while the previous group
// is interpolated (WIDE: one buffer, refilled after each group); lane (c, r)
// holds directions 4r .. 4r+3 of target c of each batch.  Per target the
// four directions are summed in FP32, the groups in FP64.
template <int W, int KB, bool WIDE>
__device__ __forceinline__ void gather_fused_body(
    float* gls, const uint16_t* __restrict__ Yt, int64_t M, const uint16_t* __restrict__ At,
    int P, const GridGeom& g, float pscale, const float* __restrict__ grid, int prange,
    int stage, const WindowArgs& win, double* __restrict__ spart, int64_t ldm, int tile,
    int range) {
    constexpr int NB = gather_nb(WIDE, W);                         // batches per wave
    constexpr int TGT = kGatherWaves * NB * 16;                    // targets per workgroup
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int c = lane & 15, r = lane >> 4;
    const int64_t mb = (int64_t)tile * TGT;
    const int64_t tw = (mb + wave * (NB * 16)) / 16;   // wave's first target tile
    const int p_begin = range * prange;
    const int p_end = min(P, p_begin + prange);
    gather_stage(grid, p_begin, min(kFuseDirs, p_end - p_begin), g.nr, gls, wave, lane);
    // target tiles past the last one read as zero
    const int64_t ntiles = (M + 15) / 16;
    const __amdgpu_buffer_rsrc_t ys =
        buffer_rsrc(Yt + tw * KB * 2 * (kSplitTileBytes / 2),
                    max((int64_t)0, min((int64_t)NB, ntiles - tw)) * KB * 2 * kSplitTileBytes);
    SplitOp<KB> yop[NB];
#pragma unroll
    for (int b = 0; b < NB; ++b) load_split<KB>(yop[b], ys, b, lane);
    double accd[NB];
#pragma unroll
    for (int b = 0; b < NB; ++b) accd[b] = 0.0;
    const WinEval<W> ev(g, win, pscale);
    // Projections of all batches on one group, k-block by k-block across
    // the batches (independent accumulations), then the interpolation.
    // Branch-free: a direction past np (ragged last group) interpolates
    // whatever its LDS row holds and the result is masked to zero by bits
    // (a select here would be turned into a branch around the LDS reads).
    auto group = [&](int np, const float* gb, const SplitOp<KB>& dop) {
        f32x4 pr[NB];
#pragma unroll
        for (int b = 0; b < NB; ++b) pr[b] = f32x4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
        for (int kb = 0; kb < KB; ++kb) {
#pragma unroll
            for (int b = 0; b < NB; ++b)
                pr[b] = __builtin_amdgcn_mfma_f32_16x16x32_f16(dop.hi[kb], yop[b].lo[kb], pr[b], 0, 0, 0);
#pragma unroll
            for (int b = 0; b < NB; ++b)
                pr[b] = __builtin_amdgcn_mfma_f32_16x16x32_f16(dop.lo[kb], yop[b].hi[kb], pr[b], 0, 0, 0);
        }
#pragma unroll
        for (int kb = 0; kb < KB; ++kb)
#pragma unroll
            for (int b = 0; b < NB; ++b)
                // C[dir][target]: lane holds directions 4r + i of target c
                pr[b] = __builtin_amdgcn_mfma_f32_16x16x32_f16(dop.hi[kb], yop[b].hi[kb], pr[b], 0, 0, 0);
#pragma unroll
        for (int b = 0; b < NB; ++b) {
            float t = 0.f;
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                const int dir = 4 * r + i;
                const float v = interp<W>(pr[b][i], gb + dir * g.nr, ev, win);
                const unsigned keep = 0u - (unsigned)(dir < np);
                t += __uint_as_float(__float_as_uint(v) & keep);
            }
            accd[b] += (double)t;
        }
    };
    // Two groups per iteration, ping-ponging buffers and direction
    // operands: a group's grids and operand are fetched while the previous
    // group is interpolated.  Before a group starts, this wave's fetches have
    // landed (vmcnt) and, after the barrier, every wave's have and no wave
    // still reads the buffer about to be refilled.
    SplitOp<KB> da, db;
    load_split<KB>(da, At, p_begin / kFuseDirs, lane);
    if constexpr (WIDE) {
        // one buffer: after a group every wave leaves it before the next
        // group's grids go in; the next direction operand still loads
        // during the group
        for (int p0 = p_begin; p0 < p_end; p0 += 2 * kFuseDirs) {
            asm volatile("s_waitcnt vmcnt(0)" ::: "memory");
            __syncthreads();
            const int p1 = p0 + kFuseDirs;
            if (p1 < p_end) load_split<KB>(db, At, p1 / kFuseDirs, lane);
            group(min(kFuseDirs, p_end - p0), gls, da);
            if (p1 >= p_end) break;
            __syncthreads();
            gather_stage(grid, p1, min(kFuseDirs, p_end - p1), g.nr, gls, wave, lane);
            asm volatile("s_waitcnt vmcnt(0)" ::: "memory");
            __syncthreads();
            const int p2 = p1 + kFuseDirs;
            if (p2 < p_end) load_split<KB>(da, At, p2 / kFuseDirs, lane);
            group(min(kFuseDirs, p_end - p1), gls, db);
            if (p2 >= p_end) break;
            __syncthreads();
            gather_stage(grid, p2, min(kFuseDirs, p_end - p2), g.nr, gls, wave, lane);
        }
    } else {
        float* buf0 = gls;
        float* buf1 = gls + stage;
        for (int p0 = p_begin; p0 < p_end; p0 += 2 * kFuseDirs) {
            asm volatile("s_waitcnt vmcnt(0)" ::: "memory");
            __syncthreads();
            const int p1 = p0 + kFuseDirs;
            if (p1 < p_end) {
                gather_stage(grid, p1, min(kFuseDirs, p_end - p1), g.nr, buf1, wave, lane);
                load_split<KB>(db, At, p1 / kFuseDirs, lane);
            }
            group(min(kFuseDirs, p_end - p0), buf0, da);
            if (p1 >= p_end) break;
            asm volatile("s_waitcnt vmcnt(0)" ::: "memory");
            __syncthreads();
            const int p2 = p1 + kFuseDirs;
            if (p2 < p_end) {
                gather_stage(grid, p2, min(kFuseDirs, p_end - p2), g.nr, buf0, wave, lane);
                load_split<KB>(da, At, p2 / kFuseDirs, lane);
            }
            group(min(kFuseDirs, p_end - p1), buf1, db);
        }
    }
    // sum the four lane groups r holding the same targets
#pragma unroll
    for (int b = 0; b < NB; ++b) {
        double v = accd[b];
        v += __shfl_xor(v, 16);
        v += __shfl_xor(v, 32);
        const int64_t m = mb + wave * (NB * 16) + 16 * b + c;
        if (r == 0 && m < M) spart[(int64_t)range * ldm + m] = v;
    }
}

// workgroup (x, y): target tile x, direction range y
template <int W, int KB, bool WIDE>
__global__ __launch_bounds__(kGatherBlock) void gather_fused_kernel(
    const uint16_t* __restrict__ Yt, int64_t M, const uint16_t* __restrict__ At, int P,
    GridGeom g, float pscale, const float* __restrict__ grid, int prange, int stage,
    WindowArgs win, double* __restrict__ spart, int64_t ldm) {
    extern __shared__ float gls[];                    // 2 x stage floats (WIDE: 1 x)
    gather_fused_body<W, KB, WIDE>(gls, Yt, M, At, P, g, pscale, grid, prange, stage, win, spart, ldm,
                             blockIdx.x, blockIdx.y);
}

// Adjoint in the targets, fused: t'_{m,p}, the derivative grid of direction
// p interpolated at tau <xi_p, y_m>, is formed in registers exactly as the
// gather forms t_{m,p}, and back-projected at once on the matrix cores:
//   G[i][m] += sum over the 16 directions p of a group of (tau xi_p)_i t'_{m,p}
// as four v_mfma_f32_16x16x4f32 per 16 coordinates.  Lane (c, r) holds t'
// of directions 4r + i of target c, which is the B operand of MFMA i
// (k = r, column c) when its A operand holds (tau xi)_{4k + i} (Ab: per
// group, MFMA i and 16-coordinate chunk dc, lane m + 16k holds
// tau xi_{16 group + 4k + i}[16 dc + m], zero past P and d).  Workgroup
// (x, y): kGradTargets targets of tile x, direction range y; writes
// gpart[(y * ldg + m) * 16 DC + i] (FP32, summed over the ranges by
// grad_reduce_kernel).
constexpr int kGradNB = 4;                                   // 16-target batches per wave
constexpr int kGradTargets = kGatherWaves * kGradNB * 16;
constexpr int kGradMaxDC = kSplitMaxD / 16;

template <int W, int KB, bool WIDE>
__global__ __launch_bounds__(kGatherBlock) void gather_grad_fused_kernel(
    const uint16_t* __restrict__ Yt, int64_t M, const uint16_t* __restrict__ At,
    const float* __restrict__ Ab, int DC, int P, GridGeom g, float pscale,
    const float* __restrict__ grid_d, int prange, int stage, WindowArgs win,
    float* __restrict__ gpart, int64_t ldg) {
    extern __shared__ float gls[];                    // 2 x stage floats
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int c = lane & 15, r = lane >> 4;
    const int64_t mb = (int64_t)blockIdx.x * kGradTargets;
    const int64_t tw = (mb + wave * (kGradNB * 16)) / 16;     // wave's first target tile
    const int p_begin = blockIdx.y * prange;
    const int p_end = min(P, p_begin + prange);
    gather_stage(grid_d, p_begin, min(kFuseDirs, p_end - p_begin), g.nr, gls, wave, lane);
    const int64_t ntiles = (M + 15) / 16;
    const __amdgpu_buffer_rsrc_t ys =
        buffer_rsrc(Yt + tw * KB * 2 * (kSplitTileBytes / 2),
                    max((int64_t)0, min((int64_t)kGradNB, ntiles - tw)) * KB * 2 * kSplitTileBytes);
    SplitOp<KB> yop[kGradNB];
#pragma unroll
    for (int b = 0; b < kGradNB; ++b) load_split<KB>(yop[b], ys, b, lane);
    f32x4 gacc[kGradNB][kGradMaxDC];
#pragma unroll
    for (int b = 0; b < kGradNB; ++b)
#pragma unroll
        for (int q = 0; q < kGradMaxDC; ++q) gacc[b][q] = f32x4{0.f, 0.f, 0.f, 0.f};
    const WinEval<W> ev(g, win, pscale);
    auto group = [&](int np, const float* gb, const SplitOp<KB>& dop, int grp) {
        f32x4 pr[kGradNB];
#pragma unroll
        for (int b = 0; b < kGradNB; ++b) pr[b] = f32x4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
        for (int kb = 0; kb < KB; ++kb) {
#pragma unroll
            for (int b = 0; b < kGradNB; ++b)
                pr[b] = __builtin_amdgcn_mfma_f32_16x16x32_f16(dop.hi[kb], yop[b].lo[kb], pr[b], 0, 0, 0);
#pragma unroll
            for (int b = 0; b < kGradNB; ++b)
                pr[b] = __builtin_amdgcn_mfma_f32_16x16x32_f16(dop.lo[kb], yop[b].hi[kb], pr[b], 0, 0, 0);
        }
#pragma unroll
        for (int kb = 0; kb < KB; ++kb)
#pragma unroll
            for (int b = 0; b < kGradNB; ++b)
                pr[b] = __builtin_amdgcn_mfma_f32_16x16x32_f16(dop.hi[kb], yop[b].hi[kb], pr[b], 0, 0, 0);
        // this lane's back-projection operands of the group
        const float* __restrict__ ag = Ab + (int64_t)grp * 4 * DC * 64 + lane;
        float abv[kGradMaxDC][4];
#pragma unroll
        for (int q = 0; q < kGradMaxDC; ++q)
#pragma unroll
            for (int i = 0; i < 4; ++i) abv[q][i] = q < DC ? ag[(i * DC + q) * 64] : 0.f;
#pragma unroll
        for (int b = 0; b < kGradNB; ++b) {
            float tv[4];
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                const int dir = 4 * r + i;
                const float v = interp<W>(pr[b][i], gb + dir * g.nr, ev, win);
                const unsigned keep = 0u - (unsigned)(dir < np);
                tv[i] = __uint_as_float(__float_as_uint(v) & keep);
            }
#pragma unroll
            for (int q = 0; q < kGradMaxDC; ++q) {
                if (q >= DC) break;
#pragma unroll
                for (int i = 0; i < 4; ++i)
                    gacc[b][q] = __builtin_amdgcn_mfma_f32_16x16x4f32(abv[q][i], tv[i], gacc[b][q],
                                                                      0, 0, 0);
            }
        }
    };
    SplitOp<KB> da, db;
    load_split<KB>(da, At, p_begin / kFuseDirs, lane);
    float* buf0 = gls;
    if constexpr (WIDE) {
        // one buffer, refilled after each group (see gather_fused_body)
        for (int p0 = p_begin; p0 < p_end; p0 += 2 * kFuseDirs) {
            asm volatile("s_waitcnt vmcnt(0)" ::: "memory");
            __syncthreads();
            const int p1 = p0 + kFuseDirs;
            if (p1 < p_end) load_split<KB>(db, At, p1 / kFuseDirs, lane);
            group(min(kFuseDirs, p_end - p0), buf0, da, p0 / kFuseDirs);
            if (p1 >= p_end) break;
            __syncthreads();
            gather_stage(grid_d, p1, min(kFuseDirs, p_end - p1), g.nr, buf0, wave, lane);
            asm volatile("s_waitcnt vmcnt(0)" ::: "memory");
            __syncthreads();
            const int p2 = p1 + kFuseDirs;
            if (p2 < p_end) load_split<KB>(da, At, p2 / kFuseDirs, lane);
            group(min(kFuseDirs, p_end - p1), buf0, db, p1 / kFuseDirs);
            if (p2 >= p_end) break;
            __syncthreads();
            gather_stage(grid_d, p2, min(kFuseDirs, p_end - p2), g.nr, buf0, wave, lane);
        }
    } else {
        float* buf1 = gls + stage;
        for (int p0 = p_begin; p0 < p_end; p0 += 2 * kFuseDirs) {
            asm volatile("s_waitcnt vmcnt(0)" ::: "memory");
            __syncthreads();
            const int p1 = p0 + kFuseDirs;
            if (p1 < p_end) {
                gather_stage(grid_d, p1, min(kFuseDirs, p_end - p1), g.nr, buf1, wave, lane);
                load_split<KB>(db, At, p1 / kFuseDirs, lane);
            }
            group(min(kFuseDirs, p_end - p0), buf0, da, p0 / kFuseDirs);
            if (p1 >= p_end) break;
            asm volatile("s_waitcnt vmcnt(0)" ::: "memory");
            __syncthreads();
            const int p2 = p1 + kFuseDirs;
            if (p2 < p_end) {
                gather_stage(grid_d, p2, min(kFuseDirs, p_end - p2), g.nr, buf0, wave, lane);
                load_split<KB>(da, At, p2 / kFuseDirs, lane);
            }
            group(min(kFuseDirs, p_end - p1), buf1, db, p1 / kFuseDirs);
        }
    }
    // lane (c, r) holds coordinates 16 q + 4 r + j of target c
    const int dcp = 16 * DC;
#pragma unroll
    for (int b = 0; b < kGradNB; ++b) {
        const int64_t m = mb + wave * (kGradNB * 16) + 16 * b + c;
        if (m >= M) continue;
        float* __restrict__ dst = gpart + ((int64_t)blockIdx.y * ldg + m) * dcp + 4 * r;
#pragma unroll
        for (int q = 0; q < kGradMaxDC; ++q) {
            if (q >= DC) break;
            *reinterpret_cast<float4*>(dst + 16 * q) =
                make_float4(gacc[b][q][0], gacc[b][q][1], gacc[b][q][2], gacc[b][q][3]);
        }
    }
}

// grad_y[m * d + i] = coef * v[m] * sum over ranges of gpart[(r * ldg + m) * 16 DC + i]
__global__ __launch_bounds__(kBlock) void grad_reduce_kernel(
    const float* __restrict__ gpart, int nrange, int64_t ldg, int DC, int64_t M, int d,
    float coef, const float* __restrict__ v, float* __restrict__ grad_y) {
    const int64_t e = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (e >= M * d) return;
    const int64_t m = e / d;
    const int i = (int)(e - m * d);
    const int dcp = 16 * DC;
    float s = 0.f;
    for (int q = 0; q < nrange; ++q) s += gpart[((int64_t)q * ldg + m) * dcp + i];
    grad_y[e] = coef * v[m] * s;
}

template <int W, int KB, int ACC>
void launch_spread_fused_t(dim3 grid, size_t lds, hipStream_t stream, const uint16_t* Xt,
                           int64_t N, const uint16_t* At, const float* w, int P,
                           const GridGeom& g, float pscale, int64_t chunk_len,
                           const float* slice_max, const WindowArgs& win, float* partial) {
    static bool attr_set = false;      // dynamic LDS above 64 KB must be enabled per kernel
    if (!attr_set) {
        (void)hipFuncSetAttribute(reinterpret_cast<const void*>(&spread_fused_kernel<W, KB, ACC>),
                                  hipFuncAttributeMaxDynamicSharedMemorySize,
                                  ACC * kSpreadBlock * (int)sizeof(int));
        attr_set = true;
    }
    hipLaunchKernelGGL((spread_fused_kernel<W, KB, ACC>), grid, dim3(kSpreadBlock), lds, stream,
                       Xt, N, At, w, P, g, pscale, chunk_len, slice_max, win, partial);
}

template <int W, int KB, bool WIDE>
void launch_gather_fused_t(dim3 grid, size_t lds, hipStream_t stream, const uint16_t* Yt,
                           int64_t M, const uint16_t* At, int P, const GridGeom& g, float pscale,
                           const float* gridv, int prange, int stage, const WindowArgs& win,
                           double* spart, int64_t ldm) {
    static bool attr_set = false;      // dynamic LDS above 64 KB must be enabled per kernel
    if (!attr_set) {
        (void)hipFuncSetAttribute(reinterpret_cast<const void*>(&gather_fused_kernel<W, KB, WIDE>),
                                  hipFuncAttributeMaxDynamicSharedMemorySize,
                                  2 * kFuseMaxCells * (int)sizeof(float));
        attr_set = true;
    }
    hipLaunchKernelGGL((gather_fused_kernel<W, KB, WIDE>), grid, dim3(kGatherBlock), lds, stream, Yt,
                       M, At, P, g, pscale, gridv, prange, stage, win, spart, ldm);
}

template <int W, int KB, bool WIDE>
void launch_gather_grad_t(dim3 grid, size_t lds, hipStream_t stream, const uint16_t* Yt,
                          int64_t M, const uint16_t* At, const float* Ab, int DC, int P,
                          const GridGeom& g, float pscale, const float* grid_d, int prange,
                          int stage, const WindowArgs& win, float* gpart, int64_t ldg) {
    static bool attr_set = false;      // dynamic LDS above 64 KB must be enabled per kernel
    if (!attr_set) {
        (void)hipFuncSetAttribute(reinterpret_cast<const void*>(&gather_grad_fused_kernel<W, KB, WIDE>),
                                  hipFuncAttributeMaxDynamicSharedMemorySize,
                                  2 * kFuseMaxCells * (int)sizeof(float));
        attr_set = true;
    }
    hipLaunchKernelGGL((gather_grad_fused_kernel<W, KB, WIDE>), grid, dim3(kGatherBlock), lds, stream,
                       Yt, M, At, Ab, DC, P, g, pscale, grid_d, prange, stage, win, gpart, ldg);
}

int64_t fused_grad_tile() { return kGradTargets; }

hipError_t launch_grad_fused(int W, const uint16_t* Yt, int64_t M, int d, const uint16_t* At,
                             const float* Ab, int P, GridGeom g, float pscale,
                             const float* grid_d, int prange, const WindowArgs& win,
                             float* gpart, int64_t ldg, float coef, const float* v,
                             float* grad_y, hipStream_t stream) {
    if (!fused_supported(d, g.nr) || prange % kFuseDirs != 0 || M > ldg) return hipErrorInvalidValue;
    using L = void (*)(dim3, size_t, hipStream_t, const uint16_t*, int64_t, const uint16_t*,
                       const float*, int, int, const GridGeom&, float, const float*, int, int,
                       const WindowArgs&, float*, int64_t);
    static const L t[2][3][2] = {
        {{launch_gather_grad_t<4, 1, false>, launch_gather_grad_t<4, 2, false>},
         {launch_gather_grad_t<6, 1, false>, launch_gather_grad_t<6, 2, false>},
         {launch_gather_grad_t<8, 1, false>, launch_gather_grad_t<8, 2, false>}},
        {{launch_gather_grad_t<4, 1, true>, launch_gather_grad_t<4, 2, true>},
         {launch_gather_grad_t<6, 1, true>, launch_gather_grad_t<6, 2, true>},
         {launch_gather_grad_t<8, 1, true>, launch_gather_grad_t<8, 2, true>}}};
    const int wi = W == 4 ? 0 : W == 6 ? 1 : W == 8 ? 2 : -1;
    if (wi < 0) return hipErrorInvalidValue;
    const int DC = (d + 15) / 16;
    const int stage = (kFuseDirs * g.nr + kDmaBytes / 4 - 1) / (kDmaBytes / 4) * (kDmaBytes / 4);
    const int nrange = (P + prange - 1) / prange;
    dim3 gd((unsigned)((M + kGradTargets - 1) / kGradTargets), (unsigned)nrange);
    const bool wide = fused_wide(g.nr);
    t[wide][wi][split_kblocks(d) - 1](gd, (size_t)(wide ? 1 : 2) * stage * sizeof(float), stream,
                                      Yt, M, At, Ab, DC, P, g, pscale, grid_d, prange, stage, win,
                                      gpart, ldg);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(grad_reduce_kernel, dim3((unsigned)((M * d + kBlock - 1) / kBlock)),
                       dim3(kBlock), 0, stream, gpart, nrange, ldg, DC, M, d, coef, v, grad_y);
    return hipGetLastError();
}

bool fused_supported(int d, int nr) {
    return d >= 1 && d <= kSplitMaxD && kFuseDirs * nr <= kFuseMaxCellsWide;
}

bool fused_wide(int nr) { return kFuseDirs * nr > kFuseMaxCells; }

int64_t fused_gather_tile(int nr, int W) {
    return (int64_t)kGatherWaves * 16 * gather_nb(fused_wide(nr), W);
}

int64_t split_tiles_bytes(int64_t rows, int d) {
    return (rows + 15) / 16 * split_kblocks(d) * 2 * kSplitTileBytes;
}

hipError_t launch_split_points(const float* Z, int64_t N, int d, float scale, uint16_t* tiles,
                               float norm2_max, int* flag, unsigned* norm_slot,
                               hipStream_t stream) {
    const int KB = split_kblocks(d);
    const int64_t ntiles = (N + 15) / 16;
    const int64_t threads = ntiles * 64;
    hipLaunchKernelGGL(split_points_kernel, dim3((unsigned)((threads + kBlock - 1) / kBlock)),
                       dim3(kBlock), 0, stream, Z, N, d, scale, KB, ntiles,
                       reinterpret_cast<u32x4*>(tiles), norm2_max, flag, norm_slot);
    return hipGetLastError();
}

void fused_occupancy(int W, int d, int nr, int* spread_blocks, int* gather_blocks) {
    *spread_blocks = 1;
    *gather_blocks = 1;
    if (!fused_supported(d, nr)) return;
    const bool wide = fused_wide(nr);
    const void* sk = nullptr;
    const void* gk = nullptr;
    // occupancy is set by LDS and registers; the larger operand shape
    // stands for both
    switch (W) {
        case 4:
            sk = wide ? (const void*)&spread_fused_kernel<4, 2, kFuseAccWide> : (const void*)&spread_fused_kernel<4, 2, kFuseAcc>;
            gk = wide ? (const void*)&gather_fused_kernel<4, 2, true> : (const void*)&gather_fused_kernel<4, 2, false>;
            break;
        case 6:
            sk = wide ? (const void*)&spread_fused_kernel<6, 2, kFuseAccWide> : (const void*)&spread_fused_kernel<6, 2, kFuseAcc>;
            gk = wide ? (const void*)&gather_fused_kernel<6, 2, true> : (const void*)&gather_fused_kernel<6, 2, false>;
            break;
        default:
            sk = wide ? (const void*)&spread_fused_kernel<8, 2, kFuseAccWide> : (const void*)&spread_fused_kernel<8, 2, kFuseAcc>;
            gk = wide ? (const void*)&gather_fused_kernel<8, 2, true> : (const void*)&gather_fused_kernel<8, 2, false>;
            break;
    }
    const int stage = (kFuseDirs * nr + kDmaBytes / 4 - 1) / (kDmaBytes / 4) * (kDmaBytes / 4);
    (void)hipFuncSetAttribute(sk, hipFuncAttributeMaxDynamicSharedMemorySize,
                              kFuseMaxCellsWide * (int)sizeof(int));
    (void)hipFuncSetAttribute(gk, hipFuncAttributeMaxDynamicSharedMemorySize,
                              2 * kFuseMaxCells * (int)sizeof(float));
    int b = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&b, sk, kSpreadBlock,
                                                     (size_t)kFuseDirs * nr * sizeof(int)) == hipSuccess && b > 0)
        *spread_blocks = b;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&b, gk, kGatherBlock,
                                                     (size_t)(wide ? 1 : 2) * stage * sizeof(float)) == hipSuccess && b > 0)
        *gather_blocks = b;
}

hipError_t launch_spread_fused(int W, const uint16_t* Xt, int64_t N, int d, const uint16_t* At,
                               const float* w, int P, GridGeom g, float pscale, int nchunk,
                               int64_t chunk_len, float* slice_max, const WindowArgs& win,
                               float* partial, hipStream_t stream) {
    if (!fused_supported(d, g.nr) || chunk_len % 16 != 0 || chunk_len <= 0)
        return hipErrorInvalidValue;
    using L = void (*)(dim3, size_t, hipStream_t, const uint16_t*, int64_t, const uint16_t*,
                       const float*, int, const GridGeom&, float, int64_t, const float*,
                       const WindowArgs&, float*);
    static const L t[2][3][2] = {
        {{launch_spread_fused_t<4, 1, kFuseAcc>, launch_spread_fused_t<4, 2, kFuseAcc>},
         {launch_spread_fused_t<6, 1, kFuseAcc>, launch_spread_fused_t<6, 2, kFuseAcc>},
         {launch_spread_fused_t<8, 1, kFuseAcc>, launch_spread_fused_t<8, 2, kFuseAcc>}},
        {{launch_spread_fused_t<4, 1, kFuseAccWide>, launch_spread_fused_t<4, 2, kFuseAccWide>},
         {launch_spread_fused_t<6, 1, kFuseAccWide>, launch_spread_fused_t<6, 2, kFuseAccWide>},
         {launch_spread_fused_t<8, 1, kFuseAccWide>, launch_spread_fused_t<8, 2, kFuseAccWide>}}};
    const int wi = W == 4 ? 0 : W == 6 ? 1 : W == 8 ? 2 : -1;
    if (wi < 0) return hipErrorInvalidValue;
    hipLaunchKernelGGL(slice_max_kernel, dim3((unsigned)((N + kSlice - 1) / kSlice)), dim3(kBlock),
                       0, stream, w, N, slice_max);
    dim3 grid((unsigned)((P + kFuseDirs - 1) / kFuseDirs), (unsigned)nchunk);
    t[fused_wide(g.nr)][wi][split_kblocks(d) - 1](grid, (size_t)kFuseDirs * g.nr * sizeof(int),
                                                  stream, Xt, N, At, w, P, g, pscale, chunk_len,
                                                  slice_max, win, partial);
    return hipGetLastError();
}

hipError_t launch_gather_fused(int W, const uint16_t* Yt, int64_t M, int d, const uint16_t* At,
                               int P, GridGeom g, float pscale, const float* grid, int prange,
                               const WindowArgs& win, double* spart, int64_t ldm,
                               hipStream_t stream) {
    if (!fused_supported(d, g.nr) || prange % kFuseDirs != 0) return hipErrorInvalidValue;
    using L = void (*)(dim3, size_t, hipStream_t, const uint16_t*, int64_t, const uint16_t*, int,
                       const GridGeom&, float, const float*, int, int, const WindowArgs&, double*,
                       int64_t);
    static const L t[2][3][2] = {
        {{launch_gather_fused_t<4, 1, false>, launch_gather_fused_t<4, 2, false>},
         {launch_gather_fused_t<6, 1, false>, launch_gather_fused_t<6, 2, false>},
         {launch_gather_fused_t<8, 1, false>, launch_gather_fused_t<8, 2, false>}},
        {{launch_gather_fused_t<4, 1, true>, launch_gather_fused_t<4, 2, true>},
         {launch_gather_fused_t<6, 1, true>, launch_gather_fused_t<6, 2, true>},
         {launch_gather_fused_t<8, 1, true>, launch_gather_fused_t<8, 2, true>}}};
    const int wi = W == 4 ? 0 : W == 6 ? 1 : W == 8 ? 2 : -1;
    if (wi < 0) return hipErrorInvalidValue;
    // one staging buffer: the group's grids rounded up to whole 1 KB pieces
    const int stage = (kFuseDirs * g.nr + kDmaBytes / 4 - 1) / (kDmaBytes / 4) * (kDmaBytes / 4);
    const int64_t tgt = fused_gather_tile(g.nr, W);
    dim3 gd((unsigned)((M + tgt - 1) / tgt),
            (unsigned)((P + prange - 1) / prange));
    const bool wide = fused_wide(g.nr);
    t[wide][wi][split_kblocks(d) - 1](gd, (size_t)(wide ? 1 : 2) * stage * sizeof(float), stream,
                                      Yt, M, At, P, g, pscale, grid, prange, stage, win, spart,
                                      ldm);
    return hipGetLastError();
}



// ---------------------------------------------------------------------------
// batched form: persistent kernels walking task lists
// ---------------------------------------------------------------------------

__global__ __launch_bounds__(kBlock) void batch_project_kernel(
    const BatchProblem* __restrict__ probs, const BatchTask* __restrict__ tasks, int ntasks,
    int P, int* __restrict__ flag) {
    __shared__ ProjSmemF32 sm;
    for (int t = blockIdx.x; t < ntasks; t += gridDim.x) {
        const BatchTask tk = tasks[t];
        const BatchProblem& pr = probs[tk.prob];
        const bool is_y = tk.a != 0;
        const float* __restrict__ X = is_y ? pr.y : pr.x;
        const int64_t n = is_y ? pr.M : pr.N;
        const int64_t n0 = (int64_t)tk.b * kProjBN;
        project_tile_f32(sm, X, n, pr.d, pr.dpad, pr.A, P, is_y ? pr.yproj : pr.xproj,
                         is_y ? pr.ldy : pr.ldx, pr.bound, flag, tk.c * kProjBM, n0);
        if (tk.c == 0) {   // the point tile's row norms, once (bound check)
            float ss = 0.f;
            if (threadIdx.x < kProjBN && n0 + threadIdx.x < n) {
                const float* __restrict__ row = X + (n0 + threadIdx.x) * pr.d;
                for (int k = 0; k < pr.d; ++k) {
                    const float v = row[k] * pr.inv_r;
                    ss = fmaf(v, v, ss);
                }
            }
            record_norm2(pr.norms + (is_y ? kNormRoleUints : 0), ss);
        }
    }
}

__global__ __launch_bounds__(kBlock) void batch_scale_kernel(
    const BatchProblem* __restrict__ probs, const BatchTask* __restrict__ tasks, int ntasks) {
    __shared__ float red[kBlock];
    for (int t = blockIdx.x; t < ntasks; t += gridDim.x) {
        const BatchTask tk = tasks[t];
        const BatchProblem& pr = probs[tk.prob];
        slice_max_tile(red, pr.w, pr.N, tk.a, pr.slice_max);
    }
}

template <int W>
__global__ __launch_bounds__(kBlock) void batch_spread_kernel(
    const BatchProblem* __restrict__ probs, const BatchTask* __restrict__ tasks, int ntasks,
    int P, WindowArgs win) {
    extern __shared__ int lds_bspread[];
    for (int t = blockIdx.x; t < ntasks; t += gridDim.x) {
        const BatchTask tk = tasks[t];
        const BatchProblem& pr = probs[tk.prob];
        spread_tile<W>(lds_bspread, pr.xproj, pr.ldx, pr.w, pr.N, P, pr.g, pr.chunk_len,
                       pr.slice_max, win, pr.partial, tk.a, tk.b);
    }
}

__global__ __launch_bounds__(kBlock) void batch_fftconv_kernel(
    const BatchProblem* __restrict__ probs, const BatchTask* __restrict__ tasks, int ntasks,
    int P) {
    extern __shared__ float2 cbuf[];
    for (int t = blockIdx.x; t < ntasks; t += gridDim.x) {
        const BatchTask tk = tasks[t];
        const BatchProblem& pr = probs[tk.prob];
        fftconv_tile(cbuf, pr.partial, pr.nchunk, P, pr.g, pr.tw, pr.mult, nullptr, pr.grid,
                     nullptr, tk.a);
    }
}

template <int W>
__global__ __launch_bounds__(kBlock) void batch_gather_kernel(
    const BatchProblem* __restrict__ probs, const BatchTask* __restrict__ tasks, int ntasks,
    int P, int pstage, WindowArgs win) {
    extern __shared__ float lds[];
    for (int t = blockIdx.x; t < ntasks; t += gridDim.x) {
        const BatchTask tk = tasks[t];
        const BatchProblem& pr = probs[tk.prob];
        const float* yp = pr.same_xy ? pr.xproj : pr.yproj;
        const int64_t ldy = pr.same_xy ? pr.ldx : pr.ldy;
        gather_tile<W, false>(lds, yp, ldy, pr.M, P, pr.g, pr.grid, pr.pg, pstage, win,
                              pr.spart, pr.ldm, nullptr, 0, tk.a, tk.b);
    }
}

// The first reduce task of a problem also finishes its bound check.
__global__ __launch_bounds__(kBlock) void batch_reduce_kernel(
    const BatchProblem* __restrict__ probs, const BatchTask* __restrict__ tasks, int ntasks,
    int P, int* __restrict__ flag) {
    for (int t = blockIdx.x; t < ntasks; t += gridDim.x) {
        const BatchTask tk = tasks[t];
        const BatchProblem& pr = probs[tk.prob];
        reduce_tile(pr.spart, pr.ngroup, pr.ldm, pr.M, 1.0 / P, pr.s,
                    (int64_t)tk.a * kBlock + threadIdx.x);
        if (tk.a == 0 && threadIdx.x < 64)
            finish_bound_check(BoundCheck{pr.norms, flag, pr.norm_lim, pr.same_xy});
    }
}

// Fused batch phases.  Split: one task per kSplitTaskTiles tiles of one
// point set.  Spread and gather: the single-problem bodies, the operand
// shape (ceil(d / 32) k-blocks) chosen per task.
__global__ __launch_bounds__(kBlock) void batch_split_kernel(
    const BatchProblem* __restrict__ probs, const BatchTask* __restrict__ tasks, int ntasks,
    int* __restrict__ flag) {
    for (int t = blockIdx.x; t < ntasks; t += gridDim.x) {
        const BatchTask tk = tasks[t];
        const BatchProblem& pr = probs[tk.prob];
        const bool is_y = tk.a != 0;
        const int64_t n = is_y ? pr.M : pr.N;
        const int64_t ntiles = (n + 15) / 16;
        const int64_t t0 = (int64_t)tk.b * kSplitTaskTiles;
        const int64_t t1 = min(ntiles, t0 + kSplitTaskTiles);
        u32x4* dst = reinterpret_cast<u32x4*>(is_y ? pr.yt : pr.xt);
        for (int64_t id = t0 * 64 + threadIdx.x; id < t1 * 64; id += kBlock)
            split_points_lane(is_y ? pr.y : pr.x, n, pr.d, pr.inv_r, pr.kb, id >> 6,
                              (int)(id & 63), dst, pr.norm2_max, flag,
                              pr.norms + (is_y ? kNormRoleUints : 0));
    }
}

// two workgroups per CU (at most 128 VGPRs), as the single-problem kernel
template <int W>
__global__ __launch_bounds__(kSpreadBlock) __attribute__((amdgpu_waves_per_eu(4))) void
batch_spread_fused_kernel(
    const BatchProblem* __restrict__ probs, const BatchTask* __restrict__ tasks, int ntasks,
    int P, WindowArgs win) {
    extern __shared__ int bcells[];
    for (int t = blockIdx.x; t < ntasks; t += gridDim.x) {
        const BatchTask tk = tasks[t];
        const BatchProblem& pr = probs[tk.prob];
        if (pr.kb == 1)
            spread_fused_body<W, 1, kFuseAcc>(bcells, pr.xt, pr.N, pr.at, pr.w, P, pr.g, pr.pscale,
                                    pr.chunk_len, pr.slice_max, win, pr.partial, tk.a, tk.b);
        else
            spread_fused_body<W, 2, kFuseAcc>(bcells, pr.xt, pr.N, pr.at, pr.w, P, pr.g, pr.pscale,
                                    pr.chunk_len, pr.slice_max, win, pr.partial, tk.a, tk.b);
        __syncthreads();
    }
}

template <int W>
__global__ __launch_bounds__(kGatherBlock) void batch_gather_fused_kernel(
    const BatchProblem* __restrict__ probs, const BatchTask* __restrict__ tasks, int ntasks,
    int P, WindowArgs win) {
    extern __shared__ float bgls[];
    for (int t = blockIdx.x; t < ntasks; t += gridDim.x) {
        const BatchTask tk = tasks[t];
        const BatchProblem& pr = probs[tk.prob];
        const int stage = (kFuseDirs * pr.g.nr + kDmaBytes / 4 - 1) / (kDmaBytes / 4) * (kDmaBytes / 4);
        const uint16_t* yt = pr.same_xy ? pr.xt : pr.yt;
        // no wave may still read the staging buffers of the previous task
        __syncthreads();
        if (pr.kb == 1)
            gather_fused_body<W, 1, false>(bgls, yt, pr.M, pr.at, P, pr.g, pr.pscale, pr.grid, pr.pg,
                                    stage, win, pr.spart, pr.ldm, tk.a, tk.b);
        else
            gather_fused_body<W, 2, false>(bgls, yt, pr.M, pr.at, P, pr.g, pr.pscale, pr.grid, pr.pg,
                                    stage, win, pr.spart, pr.ldm, tk.a, tk.b);
    }
}

size_t fused_spread_lds(int nr) { return (size_t)kFuseDirs * nr * sizeof(int); }

size_t stored_spread_lds(int nr) { return (size_t)nr * sizeof(int); }

size_t fused_gather_lds(int nr) {
    const int stage = (kFuseDirs * nr + kDmaBytes / 4 - 1) / (kDmaBytes / 4) * (kDmaBytes / 4);
    return (size_t)2 * stage * sizeof(float);
}

template <int W>
void launch_batch_fused_t(int phase, dim3 grid, const BatchProblem* probs, const BatchTask* tasks,
                          int ntasks, int P, const WindowArgs& win, size_t lds,
                          hipStream_t stream) {
    static bool attr_set = false;      // dynamic LDS above 64 KB must be enabled per kernel
    if (!attr_set) {
        (void)hipFuncSetAttribute(reinterpret_cast<const void*>(&batch_spread_fused_kernel<W>),
                                  hipFuncAttributeMaxDynamicSharedMemorySize,
                                  kFuseMaxCells * (int)sizeof(int));
        (void)hipFuncSetAttribute(reinterpret_cast<const void*>(&batch_gather_fused_kernel<W>),
                                  hipFuncAttributeMaxDynamicSharedMemorySize,
                                  2 * kFuseMaxCells * (int)sizeof(float));
        attr_set = true;
    }
    if (phase == kBatchSpread)
        hipLaunchKernelGGL((batch_spread_fused_kernel<W>), grid, dim3(kSpreadBlock), lds, stream,
                           probs, tasks, ntasks, P, win);
    else
        hipLaunchKernelGGL((batch_gather_fused_kernel<W>), grid, dim3(kGatherBlock), lds, stream,
                           probs, tasks, ntasks, P, win);
}

hipError_t launch_batch_phase_fused(int phase, int W, const BatchProblem* probs,
                                    const BatchTask* tasks, int ntasks, int P,
                                    const WindowArgs& win, int* flag, int grid_blocks,
                                    size_t lds_bytes, hipStream_t stream) {
    if (ntasks <= 0) return hipSuccess;
    if (phase == kBatchProject) {
        hipLaunchKernelGGL(batch_split_kernel, dim3((unsigned)ntasks), dim3(kBlock), 0, stream,
                           probs, tasks, ntasks, flag);
        return hipGetLastError();
    }
    if (phase != kBatchSpread && phase != kBatchGather)
        return launch_batch_phase(phase, W, probs, tasks, ntasks, P, 8, win, flag, grid_blocks,
                                  lds_bytes, stream);
    const dim3 grid((unsigned)ntasks);
    switch (W) {
        case 4: launch_batch_fused_t<4>(phase, grid, probs, tasks, ntasks, P, win, lds_bytes, stream); break;
        case 6: launch_batch_fused_t<6>(phase, grid, probs, tasks, ntasks, P, win, lds_bytes, stream); break;
        case 8: launch_batch_fused_t<8>(phase, grid, probs, tasks, ntasks, P, win, lds_bytes, stream); break;
        default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

hipError_t launch_batch_phase(int phase, int W, const BatchProblem* probs,
                              const BatchTask* tasks, int ntasks, int P, int pstage,
                              const WindowArgs& win, int* flag, int grid_blocks,
                              size_t lds_bytes, hipStream_t stream) {
    if (ntasks <= 0) return hipSuccess;
    const dim3 grid((unsigned)(grid_blocks < ntasks ? grid_blocks : ntasks)), block(kBlock);
    switch (phase) {
        case kBatchProject:
            hipLaunchKernelGGL(batch_project_kernel, grid, block, 0, stream, probs, tasks, ntasks, P, flag);
            break;
        case kBatchScale:
            hipLaunchKernelGGL(batch_scale_kernel, grid, block, 0, stream, probs, tasks, ntasks);
            break;
        case kBatchSpread:
            switch (W) {
                case 4: hipLaunchKernelGGL(batch_spread_kernel<4>, grid, block, lds_bytes, stream, probs, tasks, ntasks, P, win); break;
                case 6: hipLaunchKernelGGL(batch_spread_kernel<6>, grid, block, lds_bytes, stream, probs, tasks, ntasks, P, win); break;
                case 8: hipLaunchKernelGGL(batch_spread_kernel<8>, grid, block, lds_bytes, stream, probs, tasks, ntasks, P, win); break;
                default: return hipErrorInvalidValue;
            }
            break;
        case kBatchFftconv:
            hipLaunchKernelGGL(batch_fftconv_kernel, grid, block, lds_bytes, stream, probs, tasks, ntasks, P);
            break;
        case kBatchGather:
            switch (W) {
                case 4: hipLaunchKernelGGL(batch_gather_kernel<4>, grid, block, lds_bytes, stream, probs, tasks, ntasks, P, pstage, win); break;
                case 6: hipLaunchKernelGGL(batch_gather_kernel<6>, grid, block, lds_bytes, stream, probs, tasks, ntasks, P, pstage, win); break;
                case 8: hipLaunchKernelGGL(batch_gather_kernel<8>, grid, block, lds_bytes, stream, probs, tasks, ntasks, P, pstage, win); break;
                default: return hipErrorInvalidValue;
            }
            break;
        case kBatchReduce:
            hipLaunchKernelGGL(batch_reduce_kernel, grid, block, 0, stream, probs, tasks, ntasks, P,
                               flag);
            break;
        default:
            return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

}  // namespace fastsum
