// Device kernels of the QMC-slicing fast summation on gfx950 (MI355X).
//
// Data flow of one summation (App. I Steps 1-3 applied per direction, then
// the average over directions of eq. kernel_sum_sliced):
//   project   x~ = tau <xi_p, x_n>  (P x N, direction-major)   MFMA GEMM
//   spread    u_p[j] = sum_n w_n phi(j - u(x~_{n,p}))             LDS atomics
//   fftconv   g_p = IDFT(mult . DFT(u_p))                         LDS FFT
//   gather    s_m = (1/P) sum_p sum_j g_p[j] phi(j - u(y~_{m,p}))  FP64 sum
// mult_k = c'_k / (n phihat_k)^2 folds the Fourier coefficients of the
// rescaled 1-D kernel and the window deconvolution into one table.
#include "fastsum_impl.h"

#include <hip/hip_runtime.h>

namespace fastsum {

typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef unsigned short u16x8 __attribute__((ext_vector_type(8)));

// ---------------------------------------------------------------------------
// window weights
// ---------------------------------------------------------------------------

template <int W> struct WinShape;
template <> struct WinShape<4> { static constexpr int NE = 3, NO = 2; };  // degree 4
template <> struct WinShape<6> { static constexpr int NE = 3, NO = 3; };  // degree 5
template <> struct WinShape<8> { static constexpr int NE = 4, NO = 4; };  // degree 7

template <int W>
__device__ __forceinline__ void window_weights(float sp, const WindowArgs& win,
                                               float (&wt)[W]) {
    constexpr int NE = WinShape<W>::NE, NO = WinShape<W>::NO;
    const float q = sp * sp;
#pragma unroll
    for (int t = 0; t < W / 2; ++t) {
        float e = win.even[t][NE - 1];
#pragma unroll
        for (int j = NE - 2; j >= 0; --j) e = fmaf(e, q, win.even[t][j]);
        float o = win.odd[t][NO - 1];
#pragma unroll
        for (int j = NO - 2; j >= 0; --j) o = fmaf(o, q, win.odd[t][j]);
        o *= sp;
        wt[t] = e + o;
        wt[W - 1 - t] = e - o;
    }
}

// Position of a rescaled projection in grid cells, clamped so that all W
// taps fall in [lo, lo + nr).  Returns the first tap relative to lo.
__device__ __forceinline__ int grid_position(float xt, const GridGeom& g,
                                             int half_w_m1, float& sp) {
    float u = fmaf(xt, (float)g.n, 0.5f * (float)g.n);
    u = fminf(fmaxf(u, g.u_min), g.u_max);   // NaN maps to u_min
    const float fl = floorf(u);
    sp = u - fl - 0.5f;
    return (int)fl - half_w_m1 - g.lo;
}

// ---------------------------------------------------------------------------
// projection: out[p][j] = sum_i A[p][i] X[j][i]   (MFMA 16x16x4 f32)
// ---------------------------------------------------------------------------

constexpr int kProjBM = 64;    // directions per workgroup tile
constexpr int kProjBN = 128;   // points per workgroup tile (32 per wave)
constexpr int kProjKC = 32;    // k-chunk staged in LDS (f32)

__global__ __launch_bounds__(kBlock) void project_f32_kernel(
    const float* __restrict__ X, int64_t N, int d, int dpad,
    const float* __restrict__ A, int P, float* __restrict__ out, int64_t ld,
    float bound, int* __restrict__ flag) {
    __shared__ float As[kProjBM][kProjKC + 1];
    __shared__ float Xs[kProjBN][kProjKC + 1];
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int p0 = blockIdx.y * kProjBM;
    const int64_t n0 = (int64_t)blockIdx.x * kProjBN;
    f32x4 acc[4][2];
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j) acc[i][j] = f32x4{0.f, 0.f, 0.f, 0.f};

    for (int k0 = 0; k0 < d; k0 += kProjKC) {
        const int kc = min(kProjKC, d - k0);
        __syncthreads();
        for (int e = tid; e < kProjBM * kProjKC; e += kBlock) {
            const int r = e / kProjKC, k = e % kProjKC;
            As[r][k] = (k < kc && p0 + r < P) ? A[(int64_t)(p0 + r) * dpad + k0 + k] : 0.f;
        }
        for (int e = tid; e < kProjBN * kProjKC; e += kBlock) {
            const int r = e / kProjKC, k = e % kProjKC;
            Xs[r][k] = (k < kc && n0 + r < N) ? X[(n0 + r) * d + k0 + k] : 0.f;
        }
        __syncthreads();
        for (int ks = 0; ks < kc; ks += 4) {
            float a[4], b[2];
#pragma unroll
            for (int bi = 0; bi < 4; ++bi) a[bi] = As[bi * 16 + (lane & 15)][ks + (lane >> 4)];
#pragma unroll
            for (int bj = 0; bj < 2; ++bj)
                b[bj] = Xs[wave * 32 + bj * 16 + (lane & 15)][ks + (lane >> 4)];
#pragma unroll
            for (int bi = 0; bi < 4; ++bi)
#pragma unroll
                for (int bj = 0; bj < 2; ++bj)
                    acc[bi][bj] = __builtin_amdgcn_mfma_f32_16x16x4f32(a[bi], b[bj], acc[bi][bj], 0, 0, 0);
        }
    }
    bool bad = false;
#pragma unroll
    for (int bi = 0; bi < 4; ++bi)
#pragma unroll
        for (int bj = 0; bj < 2; ++bj)
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int p = p0 + bi * 16 + 4 * (lane >> 4) + r;
                const int64_t n = n0 + wave * 32 + bj * 16 + (lane & 15);
                if (p < P && n < N) {
                    const float v = acc[bi][bj][r];
                    out[(int64_t)p * ld + n] = v;
                    bad |= !(fabsf(v) <= bound);
                }
            }
    if (bad) atomicOr(flag, 1);
}

__device__ __forceinline__ unsigned short f32_to_bf16_rne(float f) {
    unsigned int u = __float_as_uint(f);
    if ((u & 0x7f800000u) == 0x7f800000u)          // inf / nan: keep, quiet nan
        return (unsigned short)((u >> 16) | ((u & 0xffffu) ? 0x40u : 0u));
    u += 0x7fffu + ((u >> 16) & 1u);
    return (unsigned short)(u >> 16);
}

constexpr int kProjKCh = 64;   // k-chunk staged in LDS (bf16)

__global__ __launch_bounds__(kBlock) void project_bf16_kernel(
    const float* __restrict__ X, int64_t N, int d, int dpad,
    const unsigned short* __restrict__ A, int P, float* __restrict__ out,
    int64_t ld, float bound, int* __restrict__ flag) {
    // row stride 72 halves = 144 bytes keeps 16-byte fragment loads aligned
    __shared__ __attribute__((aligned(16))) unsigned short As[kProjBM][kProjKCh + 8];
    __shared__ __attribute__((aligned(16))) unsigned short Xs[kProjBN][kProjKCh + 8];
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int p0 = blockIdx.y * kProjBM;
    const int64_t n0 = (int64_t)blockIdx.x * kProjBN;
    f32x4 acc[4][2];
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j) acc[i][j] = f32x4{0.f, 0.f, 0.f, 0.f};

    for (int k0 = 0; k0 < d; k0 += kProjKCh) {
        const int kc = min(kProjKCh, d - k0);
        __syncthreads();
        for (int e = tid; e < kProjBM * kProjKCh; e += kBlock) {
            const int r = e / kProjKCh, k = e % kProjKCh;
            As[r][k] = (k < kc && p0 + r < P) ? A[(int64_t)(p0 + r) * dpad + k0 + k] : (unsigned short)0;
        }
        for (int e = tid; e < kProjBN * kProjKCh; e += kBlock) {
            const int r = e / kProjKCh, k = e % kProjKCh;
            Xs[r][k] = (k < kc && n0 + r < N) ? f32_to_bf16_rne(X[(n0 + r) * d + k0 + k]) : (unsigned short)0;
        }
        __syncthreads();
        for (int ks = 0; ks < kc; ks += 32) {
            bf16x8 a[4], b[2];
            const int kk = ks + 8 * (lane >> 4);
#pragma unroll
            for (int bi = 0; bi < 4; ++bi)
                a[bi] = __builtin_bit_cast(bf16x8, *reinterpret_cast<const u16x8*>(&As[bi * 16 + (lane & 15)][kk]));
#pragma unroll
            for (int bj = 0; bj < 2; ++bj)
                b[bj] = __builtin_bit_cast(bf16x8, *reinterpret_cast<const u16x8*>(&Xs[wave * 32 + bj * 16 + (lane & 15)][kk]));
#pragma unroll
            for (int bi = 0; bi < 4; ++bi)
#pragma unroll
                for (int bj = 0; bj < 2; ++bj)
                    acc[bi][bj] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[bi], b[bj], acc[bi][bj], 0, 0, 0);
        }
    }
    bool bad = false;
#pragma unroll
    for (int bi = 0; bi < 4; ++bi)
#pragma unroll
        for (int bj = 0; bj < 2; ++bj)
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int p = p0 + bi * 16 + 4 * (lane >> 4) + r;
                const int64_t n = n0 + wave * 32 + bj * 16 + (lane & 15);
                if (p < P && n < N) {
                    const float v = acc[bi][bj][r];
                    out[(int64_t)p * ld + n] = v;
                    bad |= !(fabsf(v) <= bound);
                }
            }
    if (bad) atomicOr(flag, 1);
}

hipError_t launch_project_f32(const float* X, int64_t N, int d, int dpad,
                              const float* A, int P, float* out, int64_t ld,
                              float bound, int* flag, hipStream_t stream) {
    dim3 grid((unsigned)((N + kProjBN - 1) / kProjBN), (unsigned)((P + kProjBM - 1) / kProjBM));
    hipLaunchKernelGGL(project_f32_kernel, grid, dim3(kBlock), 0, stream, X, N, d,
                       dpad, A, P, out, ld, bound, flag);
    return hipGetLastError();
}

hipError_t launch_project_bf16(const float* X, int64_t N, int d, int dpad,
                               const uint16_t* A, int P, float* out, int64_t ld,
                               float bound, int* flag, hipStream_t stream) {
    dim3 grid((unsigned)((N + kProjBN - 1) / kProjBN), (unsigned)((P + kProjBM - 1) / kProjBM));
    hipLaunchKernelGGL(project_bf16_kernel, grid, dim3(kBlock), 0, stream, X, N, d,
                       dpad, reinterpret_cast<const unsigned short*>(A), P, out,
                       ld, bound, flag);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// spread: one workgroup = one direction x one chunk of sources
// ---------------------------------------------------------------------------

template <int W>
__global__ __launch_bounds__(kBlock) void spread_kernel(
    const float* __restrict__ proj, int64_t ld, const float* __restrict__ w,
    int64_t N, int P, GridGeom g, int64_t chunk_len, WindowArgs win,
    float* __restrict__ partial) {
    extern __shared__ float lds[];
    const int p = blockIdx.x;
    const int c = blockIdx.y;
    for (int j = threadIdx.x; j < g.nr; j += kBlock) lds[j] = 0.f;
    __syncthreads();
    const int64_t i0 = (int64_t)c * chunk_len;
    const int64_t i1 = min(N, i0 + chunk_len);
    const float* __restrict__ row = proj + (int64_t)p * ld;
#pragma unroll 4
    for (int64_t i = i0 + threadIdx.x; i < i1; i += kBlock) {
        float sp;
        const int base = grid_position(row[i], g, W / 2 - 1, sp);
        float wt[W];
        window_weights<W>(sp, win, wt);
        const float wi = w[i];
#pragma unroll
        for (int t = 0; t < W; ++t) atomicAdd(&lds[base + t], wi * wt[t]);
    }
    __syncthreads();
    float* __restrict__ dst = partial + ((int64_t)c * P + p) * g.nr;
    for (int j = threadIdx.x; j < g.nr; j += kBlock) dst[j] = lds[j];
}

hipError_t launch_spread(int W, const float* proj, int64_t ld, const float* w,
                         int64_t N, int P, GridGeom g, int nchunk,
                         int64_t chunk_len, const WindowArgs& win,
                         float* partial, hipStream_t stream) {
    dim3 grid((unsigned)P, (unsigned)nchunk);
    const size_t lds = (size_t)g.nr * sizeof(float);
    switch (W) {
        case 4: hipLaunchKernelGGL(spread_kernel<4>, grid, dim3(kBlock), lds, stream, proj, ld, w, N, P, g, chunk_len, win, partial); break;
        case 6: hipLaunchKernelGGL(spread_kernel<6>, grid, dim3(kBlock), lds, stream, proj, ld, w, N, P, g, chunk_len, win, partial); break;
        case 8: hipLaunchKernelGGL(spread_kernel<8>, grid, dim3(kBlock), lds, stream, proj, ld, w, N, P, g, chunk_len, win, partial); break;
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

// Stockham autosort FFT of length n (power of two) in LDS, radix-4 stages
// and one radix-2 stage when log2(n) is odd.  tw[m] = exp(-2 pi i m / n).
// Forward: X_k = sum_j x_j e^{-2 pi i jk/n}; inverse: conjugate kernel, no
// 1/n.  Returns the buffer holding the result (a or b).
__device__ float2* fft_lds(float2* a, float2* b, int n, const float2* __restrict__ tw,
                           bool inverse) {
    const float sgn = inverse ? -1.f : 1.f;
    for (int Ls = 1; Ls < n;) {
        const int r = (n / Ls >= 4) ? 4 : 2;
        const int nb = n / r;
        const int stride = n / (Ls * r);
        for (int j = threadIdx.x; j < nb; j += kBlock) {
            const int k = j & (Ls - 1);
            const int base = (j - k) * r + k;
            if (r == 4) {
                float2 a0 = a[j], a1 = a[j + nb], a2 = a[j + 2 * nb], a3 = a[j + 3 * nb];
                if (k) {
                    float2 w1 = tw[k * stride], w2 = tw[2 * k * stride], w3 = tw[3 * k * stride];
                    w1.y *= sgn; w2.y *= sgn; w3.y *= sgn;
                    a1 = cmul(a1, w1); a2 = cmul(a2, w2); a3 = cmul(a3, w3);
                }
                const float2 t0 = cadd(a0, a2), t1 = csub(a0, a2), t2 = cadd(a1, a3);
                const float2 d13 = csub(a1, a3);
                // forward: times -i ; inverse: times +i
                const float2 t3 = make_float2(sgn * d13.y, -sgn * d13.x);
                b[base] = cadd(t0, t2);
                b[base + Ls] = cadd(t1, t3);
                b[base + 2 * Ls] = csub(t0, t2);
                b[base + 3 * Ls] = csub(t1, t3);
            } else {
                float2 a0 = a[j], a1 = a[j + nb];
                if (k) {
                    float2 w1 = tw[k * stride];
                    w1.y *= sgn;
                    a1 = cmul(a1, w1);
                }
                b[base] = cadd(a0, a1);
                b[base + Ls] = csub(a0, a1);
            }
        }
        __syncthreads();
        float2* t = a; a = b; b = t;
        Ls *= r;
    }
    return a;
}

__global__ __launch_bounds__(kBlock) void fftconv_kernel(
    const float* __restrict__ partial, int nchunk, int P, GridGeom g,
    const float2* __restrict__ tw, const float2* __restrict__ mult,
    const float2* __restrict__ mult_d, float* __restrict__ grid,
    float* __restrict__ grid_d) {
    extern __shared__ float2 cbuf[];
    const int n = g.n;
    float2* b0 = cbuf;
    float2* b1 = cbuf + n;
    float2* b2 = cbuf + 2 * n;
    const int pa = 2 * blockIdx.x, pb = pa + 1;
    const bool has_b = pb < P;
    for (int j = threadIdx.x; j < n; j += kBlock) {
        float re = 0.f, im = 0.f;
        const int r = j - g.lo;
        if (r >= 0 && r < g.nr) {
            for (int c = 0; c < nchunk; ++c) {
                re += partial[((int64_t)c * P + pa) * g.nr + r];
                if (has_b) im += partial[((int64_t)c * P + pb) * g.nr + r];
            }
        }
        b0[j] = make_float2(re, im);
    }
    __syncthreads();
    float2* spec = fft_lds(b0, b1, n, tw, false);
    float2* wa = (spec == b0) ? b1 : b0;
    const int passes = grid_d ? 2 : 1;
    for (int pass = 0; pass < passes; ++pass) {
        const float2* __restrict__ m = pass ? mult_d : mult;
        float* __restrict__ out = pass ? grid_d : grid;
        for (int j = threadIdx.x; j < n; j += kBlock) wa[j] = cmul(spec[j], m[j]);
        __syncthreads();
        const float2* res = fft_lds(wa, b2, n, tw, true);
        for (int r = threadIdx.x; r < g.nr; r += kBlock) {
            const float2 v = res[g.lo + r];
            out[(int64_t)pa * g.nr + r] = v.x;
            if (has_b) out[(int64_t)pb * g.nr + r] = v.y;
        }
        __syncthreads();
    }
}

hipError_t launch_fftconv(const float* partial, int nchunk, int P, GridGeom g,
                          const float2* tw, const float2* mult,
                          const float2* mult_d, float* grid, float* grid_d,
                          hipStream_t stream) {
    dim3 grid_dim((unsigned)((P + 1) / 2));
    const size_t lds = (size_t)3 * g.n * sizeof(float2);
    hipLaunchKernelGGL(fftconv_kernel, grid_dim, dim3(kBlock), lds, stream, partial,
                       nchunk, P, g, tw, mult, mult_d, grid, grid_d);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// gather: one workgroup = a tile of targets x a group of directions
// ---------------------------------------------------------------------------

constexpr int kGatherTPT = 4;   // targets per thread

template <int W, bool WRITE_T>
__global__ __launch_bounds__(kBlock) void gather_kernel(
    const float* __restrict__ proj, int64_t ld, int64_t M, int P, GridGeom g,
    const float* __restrict__ grid, int pg, int pstage, WindowArgs win,
    double* __restrict__ spart, int64_t ldm, float* __restrict__ tout,
    int64_t ld_t) {
    extern __shared__ float lds[];
    const int tid = threadIdx.x;
    const int64_t m0 = (int64_t)blockIdx.x * (kBlock * kGatherTPT);
    const int p_begin = blockIdx.y * pg;
    const int p_end = min(P, p_begin + pg);
    double acc[kGatherTPT];
#pragma unroll
    for (int s = 0; s < kGatherTPT; ++s) acc[s] = 0.0;
    for (int ps = p_begin; ps < p_end; ps += pstage) {
        const int np = min(pstage, p_end - ps);
        __syncthreads();
        const float* __restrict__ src = grid + (int64_t)ps * g.nr;
        for (int j = tid; j < np * g.nr; j += kBlock) lds[j] = src[j];
        __syncthreads();
        for (int pp = 0; pp < np; ++pp) {
            const float* __restrict__ row = proj + (int64_t)(ps + pp) * ld;
            const float* gl = lds + pp * g.nr;
#pragma unroll
            for (int s = 0; s < kGatherTPT; ++s) {
                const int64_t m = m0 + s * kBlock + tid;
                if (m < M) {
                    float sp;
                    const int base = grid_position(row[m], g, W / 2 - 1, sp);
                    float wt[W];
                    window_weights<W>(sp, win, wt);
                    float t = 0.f;
#pragma unroll
                    for (int k = 0; k < W; ++k) t = fmaf(gl[base + k], wt[k], t);
                    if (WRITE_T)
                        tout[(int64_t)(ps + pp) * ld_t + m] = t;
                    else
                        acc[s] += (double)t;
                }
            }
        }
    }
    if (!WRITE_T) {
#pragma unroll
        for (int s = 0; s < kGatherTPT; ++s) {
            const int64_t m = m0 + s * kBlock + tid;
            if (m < M) spart[(int64_t)blockIdx.y * ldm + m] = acc[s];
        }
    }
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

__global__ __launch_bounds__(kBlock) void reduce_kernel(
    const double* __restrict__ spart, int nb, int64_t ldm, int64_t M,
    double scale, float* __restrict__ s) {
    const int64_t m = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (m >= M) return;
    double acc = 0.0;
    for (int b = 0; b < nb; ++b) acc += spart[(int64_t)b * ldm + m];
    s[m] = (float)(acc * scale);
}

hipError_t launch_reduce(const double* spart, int nb, int64_t ldm, int64_t M,
                         double scale, float* s, hipStream_t stream) {
    dim3 grid((unsigned)((M + kBlock - 1) / kBlock));
    hipLaunchKernelGGL(reduce_kernel, grid, dim3(kBlock), 0, stream, spart, nb, ldm, M, scale, s);
    return hipGetLastError();
}

constexpr int kBpDim = 32;    // dimensions per pass
constexpr int kBpP = 64;      // directions staged per LDS pass

// grad_y[m][i] = v[m] * coef * sum_p tprime[p][m] * A[p][i]   (A = tau Xi^T)
__global__ __launch_bounds__(kBlock) void backproject_kernel(
    const float* __restrict__ tprime, int64_t ld, int64_t M, int P, int d,
    const float* __restrict__ A, int dpad, float coef,
    const float* __restrict__ v, float* __restrict__ grad_y) {
    __shared__ float xs[kBpP][kBpDim];
    const int64_t m = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    const int i0 = blockIdx.y * kBpDim;
    float acc[kBpDim];
#pragma unroll
    for (int i = 0; i < kBpDim; ++i) acc[i] = 0.f;
    for (int p0 = 0; p0 < P; p0 += kBpP) {
        __syncthreads();
        for (int e = threadIdx.x; e < kBpP * kBpDim; e += kBlock) {
            const int pp = e / kBpDim, ii = e % kBpDim;
            xs[pp][ii] = (p0 + pp < P && i0 + ii < d) ? A[(int64_t)(p0 + pp) * dpad + i0 + ii] : 0.f;
        }
        __syncthreads();
        if (m < M) {
            const int np = min(kBpP, P - p0);
            for (int pp = 0; pp < np; ++pp) {
                const float t = tprime[(int64_t)(p0 + pp) * ld + m];
#pragma unroll
                for (int i = 0; i < kBpDim; ++i) acc[i] = fmaf(t, xs[pp][i], acc[i]);
            }
        }
    }
    if (m < M) {
        const float sv = v[m] * coef;
#pragma unroll
        for (int i = 0; i < kBpDim; ++i)
            if (i0 + i < d) grad_y[m * d + i0 + i] = sv * acc[i];
    }
}

hipError_t launch_backproject(const float* tprime, int64_t ld, int64_t M,
                              int P, int d, const float* A, int dpad, float coef,
                              const float* v, float* grad_y, hipStream_t stream) {
    dim3 grid((unsigned)((M + kBlock - 1) / kBlock), (unsigned)((d + kBpDim - 1) / kBpDim));
    hipLaunchKernelGGL(backproject_kernel, grid, dim3(kBlock), 0, stream, tprime, ld, M,
                       P, d, A, dpad, coef, v, grad_y);
    return hipGetLastError();
}

}  // namespace fastsum
