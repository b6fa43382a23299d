// Stored projections for any d: the tile GEMM of the projection step
// (x~_{n,p} = tau <xi_p, x_n>, App. I Step 1 applied to every direction),
// out[p * ld + n] = pscale * sum_k A[p][k] X[n][k] on MFMA, both operands
// in the split tile layout (16 rows x 32 columns per 1 KB part).
//
// PARTS parts per k-block: 2 = f16 hi + lo (three v_mfma_f32_16x16x32_f16
// per tile pair, hi*lo + lo*hi before hi*hi: FP32-level products), 1 = BF16
// (one v_mfma_f32_16x16x32_bf16, BF16 inputs with FP32 accumulation).
//
// A workgroup is eight waves, two per SIMD, in a WD x WP grid; each wave
// owns TD direction tiles x TP point tiles of the output (TD TP 16 x 16
// FP32 accumulators in registers).  Large workgroup tiles keep the operand
// traffic from L2 low (each operand tile is loaded once per workgroup) and
// large wave tiles keep the LDS reads per MFMA low: per k-block a wave reads
// (TD + TP) PARTS KB of operands for TD TP PARTS MFMAs.  The k-blocks stream
// through NBUF LDS buffers filled by LDS-direct loads (one 1 KB tile part
// per wave instruction) NBUF - 1 k-blocks ahead of the MFMAs, and each wave
// reads the operands of k-block kb + 1 from LDS into a second register set
// while the MFMAs of kb run, so neither the memory latency nor the LDS
// reads sit between MFMAs.  16 x 16 x 32 MFMAs: the 32 x 32 x 16 forms,
// with the same operands read in another lane order, measured no faster
// here (the kernel is bound by operand delivery, not MFMA issue).
#include "fastsum_impl.h"
#include "device_common.h"

#include <hip/hip_runtime.h>

#include <algorithm>

namespace fastsum {

namespace {

// Workgroup shape per operand form: WD x WP waves, each owning TD direction
// tiles x TP point tiles (16 rows each); NBUF k-block buffers in LDS, loads
// NBUF - 1 k-blocks ahead of the MFMAs; at most 256 registers per lane
// (two waves per SIMD).
template <int PARTS> struct GemmShape;
template <> struct GemmShape<1> {        // BF16: 256 directions x 256 points, 96 KB LDS
    static constexpr int TD = 8, TP = 4, WD = 2, WP = 4, NBUF = 3;
};
template <> struct GemmShape<2> {        // f16 hi + lo: 256 directions x 128 points, 144 KB LDS
    static constexpr int TD = 4, TP = 4, WD = 4, WP = 2, NBUF = 3;
};

template <int PARTS> struct GemmGeom {
    using S = GemmShape<PARTS>;
    static constexpr int kWaves = S::WD * S::WP;
    static constexpr int kThreads = 64 * kWaves;
    static constexpr int kDT = S::WD * S::TD;                  // direction tiles per workgroup
    static constexpr int kPT = S::WP * S::TP;                  // point tiles per workgroup
    static constexpr int kPieces = (kDT + kPT) * PARTS;        // 1 KB parts per k-block
    static constexpr int kPerWave = kPieces / kWaves;
    static constexpr int kBufBytes = kPieces * kSplitTileBytes;
    static constexpr int kLdsBytes = S::NBUF * kBufBytes;
    static_assert(kPieces % kWaves == 0, "pieces split evenly over the waves");
    static_assert(kLdsBytes <= 160 * 1024, "LDS of one CU");
};

// s_waitcnt vmcnt(N) lgkmcnt(0) (gfx9 encoding: vmcnt in bits 3:0 and
// 15:14, expcnt 6:4 left at its maximum, lgkmcnt 11:8): this wave's loads
// but the last N have landed and its LDS reads are done
template <int N> __device__ __forceinline__ void wait_vm_lgkm0() {
    static_assert(N >= 0 && N < 64, "vmcnt range");
    asm volatile("" ::: "memory");
    __builtin_amdgcn_s_waitcnt((N & 15) | (7 << 4) | ((N >> 4) << 14));
    asm volatile("" ::: "memory");
}

// wait until at most `ahead` k-blocks of this wave's loads (kPerWave each)
// are in flight (ahead <= 2)
template <int kPerWave> __device__ __forceinline__ void wait_blocks_ahead(int ahead) {
    if (ahead >= 2) wait_vm_lgkm0<2 * kPerWave>();
    else if (ahead == 1) wait_vm_lgkm0<kPerWave>();
    else wait_vm_lgkm0<0>();
}

// A bare s_barrier: __syncthreads() would also wait for the loads still in
// flight.
__device__ __forceinline__ void bare_barrier() {
    asm volatile("" ::: "memory");
    __builtin_amdgcn_s_barrier();
    asm volatile("" ::: "memory");
}

// LDS-direct loads of k-block kb into buf: this wave's pieces wave + W u,
// one 1 KB tile part each, from src[u] (the part's k-block 0).  A device
// function rather than a lambda in the kernel: the host pass does not
// instantiate a kernel template whose body calls this builtin directly
// from a nested lambda.
template <int kPerWave, int kWaves, int64_t kKbBytes>
__device__ __forceinline__ void gemm_stage(const char* const (&src)[kPerWave], char* buf, int kb,
                                           int wave, int lane) {
#pragma unroll
    for (int u = 0; u < kPerWave; ++u)
        __builtin_amdgcn_global_load_lds(src[u] + kb * kKbBytes + lane * 16,
                                         (lds_void*)(buf + (wave + kWaves * u) * kSplitTileBytes),
                                         16, 0, 0);
}

template <int PARTS>
__global__ __launch_bounds__(GemmGeom<PARTS>::kThreads) __attribute__((amdgpu_waves_per_eu(2, 2)))
void project_tiles_kernel(const uint16_t* __restrict__ Xt, int64_t N,
                          const uint16_t* __restrict__ At, int P, int KB, float pscale,
                          const float* __restrict__ row_scale, const float* __restrict__ gscale,
                          float* __restrict__ out, int64_t ld, int64_t ncols, float bound,
                          int* __restrict__ flag, int ndb, int npb) {
    using S = GemmShape<PARTS>;
    using G = GemmGeom<PARTS>;
    constexpr int TD = S::TD, TP = S::TP, NBUF = S::NBUF;
    constexpr int kDT = G::kDT, kWaves = G::kWaves, kPerWave = G::kPerWave;
    constexpr int64_t kKbBytes = (int64_t)PARTS * kSplitTileBytes;   // one k-block of a tile
    extern __shared__ __attribute__((aligned(16))) char gsm[];
    const int lane = threadIdx.x & 63;
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    int db, pb;
    if (!proj_tile_of_block(blockIdx.x, ndb, npb, db, pb)) return;
    const int64_t dt0 = (int64_t)db * kDT, pt0 = (int64_t)pb * G::kPT;
    const int64_t ndtiles = (P + 15) / 16, nptiles = (N + 15) / 16;

    // pieces wave + W u (u < kPerWave, W waves): tile t = piece / PARTS
    // (direction tiles first), part piece % PARTS; tiles past the ends
    // re-read the last tile (their results are not stored)
    const char* src[kPerWave];
#pragma unroll
    for (int u = 0; u < kPerWave; ++u) {
        const int piece = wave + kWaves * u;
        const int t = piece / PARTS, q = piece - t * PARTS;
        const bool is_dir = t < kDT;
        const int64_t tile = is_dir ? min(dt0 + t, ndtiles - 1) : min(pt0 + t - kDT, nptiles - 1);
        src[u] = reinterpret_cast<const char*>(is_dir ? At : Xt) +
                 (tile * KB * PARTS + q) * kSplitTileBytes;
    }
    auto buf_of = [&](int kb) { return gsm + (kb % NBUF) * G::kBufBytes; };
    auto stage = [&](int kb) {
        gemm_stage<kPerWave, kWaves, kKbBytes>(src, buf_of(kb), kb, wave, lane);
    };

    // this wave: direction tiles wd .. wd + TD - 1, point tiles wp .. wp + TP - 1
    // (workgroup-relative); a wave whose tiles are all past the ends still
    // runs its MFMAs (on re-read tiles) and stores nothing
    const int wd = TD * (wave % S::WD), wp = TP * (wave / S::WD);
    typedef h8 Ops[TD + TP][PARTS];
    auto read_ops = [&](const char* buf, Ops& o) {
#pragma unroll
        for (int i = 0; i < TD; ++i)
#pragma unroll
            for (int q = 0; q < PARTS; ++q)
                o[i][q] = *reinterpret_cast<const h8*>(
                    buf + ((wd + i) * PARTS + q) * kSplitTileBytes + lane * 16);
#pragma unroll
        for (int j = 0; j < TP; ++j)
#pragma unroll
            for (int q = 0; q < PARTS; ++q)
                o[TD + j][q] = *reinterpret_cast<const h8*>(
                    buf + ((kDT + wp + j) * PARTS + q) * kSplitTileBytes + lane * 16);
    };
    // C[point][dir]: lane (c, r) of acc[i][j] holds points 4r .. 4r+3 of
    // direction c
    f32x4 acc[TD][TP];
#pragma unroll
    for (int i = 0; i < TD; ++i)
#pragma unroll
        for (int j = 0; j < TP; ++j) acc[i][j] = f32x4{0.f, 0.f, 0.f, 0.f};
    auto mfma = [&](const Ops& o) {
        if constexpr (PARTS == 2) {
#pragma unroll
            for (int i = 0; i < TD; ++i)
#pragma unroll
                for (int j = 0; j < TP; ++j) {
                    acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_f16(o[TD + j][0], o[i][1], acc[i][j], 0, 0, 0);
                    acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_f16(o[TD + j][1], o[i][0], acc[i][j], 0, 0, 0);
                }
#pragma unroll
            for (int i = 0; i < TD; ++i)
#pragma unroll
                for (int j = 0; j < TP; ++j)
                    acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_f16(o[TD + j][0], o[i][0], acc[i][j], 0, 0, 0);
        } else {
#pragma unroll
            for (int i = 0; i < TD; ++i)
#pragma unroll
                for (int j = 0; j < TP; ++j)
                    acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(
                        __builtin_bit_cast(bf16x8, o[TD + j][0]), __builtin_bit_cast(bf16x8, o[i][0]),
                        acc[i][j], 0, 0, 0);
        }
    };
    // One k-block: make k-block kb + 1 visible to every wave (k-blocks up to
    // kb + NBUF - 1 have been issued), refill the buffer of kb (read into
    // registers in the previous step) with kb + NBUF, read kb + 1 into
    // `nxt`, then the MFMAs of kb from `cur`.
    auto step = [&](int kb, const Ops& cur, Ops& nxt) {
        if (kb + 1 < KB) {
            wait_blocks_ahead<kPerWave>(min(KB - 1, kb + NBUF - 1) - (kb + 1));
            bare_barrier();
            if (kb + NBUF < KB) stage(kb + NBUF);
            read_ops(buf_of(kb + 1), nxt);
        }
        mfma(cur);
    };

    Ops ra, rb;
#pragma unroll
    for (int k = 0; k < NBUF - 1; ++k)
        if (k < KB) stage(k);
    wait_blocks_ahead<kPerWave>(min(KB - 1, NBUF - 2));
    bare_barrier();
    if (NBUF - 1 < KB) stage(NBUF - 1);
    read_ops(buf_of(0), ra);
    for (int kb = 0; kb < KB; kb += 2) {
        step(kb, ra, rb);
        if (kb + 1 < KB) step(kb + 1, rb, ra);
    }
    if (dt0 + wd >= ndtiles || pt0 + wp >= nptiles) return;

    // out row p, column n: pscale (* gscale[0]) (* row_scale[p]) times the
    // product; columns n >= ncols are not stored
    const int c = lane & 15, r = lane >> 4;
    const float gs = gscale != nullptr ? pscale * gscale[0] : pscale;
    const bool vec4 = ((ncols | ld) & 3) == 0;
    bool bad = false;
#pragma unroll
    for (int i = 0; i < TD; ++i) {
        const int64_t p = (dt0 + wd + i) * 16 + c;
        if (p >= P) continue;
        const float rs = row_scale != nullptr ? gs * row_scale[p] : gs;
        float* __restrict__ orow = out + p * ld;
#pragma unroll
        for (int j = 0; j < TP; ++j) {
            const int64_t n = (pt0 + wp + j) * 16 + 4 * r;
            if (n >= ncols) continue;
            const f32x4 v = acc[i][j] * rs;
            if (vec4) {
                *reinterpret_cast<float4*>(orow + n) = make_float4(v[0], v[1], v[2], v[3]);
            } else {
#pragma unroll
                for (int e = 0; e < 4; ++e)
                    if (n + e < ncols) orow[n + e] = v[e];
            }
#pragma unroll
            for (int e = 0; e < 4; ++e) bad |= !(fabsf(v[e]) <= bound);
        }
    }
    if (bad && flag != nullptr) atomicOr(flag, 1);
}

// BF16 point tiles (one part per k-block): bf16(Z) in the tile layout; the
// largest |Z_row * inv_r|^2 into *norm_slot (nullable, see BoundCheck)
__global__ __launch_bounds__(kBlock) void bf16_points_kernel(
    const float* __restrict__ Z, int64_t N, int d, int KB, int64_t ntiles, u32x4* __restrict__ tiles,
    float inv_r, unsigned* __restrict__ norm_slot) {
    const int64_t id = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (id >= ntiles * 64) return;                    // whole waves
    const int lane = (int)(id & 63);
    const int64_t t = id >> 6, r0 = 16 * t;
    const int64_t nrows = N - r0 < 16 ? N - r0 : 16;
    const __amdgpu_buffer_rsrc_t zs = buffer_rsrc(Z + r0 * d, nrows * (int64_t)d * 4);
    float ss = 0.f;
    for (int kb = 0; kb < KB; ++kb) {
        const int col0 = 32 * kb + 8 * (lane >> 4);
        const int off = ((lane & 15) * d + col0) * 4;
        const u32x4 va = __builtin_amdgcn_raw_buffer_load_b128(zs, off, 0, 0);
        const u32x4 vb = __builtin_amdgcn_raw_buffer_load_b128(zs, off + 16, 0, 0);
        float v[8];
#pragma unroll
        for (int e = 0; e < 8; ++e) {
            v[e] = col0 + e < d ? __uint_as_float(e < 4 ? va[e] : vb[e - 4]) : 0.f;
            const float vs = v[e] * inv_r;
            ss = fmaf(vs, vs, ss);
        }
        tiles[(t * KB + kb) * 64 + lane] = u32x4{pack_bf16x2(v[0], v[1]), pack_bf16x2(v[2], v[3]),
                                                 pack_bf16x2(v[4], v[5]), pack_bf16x2(v[6], v[7])};
    }
    ss += __shfl_xor(ss, 16);
    ss += __shfl_xor(ss, 32);
    if (norm_slot != nullptr) record_norm2(norm_slot, ss);
}

template <int PARTS>
hipError_t launch_gemm(const uint16_t* Xt, int64_t N, const uint16_t* At, int P, int KB,
                       float pscale, const float* row_scale, const float* gscale, float* out,
                       int64_t ld, int64_t ncols, float bound, int* flag, hipStream_t stream) {
    using G = GemmGeom<PARTS>;
    static bool attr_set = false;      // dynamic LDS above 64 KB must be enabled per kernel
    if (!attr_set) {
        (void)hipFuncSetAttribute(reinterpret_cast<const void*>(&project_tiles_kernel<PARTS>),
                                  hipFuncAttributeMaxDynamicSharedMemorySize, G::kLdsBytes);
        attr_set = true;
    }
    const int ndb = (P + 16 * G::kDT - 1) / (16 * G::kDT);
    const int npb = (int)((N + 16 * G::kPT - 1) / (16 * G::kPT));
    hipLaunchKernelGGL(project_tiles_kernel<PARTS>, dim3(proj_grid_blocks(ndb, npb)),
                       dim3(G::kThreads), G::kLdsBytes, stream, Xt, N, At, P, KB, pscale,
                       row_scale, gscale, out, ld, ncols, bound, flag, ndb, npb);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Back-projection on the tile GEMM (any d, used above the fused range):
//   grad[m][i] = coef v[m] sum_p T[p][m] (tau xi_p)_i,
// the chain rule through x~_{m,p} = tau <xi_p, y_m> (eq. kernel_sum_sliced
// differentiated in y_m), T[p][m] the derivative of the 1-D sum of
// direction p at target m.  T (P x M, row stride ld) becomes split-f16 tiles
// with rows m and columns p, scaled by 2^-e so that max |T| 2^-e < 1 (the
// f16 parts then keep FP32-level accuracy relative to the largest entry);
// xi^T is a split tile operand with rows i and columns p (built once per
// plan); the GEMM's epilogue applies coef v[m] tau 2^e.
// ---------------------------------------------------------------------------

constexpr int kAbsSlots = 64;
constexpr int kAbsStride = 16;                     // one 64-byte line per slot

__global__ __launch_bounds__(kBlock) void clear_slots_kernel(unsigned* __restrict__ slots) {
    for (int j = threadIdx.x; j < kAbsSlots * kAbsStride; j += kBlock) slots[j] = 0u;
}

// largest |T[p][m]| (p < P, m < M) as float bits into the slots (a
// non-finite entry records +inf); workgroup (x, y) walks rows y + k gridDim.y
__global__ __launch_bounds__(kBlock) void abs_max_kernel(const float* __restrict__ T, int64_t ld,
                                                         int P, int64_t M,
                                                         unsigned* __restrict__ slots) {
    float mx = 0.f;
    for (int p = blockIdx.y; p < P; p += gridDim.y) {
        const float* __restrict__ row = T + (int64_t)p * ld;
        for (int64_t m = (int64_t)blockIdx.x * kBlock + threadIdx.x; m < M;
             m += (int64_t)gridDim.x * kBlock) {
            const float a = fabsf(row[m]);
            mx = (a <= 3.4e38f) ? fmaxf(mx, a) : __builtin_inff();
        }
    }
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) mx = fmaxf(mx, __shfl_xor(mx, o));
    const int b = blockIdx.x + gridDim.x * blockIdx.y;
    if ((threadIdx.x & 63) == 0) atomicMax(slots + (b % kAbsSlots) * kAbsStride, __float_as_uint(mx));
}

// e with max 2^-e < 1 from the slots (0 for an all-zero or non-finite T)
__device__ __forceinline__ int slots_exponent(const unsigned* __restrict__ slots, int lane) {
    float mx = __uint_as_float(slots[lane * kAbsStride]);      // 64 lanes, 64 slots
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) mx = fmaxf(mx, __shfl_xor(mx, o));
    int e = 0;
    if (mx > 0.f && mx <= 3.4e38f) (void)frexpf(mx, &e);     // mx < 2^e
    return e;
}

// Split tiles of T^T: tile t (rows m = 16 t + c), k-block kb (columns
// p = 32 kb + 8 j + q), lane c + 16 j; one wave per (tile, k-block).  Entry
// 0 of gscale_out receives tau 2^e.
__global__ __launch_bounds__(kBlock) void split_cols_kernel(
    const float* __restrict__ T, int64_t ld, int P, int64_t M, int KB, int64_t ntiles,
    const unsigned* __restrict__ slots, float tau, u32x4* __restrict__ tiles,
    float* __restrict__ gscale_out) {
    const int64_t id = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (id >= ntiles * KB * 64) return;               // whole waves
    const int lane = (int)(id & 63);
    const int64_t w = id >> 6;
    const int64_t t = w / KB;
    const int kb = (int)(w - t * KB);
    const int e = slots_exponent(slots, lane);
    const float s = ldexpf(1.f, -e);
    if (id == 0) gscale_out[0] = ldexpf(tau, e);
    const int64_t m = 16 * t + (lane & 15);
    const int p0 = 32 * kb + 8 * (lane >> 4);
    h8 hi, lo;
#pragma unroll
    for (int q = 0; q < 8; ++q) {
        const float v = (m < M && p0 + q < P) ? T[(int64_t)(p0 + q) * ld + m] * s : 0.f;
        const _Float16 h = (_Float16)v;
        hi[q] = h;
        lo[q] = (_Float16)(v - (float)h);
    }
    const int64_t base = (t * KB + kb) * 2 * 64 + lane;   // in 16-byte units
    tiles[base] = __builtin_bit_cast(u32x4, hi);
    tiles[base + 64] = __builtin_bit_cast(u32x4, lo);
}

}  // namespace

size_t project_tiles_bytes(int64_t rows, int d, bool bf16) {
    return (size_t)split_tiles_bytes(rows, d) / (bf16 ? 2 : 1);
}

hipError_t launch_project_tiles(const float* X, int64_t N, int d, bool bf16, const uint16_t* At,
                                int P, float inv_r, float pscale, uint16_t* xtiles, float* out,
                                int64_t ld, float bound, int* flag, unsigned* norm_slot,
                                hipStream_t stream) {
    const int KB = split_kblocks(d);
    const int64_t ntiles = (N + 15) / 16;
    hipError_t e;
    if (bf16) {
        const unsigned sb = (unsigned)((ntiles * 64 + kBlock - 1) / kBlock);
        hipLaunchKernelGGL(bf16_points_kernel, dim3(sb), dim3(kBlock), 0, stream, X, N, d, KB,
                           ntiles, reinterpret_cast<u32x4*>(xtiles), inv_r, norm_slot);
        e = hipGetLastError();
    } else {   // no per-point range check here: the projections are checked when stored
        e = launch_split_points(X, N, d, inv_r, xtiles, __builtin_inff(), flag, norm_slot, stream);
    }
    if (e != hipSuccess) return e;
    const int64_t ncols = (N + 15) / 16 * 16;          // the padded rows are stored too
    return bf16 ? launch_gemm<1>(xtiles, N, At, P, KB, pscale, nullptr, nullptr, out, ld, ncols,
                                 bound, flag, stream)
                : launch_gemm<2>(xtiles, N, At, P, KB, pscale, nullptr, nullptr, out, ld, ncols,
                                 bound, flag, stream);
}

size_t backproject_tiles_bytes(int64_t rows, int P) { return (size_t)split_tiles_bytes(rows, P); }

size_t backproject_scratch_bytes() { return (size_t)kAbsSlots * kAbsStride * 4 + 256; }

hipError_t launch_backproject_tiles(const float* T, int64_t ld, int64_t M, int P, int d,
                                    const uint16_t* xit, float tau, float coef, const float* v,
                                    float* grad, uint16_t* ttiles, void* scratch,
                                    hipStream_t stream) {
    if (M < 1 || P < 1 || d < 1) return hipErrorInvalidValue;
    unsigned* slots = static_cast<unsigned*>(scratch);
    float* gscale = reinterpret_cast<float*>(slots + kAbsSlots * kAbsStride);
    hipLaunchKernelGGL(clear_slots_kernel, dim3(1), dim3(kBlock), 0, stream, slots);
    const dim3 mg((unsigned)std::min<int64_t>(64, (M + kBlock - 1) / kBlock),
                  (unsigned)std::min(P, 32));
    hipLaunchKernelGGL(abs_max_kernel, mg, dim3(kBlock), 0, stream, T, ld, P, M, slots);
    const int KB = split_kblocks(P);
    const int64_t ntiles = (M + 15) / 16;
    const unsigned sb = (unsigned)((ntiles * KB * 64 + kBlock - 1) / kBlock);
    hipLaunchKernelGGL(split_cols_kernel, dim3(sb), dim3(kBlock), 0, stream, T, ld, P, M, KB,
                       ntiles, slots, tau, reinterpret_cast<u32x4*>(ttiles), gscale);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    // rows m of the T^T tiles in the direction role, rows i of the xi^T
    // tiles in the point role: out[m d + i]
    return launch_gemm<2>(xit, d, ttiles, (int)M, KB, coef, v, gscale, grad, d, d,
                          __builtin_inff(), nullptr, stream);
}

}  // namespace fastsum
