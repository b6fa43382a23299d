// Exact sliced sums for the energy kernel by sorting, the 1-D method the
// paper uses for the negative distance kernel (Sec. 4.3; one of the 1-D
// algorithms listed in Sec. 2.1; f(t) = -c_d |t| from Table 'tab:kernels',
// Riesz row with r = 1).  Per direction the sources and
// targets are sorted together by projection; in sorted order the FP64
// prefix sums W_< of w and S_< of w x~ over the sources give, at a target
// with projection y~,
//   sum_n w_n |x~_n - y~| = y~ (2 W_< - W) - (2 S_< - S),
// W and S the totals.  Sources tied with the target contribute zero on either
// side, so the order of equal keys does not matter.  No Fourier series, no
// grid: the only approximation left is the slicing.
#include "fastsum_impl.h"

#include <algorithm>

#include <rocprim/device/device_segmented_radix_sort.hpp>
#include <rocprim/iterator/counting_iterator.hpp>
#include <rocprim/iterator/transform_iterator.hpp>

namespace fastsum {

namespace {

constexpr int kSortBlock = 512;                // 8 waves per direction
constexpr int kSortWaves = kSortBlock / 64;
constexpr int kSortItems = 16;                 // consecutive sorted keys per thread and chunk
constexpr int kSortChunk = kSortBlock * kSortItems;
constexpr int kEnergyItems = 8;                // the forward scan: fewer registers, more workgroups
constexpr int kEnergyChunk = kSortBlock * kEnergyItems;
constexpr int kBucketShift = 12;               // targets per output bucket: 4096
constexpr int kBucket = 1 << kBucketShift;
constexpr int kBucketThreads = 256;

// offset of row p: p * L + add
struct RowOffset {
    int64_t L;
    int add;
    __host__ __device__ unsigned int operator()(unsigned int p) const {
        return (unsigned int)((int64_t)p * L + add);
    }
};

using OffsetIt = rocprim::transform_iterator<rocprim::counting_iterator<unsigned int>, RowOffset,
                                             unsigned int>;

// rows of ~1e5 keys: one 1024-thread block per segment, 12 keys per thread,
// 8-bit digits (measured fastest of the shapes tried at 2000 rows of 2e5)
using SortConfig = rocprim::segmented_radix_sort_config<8, rocprim::kernel_config<1024, 12>>;

__device__ __forceinline__ double wave_incl_scan(double v) {
    const int lane = threadIdx.x & 63;
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
        const double t = __shfl_up(v, o, 64);
        if (lane >= o) v += t;
    }
    return v;
}

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    return v;
}

// This thread's share of W = sum_n w_n and S = sum_n w_n x~_n over a row of
// N sources: 16-byte loads, two pairs in flight, then the tail.
__device__ __forceinline__ void row_totals(const float* __restrict__ xr,
                                           const float* __restrict__ w, int N, double& A,
                                           double& B) {
    constexpr int kU = 2;
    const int n4 = N / 4;
    const float4* __restrict__ x4 = reinterpret_cast<const float4*>(xr);
    const float4* __restrict__ w4 = reinterpret_cast<const float4*>(w);
    const bool aligned = ((reinterpret_cast<uintptr_t>(xr) | reinterpret_cast<uintptr_t>(w)) & 15) == 0;
    int n0 = 0;
    if (aligned) {
        int q = threadIdx.x;
        for (; q + (kU - 1) * kSortBlock < n4; q += kU * kSortBlock) {
            float4 xv[kU], wq[kU];
#pragma unroll
            for (int u = 0; u < kU; ++u) {
                xv[u] = x4[q + u * kSortBlock];
                wq[u] = w4[q + u * kSortBlock];
            }
#pragma unroll
            for (int u = 0; u < kU; ++u) {
                A += (double)wq[u].x + (double)wq[u].y + (double)wq[u].z + (double)wq[u].w;
                B += (double)wq[u].x * (double)xv[u].x + (double)wq[u].y * (double)xv[u].y +
                     (double)wq[u].z * (double)xv[u].z + (double)wq[u].w * (double)xv[u].w;
            }
        }
        for (; q < n4; q += kSortBlock) {
            const float4 xv = x4[q], wq = w4[q];
            A += (double)wq.x + (double)wq.y + (double)wq.z + (double)wq.w;
            B += (double)wq.x * (double)xv.x + (double)wq.y * (double)xv.y +
                 (double)wq.z * (double)xv.z + (double)wq.w * (double)xv.w;
        }
        n0 = 4 * n4;
    }
    for (int n = n0 + threadIdx.x; n < N; n += kSortBlock) {
        const double wn = w[n];
        A += wn;
        B += wn * (double)xr[n];
    }
}

// Keys and row positions of the kSortItems sorted entries from i0 (16-byte
// loads where the whole group lies in the row; ii = -1 past its end or for
// a position outside the row).
template <int ITEMS>
__device__ __forceinline__ void load_sorted(const float* __restrict__ kr,
                                            const unsigned int* __restrict__ vr, int64_t base,
                                            int i0, int n_tot, float (&kk)[ITEMS],
                                            int (&ii)[ITEMS]) {
    if (i0 + ITEMS <= n_tot) {
#pragma unroll
        for (int q = 0; q < ITEMS / 4; ++q) {
            const float4 kq = *reinterpret_cast<const float4*>(kr + i0 + 4 * q);
            const uint4 vq = *reinterpret_cast<const uint4*>(vr + i0 + 4 * q);
            kk[4 * q] = kq.x; kk[4 * q + 1] = kq.y; kk[4 * q + 2] = kq.z; kk[4 * q + 3] = kq.w;
            ii[4 * q] = (int)((int64_t)vq.x - base);
            ii[4 * q + 1] = (int)((int64_t)vq.y - base);
            ii[4 * q + 2] = (int)((int64_t)vq.z - base);
            ii[4 * q + 3] = (int)((int64_t)vq.w - base);
        }
    } else {
#pragma unroll
        for (int j = 0; j < ITEMS; ++j) {
            const int i = i0 + j;
            kk[j] = i < n_tot ? kr[i] : 0.f;
            ii[j] = i < n_tot ? (int)((int64_t)vr[i] - base) : -1;
        }
    }
#pragma unroll
    for (int j = 0; j < ITEMS; ++j)
        if (ii[j] < 0 || ii[j] >= n_tot) ii[j] = -1;
}

// One workgroup per direction p.  keys_in is the unsorted row (sources at
// i < N); keys / vals the sorted row with, for each key, its position
// g = p L + i in the unsorted row: i < N is source i, i in [yoff, yoff + M)
// target i - yoff, anything else padding that is skipped (same_xy: every
// i < N is source and target i).  Writes
// V[p ldm + m] = coef * sum_n w_n |x~_n - y~_m|, coef = -c_d / tau, computed in
// FP64 and stored in FP32 (relative rounding 6e-8 of one direction's sum;
// the mean over the directions is taken in FP64 by sorted_reduce_kernel).
// The writes are scattered (targets in sorted order); the workgroups of
// different directions run spread over the whole device, which measured
// The results are not written at their targets' positions (targets arrive
// in sorted order, and scattered 4-byte stores cost whole memory lines):
// target m belongs to bucket m >> kBucketShift, and each bucket of a row
// has a region of exactly its size (every target occurs once per
// direction).  Per chunk, LDS counters give each target a slot after the
// bucket's earlier entries, and the value goes to
// stv[p ldm + (bucket << kBucketShift) + slot], the target's offset in the
// bucket to sti at the same place: runs of consecutive stores.  The slot
// order follows the LDS atomics; sorted_bucket_reduce_kernel places every
// value by its offset, so the results do not depend on it.
// at most 128 VGPRs: two workgroups per CU
__global__ __launch_bounds__(kSortBlock) __attribute__((amdgpu_waves_per_eu(4))) void
sorted_energy_kernel(
    const float* __restrict__ keys_in, const float* __restrict__ keys,
    const unsigned int* __restrict__ vals, int64_t L, int N, int yoff, int M, int same_xy,
    const float* __restrict__ w, double coef, float* __restrict__ stv,
    unsigned short* __restrict__ sti, int64_t ldm) {
    __shared__ double sa[2][kSortWaves], sb[2][kSortWaves];
    __shared__ float cval[kEnergyChunk];     // the chunk's values, ordered by bucket
    __shared__ int ctgt[kEnergyChunk];       // and their targets
    // [0, nb) this chunk's counts, [nb, 2 nb) the runs of the earlier chunks,
    // [2 nb, 3 nb] this chunk's bucket offsets
    extern __shared__ unsigned int bcnt[];
    const int p = blockIdx.x, tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int n_tot = same_xy ? N : yoff + M;
    const int nb = (M + kBucket - 1) >> kBucketShift;
    unsigned int* coff = bcnt + 2 * nb;
    const int64_t base = (int64_t)p * L;
    const float* __restrict__ kr = keys + base;
    const unsigned int* __restrict__ vr = vals + base;
    float* __restrict__ vrow = stv + (int64_t)p * ldm;
    unsigned short* __restrict__ irow = sti + (int64_t)p * ldm;
    for (int b = tid; b < 2 * nb; b += kSortBlock) bcnt[b] = 0u;
    // totals W = sum w_n and S = sum w_n x~_n over the unsorted sources
    double A = 0.0, B = 0.0;
    row_totals(keys_in + base, w, N, A, B);
    A = wave_sum(A);
    B = wave_sum(B);
    if (lane == 0) { sa[1][wave] = A; sb[1][wave] = B; }
    __syncthreads();
    A = B = 0.0;
#pragma unroll
    for (int k = 0; k < kSortWaves; ++k) { A += sa[1][k]; B += sb[1][k]; }
    // exclusive prefix sums W_<, S_< over the sources in sorted order, chunk
    // by chunk: each thread holds kEnergyItems consecutive keys, waves scan by
    // shuffles, the wave totals go through LDS (two buffers: one barrier per
    // chunk suffices)
    double ca = 0.0, cb = 0.0;                        // sums of the earlier chunks
    int par = 0;
    for (int c0 = 0; c0 < n_tot; c0 += kEnergyChunk, par ^= 1) {
        const int i0 = c0 + tid * kEnergyItems;
        float kk[kEnergyItems];
        int ii[kEnergyItems];
        load_sorted<kEnergyItems>(kr, vr, base, i0, n_tot, kk, ii);
        float wv[kEnergyItems];                         // source weights (0 for targets, padding)
        double ta = 0.0, tb = 0.0;
#pragma unroll
        for (int j = 0; j < kEnergyItems; ++j) {
            if (ii[j] < 0 || ii[j] >= n_tot) ii[j] = -1;        // not a position of this row
            wv[j] = (ii[j] >= 0 && ii[j] < N) ? w[ii[j]] : 0.f;
            ta += (double)wv[j];
            tb += (double)wv[j] * (double)kk[j];
        }
        const double ia = wave_incl_scan(ta), ib = wave_incl_scan(tb);
        if (lane == 63) { sa[par][wave] = ia; sb[par][wave] = ib; }
        __syncthreads();
        double pa = ca, pb = cb;
#pragma unroll
        for (int k = 0; k < kSortWaves; ++k) {
            const double xa = sa[par][k], xb = sb[par][k];
            if (k < wave) { pa += xa; pb += xb; }
            ca += xa;
            cb += xb;
        }
        pa += ia - ta;                                  // exclusive prefix of item 0
        pb += ib - tb;
        // slots first (the targets' values follow once the chunk's counts
        // are complete, from the same running prefix sums)
        int slot[kEnergyItems];
#pragma unroll
        for (int j = 0; j < kEnergyItems; ++j) {
            const bool tgt = same_xy ? (ii[j] >= 0 && ii[j] < N) : ii[j] >= yoff;   // < n_tot
            slot[j] = -1;
            if (tgt) {
                const int m = same_xy ? ii[j] : ii[j] - yoff;
                slot[j] = (int)atomicAdd(&bcnt[m >> kBucketShift], 1u);
            }
        }
        __syncthreads();                              // this chunk's counts are complete
        // the chunk's bucket offsets: exclusive scan of the counts by wave 0,
        // 64 buckets per step
        if (wave == 0) {
            unsigned int run = 0u;
            for (int b0 = 0; b0 < nb; b0 += 64) {
                const unsigned int c = (b0 + lane < nb) ? bcnt[b0 + lane] : 0u;
                unsigned int incl = c;
#pragma unroll
                for (int o = 1; o < 64; o <<= 1) {
                    const unsigned int t = (unsigned int)__shfl_up((int)incl, o, 64);
                    if (lane >= o) incl += t;
                }
                if (b0 + lane < nb) coff[b0 + lane] = run + incl - c;
                run += (unsigned int)__shfl((int)incl, 63, 64);
            }
            if (lane == 0) coff[nb] = run;
        }
        __syncthreads();
        // values in LDS by bucket (chunk offset + slot), with their targets
#pragma unroll
        for (int j = 0; j < kEnergyItems; ++j) {
            if (slot[j] >= 0) {
                const int m = same_xy ? ii[j] : ii[j] - yoff;
                const int k = (int)coff[m >> kBucketShift] + slot[j];
                const double y = kk[j];
                cval[k] = (float)(coef * (y * (2.0 * pa - A) - (2.0 * pb - B)));
                ctgt[k] = m;
            }
            pa += (double)wv[j];
            pb += (double)wv[j] * (double)kk[j];
        }
        __syncthreads();
        // consecutive LDS entries of a bucket go to consecutive positions of
        // its region: the stores of a wave cover whole runs
        const int nchunk = (int)coff[nb];
        for (int k = tid; k < nchunk; k += kSortBlock) {
            const int m = ctgt[k];
            const int bk = m >> kBucketShift;
            const int64_t pos = ((int64_t)bk << kBucketShift) + bcnt[nb + bk] + (k - (int)coff[bk]);
            vrow[pos] = cval[k];
            irow[pos] = (unsigned short)(m & (kBucket - 1));
        }
        __syncthreads();                              // every entry has been stored
        for (int bk = tid; bk < nb; bk += kSortBlock) {
            bcnt[nb + bk] += bcnt[bk];
            bcnt[bk] = 0u;
        }
        // the next chunk's atomics follow its scan barrier
    }
}

// Mean over directions of the bucketed per-direction sums: workgroup
// (bucket b, direction range r) places each direction's values of the
// bucket into LDS by their target offsets, then adds them into FP64
// accumulators in direction order; part[r ldm + m] receives the range's sum.
__global__ __launch_bounds__(kBucketThreads) void sorted_bucket_reduce_kernel(
    const float* __restrict__ stv, const unsigned short* __restrict__ sti, int P, int prange,
    int64_t ldm, int M, double* __restrict__ part) {
    __shared__ float vals_lds[kBucket];
    constexpr int kPer = kBucket / kBucketThreads;
    const int tid = threadIdx.x, bk = blockIdx.x;
    const int64_t m0 = (int64_t)bk << kBucketShift;
    const int size = (int)min((int64_t)kBucket, (int64_t)M - m0);
    const int p0 = blockIdx.y * prange, p1 = min(P, p0 + prange);
    double acc[kPer];
#pragma unroll
    for (int k = 0; k < kPer; ++k) acc[k] = 0.0;
    // direction p's entries in registers while p - 1's are summed
    float v[kPer];
    unsigned short ix[kPer];
    auto load = [&](int p) {
        const int64_t base = (int64_t)p * ldm + m0;
#pragma unroll
        for (int k = 0; k < kPer; ++k) {
            const int e = tid + k * kBucketThreads;
            const bool in = e < size && p < p1;
            v[k] = in ? stv[base + e] : 0.f;
            ix[k] = in ? sti[base + e] : (unsigned short)0;
        }
    };
    load(p0);
    for (int p = p0; p < p1; ++p) {
#pragma unroll
        for (int k = 0; k < kPer; ++k)
            if (tid + k * kBucketThreads < size) vals_lds[ix[k]] = v[k];
        __syncthreads();
        load(p + 1);
#pragma unroll
        for (int k = 0; k < kPer; ++k) {
            const int e = tid + k * kBucketThreads;
            if (e < size) acc[k] += (double)vals_lds[e];
        }
        __syncthreads();
    }
#pragma unroll
    for (int k = 0; k < kPer; ++k) {
        const int e = tid + k * kBucketThreads;
        if (e < size) part[(int64_t)blockIdx.y * ldm + m0 + e] = acc[k];
    }
}

// The sort is stable: equal keys keep the order of their positions.  The
// radix order puts -0.0 below +0.0; the projections never produce -0.0
// (their accumulations start from +0.0, and +0.0 + -0.0 = +0.0), so equal
// keys are equal bit patterns.
hipError_t run_sort(void* temp, size_t& temp_bytes, const float* keys_in, float* keys_out,
                    unsigned int* vals_out, int64_t L, int P, int n_tot, hipStream_t stream) {
    const rocprim::counting_iterator<unsigned int> rows(0u);
    const OffsetIt begin(rows, RowOffset{L, 0});
    const OffsetIt end(rows, RowOffset{L, n_tot});
    return rocprim::segmented_radix_sort_pairs<SortConfig>(temp, temp_bytes, keys_in, keys_out,
                                               rocprim::counting_iterator<unsigned int>(0u),
                                               vals_out, (unsigned int)(P * L), (unsigned int)P,
                                               begin, end, 0, 32, stream);
}

// Adjoint of the sorted energy sums, from the ascending sort the exec made.
// The row holds the sources x (weights w, positions i < N) and the targets
// y (cotangent v, positions yoff + m; same_xy: every i < N is source and
// target i).  Per direction, with coef = -c_d / tau and sign(0) = 0:
//   Ty[p][m] = coef sum_n w_n sign(y~_m - x~_n) = coef (W_< - W_>)   (d/dy~ of the sum)
//   Tx[p][n] = coef sum_m v_m sign(x~_n - y~_m) = coef (V_< - V_>)   (d/dx~ of the transposed sum)
//   U[p][n]  = coef sum_m v_m |x~_n - y~_m|                         (the transposed sum)
// with W_<, W_> the weight of the sources of strictly smaller / larger key.
// Equal keys are adjacent in sorted order, so the entries of one key form a
// run and share Ty and Tx: at the run's last entry, with Wi the inclusive
// prefix sum of w there and Wr the run's own weight, W_< = Wi - Wr and
// W_> = W - Wi, so Ty = coef (2 Wi - Wr - W) (Tx likewise with v).  The run
// sums are a segmented scan (restarted where the key changes); each run's
// values go to an LDS slot named by its first entry, which every entry of
// the run finds by a max-scan of run starts.  A run still open at the end
// of a chunk is written once it ends: its entries in earlier chunks are
// read back from the sorted row.  U needs no runs: tied pairs add |0|.
// The values leave as the forward's do, staged by 4096-index bucket
// (stage_bucketed): each output has a value row and an offset row per
// direction, which sorted_place_kernel (Ty, Tx) puts back in index order
// and sorted_bucket_reduce_kernel (U) sums over the directions.
// want: bit 0 Ty, bit 1 Tx, bit 2 U (the others are neither read nor
// written).  FULL = false serves want == 1 alone: no v sums, fewer
// registers, two workgroups per CU.
constexpr int kAdjItems = 8;
constexpr int kAdjChunk = kSortBlock * kAdjItems;

// LDS of one staging round and the bucket counters of the three outputs.
struct StageLds {
    float* cval;             // kAdjChunk values of the round, ordered by bucket
    int* cidx;               // and their indices
    unsigned int* cnt;       // [nbmax] this round's counts per bucket (zero between rounds)
    unsigned int* coff;      // [nbmax + 1] this round's bucket offsets
};

// One staging round of up to kAdjChunk entries (idx < 0: none) of the
// workgroup: slots from LDS counters per bucket idx >> kBucketShift, the
// values ordered by bucket in LDS, then written as runs after the entries
// the bucket's region already holds (run[b]); each value's offset in its
// bucket goes beside it.  Called by every thread (barriers inside).
__device__ __forceinline__ void stage_bucketed(const int (&idx)[kAdjItems],
                                               const float (&val)[kAdjItems], int nb,
                                               const StageLds& sl, unsigned int* run,
                                               float* __restrict__ outv,
                                               unsigned short* __restrict__ outi) {
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    int slot[kAdjItems];
#pragma unroll
    for (int j = 0; j < kAdjItems; ++j)
        slot[j] = idx[j] >= 0 ? (int)atomicAdd(&sl.cnt[idx[j] >> kBucketShift], 1u) : -1;
    __syncthreads();
    if (wave == 0) {
        unsigned int acc = 0u;
        for (int b0 = 0; b0 < nb; b0 += 64) {
            const unsigned int c = (b0 + lane < nb) ? sl.cnt[b0 + lane] : 0u;
            unsigned int incl = c;
#pragma unroll
            for (int o = 1; o < 64; o <<= 1) {
                const unsigned int t = (unsigned int)__shfl_up((int)incl, o, 64);
                if (lane >= o) incl += t;
            }
            if (b0 + lane < nb) sl.coff[b0 + lane] = acc + incl - c;
            acc += (unsigned int)__shfl((int)incl, 63, 64);
        }
        if (lane == 0) sl.coff[nb] = acc;
    }
    __syncthreads();
#pragma unroll
    for (int j = 0; j < kAdjItems; ++j) {
        if (slot[j] >= 0) {
            const int k = (int)sl.coff[idx[j] >> kBucketShift] + slot[j];
            sl.cval[k] = val[j];
            sl.cidx[k] = idx[j];
        }
    }
    __syncthreads();
    const int total = (int)sl.coff[nb];
    for (int k = tid; k < total; k += kSortBlock) {
        const int m = sl.cidx[k];
        const int bk = m >> kBucketShift;
        const int64_t pos = ((int64_t)bk << kBucketShift) + run[bk] + (k - (int)sl.coff[bk]);
        outv[pos] = sl.cval[k];
        outi[pos] = (unsigned short)(m & (kBucket - 1));
    }
    __syncthreads();
    for (int bk = tid; bk < nb; bk += kSortBlock) {
        run[bk] += sl.cnt[bk];
        sl.cnt[bk] = 0u;
    }
    __syncthreads();
}

template <bool FULL>
__global__ __launch_bounds__(kSortBlock) __attribute__((amdgpu_waves_per_eu(FULL ? 1 : 4))) void
sorted_adjoint_kernel(const float* __restrict__ keys_in, const float* __restrict__ keys,
                      const unsigned int* __restrict__ vals, int64_t L, int N, int yoff, int M,
                      int same_xy, const float* __restrict__ w, const float* __restrict__ v,
                      double coef, float* __restrict__ Tyv, unsigned short* __restrict__ Tyo,
                      float* __restrict__ Txv, unsigned short* __restrict__ Txo,
                      float* __restrict__ Uv, unsigned short* __restrict__ Uo, int64_t ldm,
                      int want) {
    __shared__ double sa[2][kSortWaves], sb[2][kSortWaves], sc[2][kSortWaves];
    __shared__ double ra[2][kSortWaves], rb[2][kSortWaves];   // run sums of w, v
    __shared__ int rf[2][kSortWaves], rs[2][kSortWaves];       // a run starts inside; last start
    __shared__ float slot_y[kAdjChunk], slot_x[FULL ? kAdjChunk : 1];
    __shared__ float cval[kAdjChunk];
    __shared__ int cidx[kAdjChunk];
    __shared__ int open_start[2];
    __shared__ double open_w[2], open_v[2];
    // [0, nbm) counts, [nbm, 2 nbm + 1) offsets, then the running counts of
    // Ty (nby), Tx (nbx) and U (nbx)
    extern __shared__ unsigned int bcnt[];
    const int p = blockIdx.x, tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int n_tot = same_xy ? N : yoff + M;
    const int toff = same_xy ? 0 : yoff;
    const int nby = (M + kBucket - 1) >> kBucketShift, nbx = (N + kBucket - 1) >> kBucketShift;
    const int nbm = max(nby, nbx);
    const StageLds sl{cval, cidx, bcnt, bcnt + nbm};
    unsigned int* run_y = bcnt + 2 * nbm + 1;
    unsigned int* run_x = run_y + nby;
    unsigned int* run_u = run_x + nbx;
    for (int b = tid; b < 2 * nbm + 1 + nby + 2 * nbx; b += kSortBlock) bcnt[b] = 0u;
    const int64_t base = (int64_t)p * L;
    const float* __restrict__ kr = keys + base;
    const unsigned int* __restrict__ vr = vals + base;
    float* __restrict__ tyv = Tyv + (int64_t)p * ldm;
    unsigned short* __restrict__ tyo = Tyo + (int64_t)p * ldm;
    float* __restrict__ txv = Txv + (int64_t)p * ldm;
    unsigned short* __restrict__ txo = Txo + (int64_t)p * ldm;
    float* __restrict__ uv = Uv + (int64_t)p * ldm;
    unsigned short* __restrict__ uo = Uo + (int64_t)p * ldm;
    // totals W = sum w, V = sum v, SV = sum v y~ over the unsorted row
    double W = 0.0, V = 0.0, SV = 0.0;
    {
        const float* __restrict__ xr = keys_in + base;
        for (int n = tid; n < N; n += kSortBlock) W += (double)w[n];
        if constexpr (FULL) {
            for (int m = tid; m < M; m += kSortBlock) {
                const double vm = v[m];
                V += vm;
                SV += vm * (double)xr[toff + m];
            }
        }
        W = wave_sum(W);
        if constexpr (FULL) {
            V = wave_sum(V);
            SV = wave_sum(SV);
        }
        if (lane == 0) { sa[1][wave] = W; sb[1][wave] = V; sc[1][wave] = SV; }
        __syncthreads();
        W = V = SV = 0.0;
#pragma unroll
        for (int k = 0; k < kSortWaves; ++k) { W += sa[1][k]; V += sb[1][k]; SV += sc[1][k]; }
    }
    double cw = 0.0, cv = 0.0, csv = 0.0;       // plain sums of the earlier chunks
    int ostart = -1;                            // first entry of the run open at the last chunk's end
    double ow = 0.0, ov = 0.0;                  // and its sums so far
    int par = 0;
    for (int c0 = 0; c0 < n_tot; c0 += kAdjChunk, par ^= 1) {
        const int i0 = c0 + tid * kAdjItems;
        float kk[kAdjItems];
        int ii[kAdjItems];
        load_sorted<kAdjItems>(kr, vr, base, i0, n_tot, kk, ii);
        const float kprev = (i0 > 0 && i0 <= n_tot) ? kr[i0 - 1] : 0.f;
        const float knext = (i0 + kAdjItems < n_tot) ? kr[i0 + kAdjItems] : 0.f;
        float lw[kAdjItems], lv[kAdjItems];
        unsigned int fst = 0u, lst = 0u;        // bit j: item j starts / ends a run
        double tw = 0.0, tv = 0.0, tsv = 0.0;
        bool tf = false;                        // this thread's run aggregate
        double trw = 0.0, trv = 0.0;
        int ts = -1;
#pragma unroll
        for (int j = 0; j < kAdjItems; ++j) {
            const int i = i0 + j, pos = ii[j];
            const bool src = pos >= 0 && pos < N;
            lw[j] = src ? w[pos] : 0.f;
            tw += (double)lw[j];
            if constexpr (FULL) {
                const bool tgt = same_xy ? src : pos >= yoff;      // pos < n_tot
                lv[j] = tgt ? v[pos - toff] : 0.f;
                tv += (double)lv[j];
                tsv += (double)lv[j] * (double)kk[j];
            } else {
                lv[j] = 0.f;
            }
            const float kp = j == 0 ? kprev : kk[j - 1];
            const float kn = j == kAdjItems - 1 ? knext : kk[j + 1];
            const bool valid = i < n_tot;
            if (!valid || i == 0 || kk[j] != kp) {
                fst |= 1u << j;
                tf = true;
                trw = trv = 0.0;
                ts = i;
            }
            if (!valid || i + 1 >= n_tot || kk[j] != kn) lst |= 1u << j;
            trw += (double)lw[j];
            if constexpr (FULL) trv += (double)lv[j];
        }
        const double iw = wave_incl_scan(tw);
        double iv = 0.0, isv = 0.0;
        if constexpr (FULL) {
            iv = wave_incl_scan(tv);
            isv = wave_incl_scan(tsv);
        }
        // segmented inclusive scan of the run sums (a start discards what is
        // before it) and max-scan of the run starts
        double sw = trw, sv = trv;
        int sf = tf ? 1 : 0, ss = ts;
#pragma unroll
        for (int o = 1; o < 64; o <<= 1) {
            const double pw = __shfl_up(sw, o, 64);
            double pv = 0.0;
            if constexpr (FULL) pv = __shfl_up(sv, o, 64);
            const int pf = __shfl_up(sf, o, 64), ps = __shfl_up(ss, o, 64);
            if (lane >= o) {
                if (!sf) {
                    sw += pw;
                    if constexpr (FULL) sv += pv;
                }
                sf |= pf;
                ss = max(ss, ps);
            }
        }
        if (lane == 63) {
            sa[par][wave] = iw; sb[par][wave] = iv; sc[par][wave] = isv;
            ra[par][wave] = sw; rb[par][wave] = sv; rf[par][wave] = sf; rs[par][wave] = ss;
        }
        // the lane before's inclusive aggregate is this lane's exclusive one
        const double xw = __shfl_up(sw, 1, 64);
        double xv = 0.0;
        if constexpr (FULL) xv = __shfl_up(sv, 1, 64);
        const int xf = __shfl_up(sf, 1, 64), xs = __shfl_up(ss, 1, 64);
        __syncthreads();
        double ew = cw, ev = cv, esv = csv;
        double rw = ow, rv = ov;                // run sums entering this thread
        int rstart = ostart;
#pragma unroll
        for (int k = 0; k < kSortWaves; ++k) {
            const double xa = sa[par][k];
            double xb = 0.0, xc = 0.0;
            if constexpr (FULL) { xb = sb[par][k]; xc = sc[par][k]; }
            if (k < wave) {
                ew += xa; ev += xb; esv += xc;
                if (rf[par][k]) {
                    rw = ra[par][k];
                    if constexpr (FULL) rv = rb[par][k];
                } else {
                    rw += ra[par][k];
                    if constexpr (FULL) rv += rb[par][k];
                }
                rstart = max(rstart, rs[par][k]);
            }
            cw += xa;
            cv += xb;
            csv += xc;
        }
        if (lane > 0) {
            if (xf) { rw = xw; rv = xv; }
            else { rw += xw; rv += xv; }
            rstart = max(rstart, xs);
        }
        ew += iw - tw;                          // exclusive prefixes of item 0
        ev += iv - tv;
        esv += isv - tsv;
        int start[kAdjItems];
        float uval[kAdjItems];
#pragma unroll
        for (int j = 0; j < kAdjItems; ++j) {
            if ((fst >> j) & 1u) { rw = rv = 0.0; rstart = i0 + j; }
            rw += (double)lw[j];
            if constexpr (FULL) rv += (double)lv[j];
            start[j] = rstart;
            const double inw = ew + (double)lw[j], inv = ev + (double)lv[j];
            if (((lst >> j) & 1u) && i0 + j < n_tot) {
                const int sl_ = max(rstart, c0) - c0;
                slot_y[sl_] = (float)(coef * (2.0 * inw - rw - W));
                if constexpr (FULL) slot_x[sl_] = (float)(coef * (2.0 * inv - rv - V));
            }
            if constexpr (FULL) {
                const double x = kk[j];
                uval[j] = (float)(coef * (x * (2.0 * ev - V) - (2.0 * esv - SV)));
                esv += (double)lv[j] * (double)kk[j];
            }
            ew = inw;
            ev = inv;
        }
        // a run still open at the chunk's end ends at its last entry, item
        // kAdjItems - 1 of the last thread (a chunk that ends the row closes it)
        if (tid == kSortBlock - 1) {
            const bool open = !((lst >> (kAdjItems - 1)) & 1u);
            open_start[par] = open ? start[kAdjItems - 1] : -1;
            open_w[par] = rw;
            open_v[par] = rv;
        }
        __syncthreads();
        const int still_open = open_start[par];
        // this chunk's entries of the runs that ended in it
        {
            int idx[kAdjItems];
            float val[kAdjItems];
            if (want & 1) {
#pragma unroll
                for (int j = 0; j < kAdjItems; ++j) {
                    const int pos = ii[j];
                    const bool tgt = pos >= 0 && (same_xy ? pos < N : pos >= yoff);
                    idx[j] = (tgt && start[j] != still_open) ? pos - toff : -1;
                    val[j] = slot_y[max(start[j], c0) - c0];
                }
                stage_bucketed(idx, val, nby, sl, run_y, tyv, tyo);
            }
            if constexpr (FULL) {
                if (want & 2) {
#pragma unroll
                    for (int j = 0; j < kAdjItems; ++j) {
                        const int pos = ii[j];
                        idx[j] = (pos >= 0 && pos < N && start[j] != still_open) ? pos : -1;
                        val[j] = slot_x[max(start[j], c0) - c0];
                    }
                    stage_bucketed(idx, val, nbx, sl, run_x, txv, txo);
                }
                if (want & 4) {
#pragma unroll
                    for (int j = 0; j < kAdjItems; ++j) idx[j] = (ii[j] >= 0 && ii[j] < N) ? ii[j] : -1;
                    stage_bucketed(idx, uval, nbx, sl, run_u, uv, uo);
                }
            }
        }
        // the entries before this chunk of a run that ends in it (slot 0),
        // kAdjChunk at a time
        if (ostart >= 0 && still_open != ostart) {
            for (int b0 = ostart; b0 < c0; b0 += kAdjChunk) {
                int pos[kAdjItems], idx[kAdjItems];
                float val[kAdjItems];
#pragma unroll
                for (int j = 0; j < kAdjItems; ++j) {
                    const int i = b0 + tid * kAdjItems + j;
                    const int q = i < c0 ? (int)((int64_t)vr[i] - base) : -1;
                    pos[j] = (q >= 0 && q < n_tot) ? q : -1;
                }
                if (want & 1) {
#pragma unroll
                    for (int j = 0; j < kAdjItems; ++j) {
                        const bool tgt = pos[j] >= 0 && (same_xy ? pos[j] < N : pos[j] >= yoff);
                        idx[j] = tgt ? pos[j] - toff : -1;
                        val[j] = slot_y[0];
                    }
                    stage_bucketed(idx, val, nby, sl, run_y, tyv, tyo);
                }
                if constexpr (FULL) {
                    if (want & 2) {
#pragma unroll
                        for (int j = 0; j < kAdjItems; ++j) {
                            idx[j] = (pos[j] >= 0 && pos[j] < N) ? pos[j] : -1;
                            val[j] = slot_x[0];
                        }
                        stage_bucketed(idx, val, nbx, sl, run_x, txv, txo);
                    }
                }
            }
        }
        ostart = still_open;
        ow = open_w[par];
        ov = open_v[par];
    }
}

// Rows of per-direction values staged by 4096-index bucket (values and
// their offsets in the bucket) put back in index order: workgroup (bucket,
// direction range) places each direction's entries into LDS by offset and
// writes them out contiguously.
__global__ __launch_bounds__(kBucketThreads) void sorted_place_kernel(
    const float* __restrict__ stv, const unsigned short* __restrict__ sti, int P, int prange,
    int64_t ldm, int M, float* __restrict__ out) {
    __shared__ float vals_lds[kBucket];
    constexpr int kPer = kBucket / kBucketThreads;
    const int tid = threadIdx.x, bk = blockIdx.x;
    const int64_t m0 = (int64_t)bk << kBucketShift;
    const int size = (int)min((int64_t)kBucket, (int64_t)M - m0);
    const int p0 = blockIdx.y * prange, p1 = min(P, p0 + prange);
    float v[kPer];
    unsigned short ix[kPer];
    auto load = [&](int p) {
        const int64_t base = (int64_t)p * ldm + m0;
#pragma unroll
        for (int k = 0; k < kPer; ++k) {
            const int e = tid + k * kBucketThreads;
            const bool in = e < size && p < p1;
            v[k] = in ? stv[base + e] : 0.f;
            ix[k] = in ? sti[base + e] : (unsigned short)0;
        }
    };
    load(p0);
    for (int p = p0; p < p1; ++p) {
#pragma unroll
        for (int k = 0; k < kPer; ++k)
            if (tid + k * kBucketThreads < size) vals_lds[ix[k]] = v[k];
        __syncthreads();
        load(p + 1);
        float* __restrict__ row = out + (int64_t)p * ldm + m0;
#pragma unroll
        for (int k = 0; k < kPer; ++k) {
            const int e = tid + k * kBucketThreads;
            if (e < size) row[e] = vals_lds[e];
        }
        __syncthreads();
    }
}

// s[m] = scale * sum_p V[p ldm + m], FP64 over the directions in order.
__global__ __launch_bounds__(256) void sorted_reduce_kernel(const float* __restrict__ V, int P,
                                                            int64_t ldm, int64_t M, double scale,
                                                            float* __restrict__ s, BoundCheck bc) {
    const int64_t m = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (blockIdx.x == 0 && threadIdx.x < 64) finish_bound_check(bc);
    if (m >= M) return;
    double acc = 0.0;
    for (int p = 0; p < P; ++p) acc += (double)V[(int64_t)p * ldm + m];
    s[m] = (float)(scale * acc);
}

}  // namespace

hipError_t launch_sorted_reduce(const float* V, int P, int64_t ldm, int64_t M, double scale,
                                float* s, const BoundCheck& bc, hipStream_t stream) {
    hipLaunchKernelGGL(sorted_reduce_kernel, dim3((unsigned)((M + 255) / 256)), dim3(256), 0,
                       stream, V, P, ldm, M, scale, s, bc);
    return hipGetLastError();
}

size_t sorted_energy_temp_bytes(int64_t L, int P) {
    size_t bytes = 0;
    if (run_sort(nullptr, bytes, nullptr, nullptr, nullptr, L, P, (int)L, nullptr) != hipSuccess)
        return 0;
    return bytes;
}

int sorted_reduce_ranges(int64_t M, int P) {
    // about 2048 workgroups (8 per CU) over the buckets and direction ranges
    const int64_t nb = (M + kBucket - 1) / kBucket;
    return (int)std::max<int64_t>(1, std::min<int64_t>({(int64_t)kSortMaxRanges, (int64_t)P,
                                                         (2048 + nb - 1) / nb}));
}

hipError_t launch_sorted_grad(const float* keys_in, const float* keys_sorted,
                              const unsigned int* vals, int64_t L, int P, int N, int yoff, int M,
                              int same_xy, const float* w, const float* v, double coef,
                              float* Tyv, unsigned short* Tyo, float* Txv, unsigned short* Txo,
                              float* Uv, unsigned short* Uo, int64_t ldm, int want,
                              hipStream_t stream) {
    const int n_tot = same_xy ? N : yoff + M;
    if (N < 1 || M < 1 || (same_xy && M != N) || (!same_xy && yoff < N) || n_tot > L ||
        N > ldm || M > ldm || (int64_t)P * L >= ((int64_t)1 << 32))
        return hipErrorInvalidValue;
    const int nby = (M + kBucket - 1) >> kBucketShift, nbx = (N + kBucket - 1) >> kBucketShift;
    const size_t lds = (size_t)(2 * std::max(nby, nbx) + 1 + nby + 2 * nbx) * sizeof(unsigned int);
    if (want == 1)
        hipLaunchKernelGGL(sorted_adjoint_kernel<false>, dim3((unsigned)P), dim3(kSortBlock), lds,
                           stream, keys_in, keys_sorted, vals, L, N, yoff, M, same_xy, w, v, coef,
                           Tyv, Tyo, Txv, Txo, Uv, Uo, ldm, want);
    else
        hipLaunchKernelGGL(sorted_adjoint_kernel<true>, dim3((unsigned)P), dim3(kSortBlock), lds,
                           stream, keys_in, keys_sorted, vals, L, N, yoff, M, same_xy, w, v, coef,
                           Tyv, Tyo, Txv, Txo, Uv, Uo, ldm, want);
    return hipGetLastError();
}

hipError_t launch_sorted_place(const float* stv, const unsigned short* sti, int P, int64_t ldm,
                               int M, float* out, hipStream_t stream) {
    const int nb = (M + kBucket - 1) >> kBucketShift;
    const int nr = sorted_reduce_ranges(M, P);
    const int prange = (P + nr - 1) / nr;
    hipLaunchKernelGGL(sorted_place_kernel, dim3((unsigned)nb, (unsigned)((P + prange - 1) / prange)),
                       dim3(kBucketThreads), 0, stream, stv, sti, P, prange, ldm, M, out);
    return hipGetLastError();
}


hipError_t launch_sorted_energy(const float* keys_in, float* keys_out, unsigned int* vals_out,
                                void* temp, size_t temp_bytes, int64_t L, int P, int N, int yoff,
                                int M, int same_xy, const float* w, double coef, float* stv,
                                unsigned short* sti, int64_t ldm, hipStream_t stream) {
    const int n_tot = same_xy ? N : yoff + M;
    if (N < 1 || M < 1 || (!same_xy && yoff < N) || n_tot > L || M > ldm ||
        (int64_t)P * L >= ((int64_t)1 << 32))
        return hipErrorInvalidValue;
    size_t bytes = temp_bytes;
    hipError_t e = run_sort(temp, bytes, keys_in, keys_out, vals_out, L, P, n_tot, stream);
    if (e != hipSuccess) return e;
    const int nb = (M + kBucket - 1) >> kBucketShift;
    hipLaunchKernelGGL(sorted_energy_kernel, dim3((unsigned)P), dim3(kSortBlock),
                       (size_t)(3 * nb + 1) * sizeof(unsigned int), stream, keys_in, keys_out, vals_out,
                       L, N, yoff, M, same_xy, w, coef, stv, sti, ldm);
    return hipGetLastError();
}

hipError_t launch_sorted_bucket_reduce(const float* stv, const unsigned short* sti, int P,
                                       int64_t ldm, int M, double* part, double scale, float* s,
                                       const BoundCheck& bc, hipStream_t stream) {
    const int nb = (M + kBucket - 1) >> kBucketShift;
    const int nr = sorted_reduce_ranges(M, P);
    const int prange = (P + nr - 1) / nr;
    hipLaunchKernelGGL(sorted_bucket_reduce_kernel, dim3((unsigned)nb, (unsigned)((P + prange - 1) / prange)),
                       dim3(kBucketThreads), 0, stream, stv, sti, P, prange, ldm, M, part);
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    return launch_reduce(part, (P + prange - 1) / prange, ldm, M, scale, s, bc, stream);
}

}  // namespace fastsum
