// Exact sliced sums for the energy kernel by sorting, the 1-D method the
// paper uses for the negative distance kernel (Sec. 4; f(t) = -c_d |t| from
// Table 'tab:kernels', Riesz row with r = 1).  Per direction the sources and
// targets are sorted together by projection; in sorted order the FP64
// prefix sums W_< of w and S_< of w x~ over the sources give, at a target
// with projection y~,
//   sum_n w_n |x~_n - y~| = y~ (2 W_< - W) - (2 S_< - S),
// W and S the totals.  Sources tied with the target contribute zero on either
// side, so the order of equal keys does not matter.  No Fourier series, no
// grid: the only approximation left is the slicing.
#include "fastsum_impl.h"

#include <rocprim/device/device_segmented_radix_sort.hpp>
#include <rocprim/iterator/counting_iterator.hpp>
#include <rocprim/iterator/transform_iterator.hpp>

namespace fastsum {

namespace {

constexpr int kSortBlock = 256;
constexpr int kSortItems = 4;        // sorted elements per thread and chunk

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

__device__ __forceinline__ void block_sum2(double& a, double& b, double* sa, double* sb) {
    const int tid = threadIdx.x;
    sa[tid] = a;
    sb[tid] = b;
    __syncthreads();
    for (int h = kSortBlock / 2; h > 0; h >>= 1) {
        if (tid < h) {
            sa[tid] += sa[tid + h];
            sb[tid] += sb[tid + h];
        }
        __syncthreads();
    }
    a = sa[0];
    b = sb[0];
    __syncthreads();
}

// One workgroup per direction p.  vals holds, for each sorted key, its
// position g = p L + i in the unsorted row: i < N is source i, i in
// [yoff, yoff + M) target i - yoff, anything else padding that is skipped
// (same_xy: every i < N is source and target i).  Writes
// V[p ldm + m] = coef * sum_n w_n |x~_n - y~_m|, coef = -c_d / tau.
__global__ __launch_bounds__(kSortBlock) void sorted_energy_kernel(
    const float* __restrict__ keys, const unsigned int* __restrict__ vals, int64_t L, int N,
    int yoff, int M, int same_xy, const float* __restrict__ w, double coef, double* __restrict__ V,
    int64_t ldm) {
    __shared__ double sa[kSortBlock], sb[kSortBlock];
    const int p = blockIdx.x, tid = threadIdx.x;
    const int n_tot = same_xy ? N : yoff + M;
    const int64_t base = (int64_t)p * L;
    const float* __restrict__ kr = keys + base;
    const unsigned int* __restrict__ vr = vals + base;
    double* __restrict__ vrow = V + (int64_t)p * ldm;
    // totals over the sources
    double A = 0.0, B = 0.0;
    for (int i = tid; i < n_tot; i += kSortBlock) {
        const int idx = (int)((int64_t)vr[i] - base);
        if (idx >= 0 && idx < N) {
            const double wi = w[idx];
            A += wi;
            B += wi * (double)kr[i];
        }
    }
    block_sum2(A, B, sa, sb);
    // chunked exclusive scan in sorted order
    double ca = 0.0, cb = 0.0;                        // sums of the earlier chunks
    for (int c0 = 0; c0 < n_tot; c0 += kSortBlock * kSortItems) {
        float kk[kSortItems];
        int ii[kSortItems];
        double la[kSortItems], lb[kSortItems];
        double ta = 0.0, tb = 0.0;
#pragma unroll
        for (int j = 0; j < kSortItems; ++j) {
            const int i = c0 + tid * kSortItems + j;
            ii[j] = -1;
            la[j] = lb[j] = 0.0;
            kk[j] = 0.f;
            if (i < n_tot) {
                kk[j] = kr[i];
                ii[j] = (int)((int64_t)vr[i] - base);
                if (ii[j] < 0 || ii[j] >= n_tot) ii[j] = -1;     // not a position of this row
                if (ii[j] >= 0 && ii[j] < N) {
                    la[j] = w[ii[j]];
                    lb[j] = la[j] * (double)kk[j];
                }
            }
            ta += la[j];
            tb += lb[j];
        }
        // inclusive scan of the thread totals (Hillis-Steele in LDS, FP64)
        sa[tid] = ta;
        sb[tid] = tb;
        __syncthreads();
        for (int h = 1; h < kSortBlock; h <<= 1) {
            const double xa = tid >= h ? sa[tid - h] : 0.0;
            const double xb = tid >= h ? sb[tid - h] : 0.0;
            __syncthreads();
            sa[tid] += xa;
            sb[tid] += xb;
            __syncthreads();
        }
        double pa = ca + sa[tid] - ta, pb = cb + sb[tid] - tb;   // exclusive
        const double chunk_a = sa[kSortBlock - 1], chunk_b = sb[kSortBlock - 1];
#pragma unroll
        for (int j = 0; j < kSortItems; ++j) {
            const bool tgt = same_xy ? (ii[j] >= 0 && ii[j] < N) : ii[j] >= yoff;   // < n_tot
            if (tgt) {
                const int m = same_xy ? ii[j] : ii[j] - yoff;
                const double y = kk[j];
                vrow[m] = coef * (y * (2.0 * pa - A) - (2.0 * pb - B));
            }
            pa += la[j];
            pb += lb[j];
        }
        ca += chunk_a;
        cb += chunk_b;
        __syncthreads();
    }
}

hipError_t run_sort(void* temp, size_t& temp_bytes, const float* keys_in, float* keys_out,
                    unsigned int* vals_out, int64_t L, int P, int n_tot, hipStream_t stream) {
    const rocprim::counting_iterator<unsigned int> rows(0u);
    const OffsetIt begin(rows, RowOffset{L, 0});
    const OffsetIt end(rows, RowOffset{L, n_tot});
    return rocprim::segmented_radix_sort_pairs(temp, temp_bytes, keys_in, keys_out,
                                               rocprim::counting_iterator<unsigned int>(0u),
                                               vals_out, (unsigned int)(P * L), (unsigned int)P,
                                               begin, end, 0, 32, stream);
}

}  // namespace

size_t sorted_energy_temp_bytes(int64_t L, int P) {
    size_t bytes = 0;
    if (run_sort(nullptr, bytes, nullptr, nullptr, nullptr, L, P, (int)L, nullptr) != hipSuccess)
        return 0;
    return bytes;
}

hipError_t launch_sorted_energy(const float* keys_in, float* keys_out, unsigned int* vals_out,
                                void* temp, size_t temp_bytes, int64_t L, int P, int N, int yoff,
                                int M, int same_xy, const float* w, double coef, double* V,
                                int64_t ldm, hipStream_t stream) {
    const int n_tot = same_xy ? N : yoff + M;
    if (N < 1 || M < 1 || (!same_xy && yoff < N) || n_tot > L || M > ldm ||
        (int64_t)P * L >= ((int64_t)1 << 32))
        return hipErrorInvalidValue;
    size_t bytes = temp_bytes;
    hipError_t e = run_sort(temp, bytes, keys_in, keys_out, vals_out, L, P, n_tot, stream);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(sorted_energy_kernel, dim3((unsigned)P), dim3(kSortBlock), 0, stream,
                       keys_out, vals_out, L, N, yoff, M, same_xy, w, coef, V, ldm);
    return hipGetLastError();
}

}  // namespace fastsum
