// Momentum step of the MMD gradient flow (App. MMD flows):
//   v <- grad G(x) + m v,   x <- x - tau v,
// one pass over the particles that also copies the new x into the flow's
// source rows and takes the largest new squared norm, which the next
// step's bound (App. J, eq. radius_xy) needs.
#include "fastsum.h"
#include "fastsum_impl.h"

#include <cmath>

namespace fastsum {

namespace {

constexpr int kFlowBlock = 256;      // four rows per workgroup, one wave each

__global__ void flow_clear_kernel(unsigned int* __restrict__ slot) { *slot = 0u; }

// Row `row` of N x d, lane-strided; the row's ||x_new||^2 goes into *max_bits
// by an atomic max on its bits (non-negative floats, +inf and NaN order as
// their bit patterns).
__global__ __launch_bounds__(kFlowBlock) void flow_update_kernel(
    const float* __restrict__ g, float* __restrict__ v, float* __restrict__ x,
    float* __restrict__ z, int64_t N, int d, float m, float tau,
    unsigned int* __restrict__ max_bits) {
    const int lane = threadIdx.x & 63;
    const int64_t row = (int64_t)blockIdx.x * (kFlowBlock / 64) + (threadIdx.x >> 6);
    if (row >= N) return;                       // whole waves
    const int64_t o = row * d;
    const float* __restrict__ gr = g + o;
    float* __restrict__ vr = v + o;
    float* __restrict__ xr = x + o;
    float* __restrict__ zr = z ? z + o : nullptr;
    float acc = 0.f;
    const uintptr_t al = reinterpret_cast<uintptr_t>(gr) | reinterpret_cast<uintptr_t>(vr) |
                         reinterpret_cast<uintptr_t>(xr) | reinterpret_cast<uintptr_t>(zr);
    int j0 = 0;
    if ((al & 15) == 0) {
        const int d4 = d / 4;
        for (int j = lane; j < d4; j += 64) {
            const float4 gg = reinterpret_cast<const float4*>(gr)[j];
            float4 vv = reinterpret_cast<const float4*>(vr)[j];
            float4 xx = reinterpret_cast<const float4*>(xr)[j];
            vv.x = fmaf(m, vv.x, gg.x);
            vv.y = fmaf(m, vv.y, gg.y);
            vv.z = fmaf(m, vv.z, gg.z);
            vv.w = fmaf(m, vv.w, gg.w);
            xx.x = fmaf(-tau, vv.x, xx.x);
            xx.y = fmaf(-tau, vv.y, xx.y);
            xx.z = fmaf(-tau, vv.z, xx.z);
            xx.w = fmaf(-tau, vv.w, xx.w);
            reinterpret_cast<float4*>(vr)[j] = vv;
            reinterpret_cast<float4*>(xr)[j] = xx;
            if (zr) reinterpret_cast<float4*>(zr)[j] = xx;
            acc += xx.x * xx.x + xx.y * xx.y + xx.z * xx.z + xx.w * xx.w;
        }
        j0 = 4 * d4;
    }
    for (int j = j0 + lane; j < d; j += 64) {
        const float vn = fmaf(m, vr[j], gr[j]);
        const float xn = fmaf(-tau, vn, xr[j]);
        vr[j] = vn;
        xr[j] = xn;
        if (zr) zr[j] = xn;
        acc += xn * xn;
    }
#pragma unroll
    for (int s = 32; s > 0; s >>= 1) acc += __shfl_xor(acc, s, 64);
    if (lane == 0) atomicMax(max_bits, __float_as_uint(acc));
}

}  // namespace

}  // namespace fastsum

extern "C" fastsum_status fastsum_flow_update(int64_t N, int32_t d, float momentum, float step,
                                              const float* g, float* v, float* x, float* z,
                                              float* max_norm2, void* stream) {
    if (!g || !v || !x || !max_norm2 || N < 1 || d < 1 || !std::isfinite(momentum) ||
        !std::isfinite(step))
        return FASTSUM_EINVAL;
    if (z == x) z = nullptr;                    // the rows are already the particles
    hipStream_t st = (hipStream_t)stream;
    unsigned int* slot = reinterpret_cast<unsigned int*>(max_norm2);
    hipLaunchKernelGGL(fastsum::flow_clear_kernel, dim3(1), dim3(1), 0, st, slot);
    const int rows = fastsum::kFlowBlock / 64;
    hipLaunchKernelGGL(fastsum::flow_update_kernel, dim3((unsigned)((N + rows - 1) / rows)),
                       dim3(fastsum::kFlowBlock), 0, st, g, v, x, z, N, (int)d, momentum, step,
                       slot);
    return hipGetLastError() == hipSuccess ? FASTSUM_OK : FASTSUM_EDEVICE;
}
