// Device-side types and helpers shared by the HIP sources of the library.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace fastsum {

typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef float f32x16 __attribute__((ext_vector_type(16)));
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef __bf16 bf16x2v __attribute__((ext_vector_type(2)));
typedef float f32x2v __attribute__((ext_vector_type(2)));
typedef _Float16 h8 __attribute__((ext_vector_type(8)));
typedef unsigned int u32x4 __attribute__((ext_vector_type(4)));
typedef __attribute__((address_space(3))) void lds_void;

// Two floats to BF16, round to nearest even (one v_cvt_pk_bf16_f32 on
// gfx950), packed low half first.
__device__ __forceinline__ unsigned pack_bf16x2(float a, float b) {
    return __builtin_bit_cast(unsigned, __builtin_convertvector((f32x2v){a, b}, bf16x2v));
}

// Raw buffer resource over [p, p + bytes) (bytes < 2^31): loads outside it
// return zero without touching memory (checked per dword).  Third
// descriptor word: 32-bit data format, no swizzle (gfx9).
__device__ __forceinline__ __amdgpu_buffer_rsrc_t buffer_rsrc(const void* p, int64_t bytes) {
    return __builtin_amdgcn_make_buffer_rsrc(const_cast<void*>(p), (short)0, (int)bytes,
                                             0x00020000);
}

__device__ __forceinline__ float buffer_load_f32(__amdgpu_buffer_rsrc_t rs, int byte_off) {
    return __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(rs, byte_off, 0, 0));
}

__device__ __forceinline__ h8 buffer_load_h8(__amdgpu_buffer_rsrc_t rs, int byte_off) {
    return __builtin_bit_cast(h8, __builtin_amdgcn_raw_buffer_load_b128(rs, byte_off, 0, 0));
}

// XCD-aware tile order for the stored projection grids: workgroups are
// dispatched round-robin over the 8 XCDs, so block b runs on XCD b % 8.
// Point tile pt and all direction tiles of it go to one XCD (its L2 keeps the
// point tile while every direction tile reads it): b = 8 (g * ndt + dt) + x
// with pt = 8 g + x.  With fewer than 8 point tiles the order is plain
// (b = pt * ndt + dt), which spreads the direction tiles over the XCDs.
// Returns false for the padding blocks.
__device__ __forceinline__ bool proj_tile_of_block(int b, int ndt, int npt, int& dt, int& pt) {
    if (npt < 8) {
        dt = b % ndt;
        pt = b / ndt;
        return pt < npt;
    }
    const int x = b & 7, j = b >> 3;
    dt = j % ndt;
    pt = (j / ndt) * 8 + x;
    return pt < npt;
}

inline unsigned proj_grid_blocks(int ndt, int npt) {
    return npt < 8 ? (unsigned)(ndt * npt) : (unsigned)(8 * ndt * ((npt + 7) / 8));
}

}  // namespace fastsum
