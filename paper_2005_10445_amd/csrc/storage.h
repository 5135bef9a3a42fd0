// Storage formats of the segment spectra and the replica bank.
//
// FP32 stores complex64.  FP16 and BF16 store each complex value as two
// 16-bit halves packed into 32 bits (real in the low half), rounded to nearest
// even; all arithmetic after loading is FP32.  The caller applies power-of-two
// prescales so that typical magnitudes are near 1 (exact, undone in FP32).
#pragma once

#include <hip/hip_runtime.h>
#include <cstdint>

#include "acq.h"

namespace acq {
namespace dev {

template <int PREC>
struct Storage;

template <>
struct Storage<ACQ_FP32> {
    using T = float2;
    static constexpr int BYTES = 8;
    __device__ __forceinline__ static T pack(float2 v) { return v; }
    __device__ __forceinline__ static float2 unpack(T v) { return v; }
    __device__ __forceinline__ static float2 bload(__amdgpu_buffer_rsrc_t r, int voff, int soff) {
        return __builtin_bit_cast(float2, __builtin_amdgcn_raw_buffer_load_b64(r, voff, soff, 0));
    }
};

template <>
struct Storage<ACQ_FP16> {
    using T = uint32_t;
    static constexpr int BYTES = 4;
    __device__ __forceinline__ static T pack(float2 v) {
        const _Float16 re = (_Float16)v.x, im = (_Float16)v.y;   // round to nearest even
        return uint32_t(__builtin_bit_cast(uint16_t, re)) | (uint32_t(__builtin_bit_cast(uint16_t, im)) << 16);
    }
    __device__ __forceinline__ static float2 unpack(T v) {
        const _Float16 re = __builtin_bit_cast(_Float16, uint16_t(v & 0xffffu));
        const _Float16 im = __builtin_bit_cast(_Float16, uint16_t(v >> 16));
        return make_float2(float(re), float(im));
    }
    __device__ __forceinline__ static float2 bload(__amdgpu_buffer_rsrc_t r, int voff, int soff) {
        return unpack(__builtin_amdgcn_raw_buffer_load_b32(r, voff, soff, 0));
    }
};

template <>
struct Storage<ACQ_BF16> {
    using T = uint32_t;
    static constexpr int BYTES = 4;
    // FP32 -> BF16, round to nearest even (inputs are finite)
    __device__ __forceinline__ static uint32_t to_bf16(float f) {
        const uint32_t u = __float_as_uint(f);
        return (u + 0x7fffu + ((u >> 16) & 1u)) >> 16;
    }
    __device__ __forceinline__ static T pack(float2 v) { return to_bf16(v.x) | (to_bf16(v.y) << 16); }
    __device__ __forceinline__ static float2 unpack(T v) {
        return make_float2(__uint_as_float(v << 16), __uint_as_float(v & 0xffff0000u));
    }
    __device__ __forceinline__ static float2 bload(__amdgpu_buffer_rsrc_t r, int voff, int soff) {
        return unpack(__builtin_amdgcn_raw_buffer_load_b32(r, voff, soff, 0));
    }
};

}  // namespace dev
}  // namespace acq
