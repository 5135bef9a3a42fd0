// Device helpers shared by the kernel files: wave reductions and the
// Stockham engine wrapper with the same interface as the 2^14-point engine.
#pragma once

#include <hip/hip_runtime.h>

#include "device_fft.h"
#include "fft14.h"
#include "storage.h"

namespace acq {
namespace kdev {

using dev::cadd;
using dev::cmul;
using dev::cmulc;
using dev::Fft;
using dev::dft16;

// One step of a wave sum: each lane adds the value DPP control CTRL routes to
// it (lanes with no source, or in rows outside ROW_MASK, add +0).
template <int CTRL, int ROW_MASK>
__device__ __forceinline__ double dpp_add_step(double v) {
    const unsigned long long b = static_cast<unsigned long long>(__double_as_longlong(v));
    const int lo = __builtin_amdgcn_update_dpp(0, int(unsigned(b)), CTRL, ROW_MASK, 0xf, true);
    const int hi = __builtin_amdgcn_update_dpp(0, int(unsigned(b >> 32)), CTRL, ROW_MASK, 0xf, true);
    return v + __longlong_as_double(static_cast<long long>((static_cast<unsigned long long>(unsigned(hi)) << 32) |
                                                          unsigned(lo)));
}

// Sum over the wave in a fixed order (uniform result, no LDS): row_shr 1, 2,
// 4, 8 leave each 16-lane row's sum in its lane 15; row_bcast 15 (into rows 1
// and 3) and row_bcast 31 (into rows 2 and 3) carry the total to lane 63, each
// lane's value counted once.
__device__ __forceinline__ double wave_sum(double v) {
    v = dpp_add_step<0x111, 0xf>(v);
    v = dpp_add_step<0x112, 0xf>(v);
    v = dpp_add_step<0x114, 0xf>(v);
    v = dpp_add_step<0x118, 0xf>(v);
    v = dpp_add_step<0x142, 0xa>(v);
    v = dpp_add_step<0x143, 0xc>(v);
    const unsigned long long b = static_cast<unsigned long long>(__double_as_longlong(v));
    const unsigned lo = unsigned(__builtin_amdgcn_readlane(int(unsigned(b)), 63));
    const unsigned hi = unsigned(__builtin_amdgcn_readlane(int(unsigned(b >> 32)), 63));
    return __longlong_as_double(static_cast<long long>((static_cast<unsigned long long>(hi) << 32) | lo));
}

// One step of a wave maximum: each lane takes the larger of its value and the
// value DPP control CTRL routes to it (lanes with no source, or in rows outside
// ROW_MASK, see 0).
template <int CTRL, int ROW_MASK>
__device__ __forceinline__ unsigned long long dpp_max_step(unsigned long long v) {
    const int lo = __builtin_amdgcn_update_dpp(0, int(unsigned(v)), CTRL, ROW_MASK, 0xf, true);
    const int hi = __builtin_amdgcn_update_dpp(0, int(unsigned(v >> 32)), CTRL, ROW_MASK, 0xf, true);
    const unsigned long long t = (static_cast<unsigned long long>(unsigned(hi)) << 32) | unsigned(lo);
    return t > v ? t : v;
}

// Maximum over the wave (uniform result, no LDS): row_shr 1, 2, 4, 8 leave each
// 16-lane row's maximum in its lane 15; row_bcast 15 (into rows 1 and 3) and
// row_bcast 31 (into rows 2 and 3) carry the total to lane 63.
__device__ __forceinline__ unsigned long long wave_max(unsigned long long v) {
    v = dpp_max_step<0x111, 0xf>(v);
    v = dpp_max_step<0x112, 0xf>(v);
    v = dpp_max_step<0x114, 0xf>(v);
    v = dpp_max_step<0x118, 0xf>(v);
    v = dpp_max_step<0x142, 0xa>(v);
    v = dpp_max_step<0x143, 0xc>(v);
    const unsigned lo = unsigned(__builtin_amdgcn_readlane(int(unsigned(v)), 63));
    const unsigned hi = unsigned(__builtin_amdgcn_readlane(int(unsigned(v >> 32)), 63));
    return (static_cast<unsigned long long>(hi) << 32) | lo;
}

// ------------------------------------------------------------------ transform engines
// Both engines take v[m] = a[in_index(m)] and leave output index
// out_base() + out_off(r) in v[r].

// Stockham passes (2^10 .. 2^13 points), see device_fft.h.
template <int LOGN_>
struct StockhamEngine {
    using F = Fft<LOGN_>;
    static constexpr int LOGN = LOGN_;
    static constexpr int N = F::N;
    static constexpr int NT = F::NT;
    static constexpr int LDS = F::LDS;
    static constexpr int EXTRA = 1;
    static constexpr int B1_TABLE = 1;
    int t;
    const float2* roots;
    __device__ __forceinline__ void init(const float2* __restrict__ r, float2*) {
        t = int(threadIdx.x);
        roots = r;
    }
    __device__ __forceinline__ int in_index(int m) const { return t + m * NT; }
    __device__ __forceinline__ int out_base() const { return t; }
    // smallest / largest out_base() over the wave (wave-uniform)
    __device__ __forceinline__ int out_min() const { return __builtin_amdgcn_readfirstlane(t & ~63); }
    __device__ __forceinline__ int out_max() const { return out_min() + 63; }
    static constexpr int out_off(int r) { return r * NT; }
    static constexpr int HI_OFF = 1 << 30;      // no output is ever pruned
    // register holding the rr-th smallest output offset
    static constexpr int visit(int rr) { return rr; }
    template <int S>
    __device__ __forceinline__ void transform(float2 (&v)[16], float2* lds, __amdgpu_buffer_rsrc_t,
                                              const float2*, bool = true) const {
        int tq = t;
        asm volatile("" : "+v"(tq));            // recompute addressing per call, no hoisting
        F::template transform<S>(v, lds, roots, tq);
    }
};

using dev::bload;
using dev::Fft14;
using dev::make_rsrc;

}  // namespace kdev
}  // namespace acq
