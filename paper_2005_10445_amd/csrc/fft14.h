// 16384-point FFT on one workgroup of 16 waves, with a single workgroup-wide
// exchange per transform.
//
// Thread t = 64 w + l (wave w, lane l) holds v[m] = x[t + 1024 m] on entry.
// With N = 16384 = 16 * 1024 and 1024 = 16 * 64 = 16 * (16 * 4):
//
//   A : 16-point DFT over m in registers -> A[t][k1]
//   X1: workgroup exchange through LDS: wave w' receives A[l + 64 m'][k1 = w'];
//       the outer twiddle exp(s j 2 pi t k1 / N) is split into a wave-uniform
//       part exp(s j 2 pi w' m' / 256) (scalar registers) and a per-lane part
//       exp(s j 2 pi w' l / N) that is common to all m' and is folded into the
//       next twiddle layer;
//   B1: 16-point DFT over m' -> k2a, twiddle exp(s j 2 pi l (w' + 16 k2a) / N)
//       from a table laid out [w'][k2a][l] (prefetched while the workgroup
//       waits at X1);
//   X2: wave-private exchange: lane (k2a, q) receives the 16 values l = q + 4 m'';
//   B2: 16-point DFT over m'' -> kb1, twiddle exp(s j 2 pi q kb1 / 64) (LDS table);
//   X3: wave-private 4 x 4 exchange inside each lane quad;
//   B3: 4-point DFTs over q.
//
// On exit lane l of wave w holds, in v[4 j + kb2], the output with index
//   u = w + 16 (l >> 2) + 1024 (l & 3) + 256 j + 4096 kb2.
//
// Every wave works on its own slice of LDS after X1, so only X1 needs
// workgroup barriers; X2 and X3 are ordered within the wave.  Each slice is 16
// rows of 64 complex plus 4 pad, which makes every exchange free of bank
// conflicts (for both 32 and 64 four-byte banks).  A transform begins with a
// barrier before its X1 writes (the previous transform's X2/X3 use every
// slice), so work before that point -- loading and scaling the next input and
// stage A -- overlaps the slower waves' end of the previous transform.
// With hi = false only outputs kb2 = 0, 1 (u < 8192) are formed.
#pragma once

#include <hip/hip_runtime.h>

#include "device_fft.h"

namespace acq {
namespace dev {

__device__ __forceinline__ __amdgpu_buffer_rsrc_t make_rsrc(const void* p, uint32_t bytes) {
    // raw buffer, stride 0, num_records in bytes; loads past the end return 0
    return __builtin_amdgcn_make_buffer_rsrc(const_cast<void*>(p), (short)0, (int)bytes, 0x00020000);
}

__device__ __forceinline__ float2 bload(__amdgpu_buffer_rsrc_t r, int voff_bytes, int soff_bytes) {
    return __builtin_bit_cast(float2, __builtin_amdgcn_raw_buffer_load_b64(r, voff_bytes, soff_bytes, 0));
}

// Order LDS accesses of one wave (LDS executes a wave's instructions in order;
// this only keeps the compiler from moving them across).
__device__ __forceinline__ void wave_lds_order() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

template <int S>
__device__ __forceinline__ float2 tw_sign(float2 w) {
    return S > 0 ? w : make_float2(w.x, -w.y);
}

struct Fft14 {
    static constexpr int LOGN = 14;
    static constexpr int N = 1 << 14;
    static constexpr int NT = 1024;
    static constexpr int ROW = 68;                  // 64 + 4 pad
    static constexpr int SLICE = 16 * ROW;
    static constexpr int LDS = 16 * SLICE;          // complex elements
    // B2 twiddles [q][kb1] = exp(+j 2 pi q kb1 / 64) in rows of 17 entries: a
    // lane reads its row from one base register with immediate offsets, and
    // the four rows of a lane quad start on distinct LDS banks (rows of 16
    // put q = 0, 2 and q = 1, 3 on the same banks)
    static constexpr int EXTRA = 4 * 17;
    // B1 twiddle table entries: [w][k2a][l] = exp(+j 2 pi l (w + 16 k2a) / N)
    static constexpr int B1_TABLE = 16 * 16 * 64;

    int w, l;
    float2 wu[16];                                  // exp(+j 2 pi w m / 256), wave-uniform

    // roots: exp(+j 2 pi x / N), x < N.  extra: LDS table of EXTRA entries,
    // visible to the workgroup after the first transform's X1 barrier.
    __device__ __forceinline__ void init(const float2* __restrict__ roots, float2* extra) {
        w = __builtin_amdgcn_readfirstlane(int(threadIdx.x) >> 6);
        l = int(threadIdx.x) & 63;
#pragma unroll
        for (int m = 0; m < 16; ++m) wu[m] = roots[(w * m * 64) & (N - 1)];
        if (threadIdx.x < EXTRA) extra[threadIdx.x] = roots[(((threadIdx.x / 17) * (threadIdx.x % 17)) & 63) * (N / 64)];
    }

    // index of the element in input register m
    __device__ __forceinline__ int in_index(int m) const { return (w << 6) + l + m * NT; }
    // output register r = 4 j + kb2 holds index out_base() + out_off(r)
    __device__ __forceinline__ int out_base() const { return w + 16 * (l >> 2) + 1024 * (l & 3); }
    // smallest / largest out_base() over the wave (wave-uniform)
    __device__ __forceinline__ int out_min() const { return w; }
    __device__ __forceinline__ int out_max() const { return w + 16 * 15 + 1024 * 3; }
    static constexpr int out_off(int r) { return 256 * (r >> 2) + 4096 * (r & 3); }
    static constexpr int HI_OFF = 8192;         // outputs with kb2 >= 2 start here
    // register holding the rr-th smallest output offset (out_off increases with rr)
    static constexpr int visit(int rr) { return ((rr & 3) << 2) | (rr >> 2); }

    template <int S>
    __device__ __forceinline__ void transform(float2 (&v)[16], float2* lds, __amdgpu_buffer_rsrc_t b1tab,
                                              const float2* extra, bool hi = true) const {
        int ln = l;
        asm volatile("" : "+v"(ln));            // recompute lane addressing per call
        // A
        dft16<S>(v);
        // B1 twiddles of this lane, table row [w][k2a][l]: the first PRE are
        // prefetched across the barriers, the rest are loaded after X1
        constexpr int PRE = 8;
        const int tboff = (w * 1024 + ln) * 8;
        float2 tb[16];
#pragma unroll
        for (int k2a = 0; k2a < PRE; ++k2a) tb[k2a] = bload(b1tab, tboff, k2a * 512);
        __syncthreads();                        // every wave is done with the previous transform's slices
        // X1 write: element (t, k1) -> slice k1, row w, column l.  Slices 8..15
        // lie beyond the 64 KiB reach of a DS immediate offset, so they get a
        // base register of their own (else every store there needs an add).
        {
            float2* p = lds + w * ROW + ln;
            int hi8 = 8 * SLICE;
            asm("" : "+s"(hi8));
            float2* p8 = p + hi8;
#pragma unroll
            for (int k1 = 0; k1 < 8; ++k1) p[k1 * SLICE] = v[k1];
#pragma unroll
            for (int k1 = 0; k1 < 8; ++k1) p8[k1 * SLICE] = v[k1 + 8];
        }
        __syncthreads();
        float2* sl = lds + w * SLICE;
        // X1 read: wave w gets A[l + 64 m][w]
        {
            const float2* q = sl + ln;
#pragma unroll
            for (int m = 0; m < 16; ++m) v[m] = q[m * ROW];
        }
#pragma unroll
        for (int k2a = PRE; k2a < 16; ++k2a) tb[k2a] = bload(b1tab, tboff, k2a * 512);
#pragma unroll
        for (int m = 1; m < 16; ++m) v[m] = cmul(v[m], tw_sign<S>(wu[m]));
        // B1
        dft16<S>(v);
#pragma unroll
        for (int k2a = 0; k2a < 16; ++k2a) v[k2a] = cmul(v[k2a], tw_sign<S>(tb[k2a]));
        // X2: row k2a, column l; lane (k2a', q) reads columns q + 4 m''
        wave_lds_order();
        {
            float2* p = sl + ln;
#pragma unroll
            for (int k2a = 0; k2a < 16; ++k2a) p[k2a * ROW] = v[k2a];
        }
        wave_lds_order();
        const int k2 = ln >> 2, q = ln & 3;
        float2* row = sl + k2 * ROW;
        {
            const float2* p = row + q;
#pragma unroll
            for (int m = 0; m < 16; ++m) v[m] = p[4 * m];
        }
        // B2
        dft16<S>(v);
        {
            int qrow = 17 * q;
            asm("" : "+v"(qrow));                   // keep the row base in one register
            const float2* tq = extra + qrow;
#pragma unroll
            for (int kb1 = 1; kb1 < 16; ++kb1) v[kb1] = cmul(v[kb1], tw_sign<S>(tq[kb1]));
        }
        // X3: (q, kb1) -> column 4 kb1 + ((q + kb1/4) & 3); lane (k2a, p) reads kb1 = 4 p + j
        wave_lds_order();
#pragma unroll
        for (int a = 0; a < 4; ++a) {
            float2* p = row + ((q + a) & 3) + 16 * a;
#pragma unroll
            for (int b = 0; b < 4; ++b) p[4 * b] = v[4 * a + b];
        }
        wave_lds_order();
#pragma unroll
        for (int qq = 0; qq < 4; ++qq) {
            const float2* p = row + 16 * q + ((qq + q) & 3);
#pragma unroll
            for (int j = 0; j < 4; ++j) v[4 * j + qq] = p[4 * j];
        }
        // B3
        if (hi) {
#pragma unroll
            for (int j = 0; j < 4; ++j) dft4<S>(v[4 * j], v[4 * j + 1], v[4 * j + 2], v[4 * j + 3]);
        } else {
#pragma unroll
            for (int j = 0; j < 4; ++j) dft4_low<S>(v[4 * j], v[4 * j + 1], v[4 * j + 2], v[4 * j + 3]);
        }
    }
};

}  // namespace dev
}  // namespace acq
