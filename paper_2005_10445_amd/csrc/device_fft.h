// Workgroup-level power-of-two FFTs for gfx950, staged through LDS.
//
// An N-point transform (N = 2^LOGN, 2^10 <= N <= 2^14) runs on N/16 threads.
// Thread t holds 16 complex values in registers, v[m] = a[t + m*N/16], both
// before and after the transform (natural order in and out).  The transform is
// a Stockham autosort sequence of radix-16 passes plus one final radix-2/4/8
// pass when log2(N) is not a multiple of four:
//
//   pass (Ns, R): butterfly b reads a[b + r*N/R] (r < R), multiplies input r by
//   exp(s j 2 pi (b mod Ns) r / (Ns R)), takes an R-point DFT and writes output
//   r to (b / Ns) * Ns * R + (b mod Ns) + r * Ns;  Ns = 1, 16, 256, ...
//
// With 16 values per thread every pass reads the same index set t + m*N/16,
// so values stay in registers and LDS is used only to exchange them between
// passes (one write, one read per pass).  LDS indices are padded by one
// complex per 16 (i + i/16) so the stride-16 writes of the first pass hit
// distinct banks.  Sign s = -1 is the forward DFT, s = +1 the inverse
// (unnormalised).  Twiddles come from a table of exp(+j 2 pi m / N).
#pragma once

#include <hip/hip_runtime.h>

namespace acq {
namespace dev {

__device__ __forceinline__ float2 cadd(float2 a, float2 b) { return make_float2(a.x + b.x, a.y + b.y); }
__device__ __forceinline__ float2 csub(float2 a, float2 b) { return make_float2(a.x - b.x, a.y - b.y); }
__device__ __forceinline__ float2 cmul(float2 a, float2 b) {
    return make_float2(fmaf(a.x, b.x, -a.y * b.y), fmaf(a.x, b.y, a.y * b.x));
}
// a * conj(b)
__device__ __forceinline__ float2 cmulc(float2 a, float2 b) {
    return make_float2(fmaf(a.x, b.x, a.y * b.y), fmaf(a.y, b.x, -a.x * b.y));
}
__device__ __forceinline__ float2 cscale(float2 a, float s) { return make_float2(a.x * s, a.y * s); }
// a * (S j), S = +1 or -1
template <int S>
__device__ __forceinline__ float2 mul_sj(float2 a) {
    return S > 0 ? make_float2(-a.y, a.x) : make_float2(a.y, -a.x);
}

constexpr float kRsqrt2 = 0.70710678118654752440f;
constexpr float kCos8 = 0.92387953251128675613f;   // cos(pi/8)
constexpr float kSin8 = 0.38268343236508977173f;   // sin(pi/8)

// a * exp(S j pi/4)
template <int S>
__device__ __forceinline__ float2 mul_w8(float2 a) {
    return S > 0 ? make_float2((a.x - a.y) * kRsqrt2, (a.x + a.y) * kRsqrt2)
                 : make_float2((a.x + a.y) * kRsqrt2, (a.y - a.x) * kRsqrt2);
}
// a * exp(S j 3pi/4)
template <int S>
__device__ __forceinline__ float2 mul_w8_3(float2 a) {
    return S > 0 ? make_float2(-(a.x + a.y) * kRsqrt2, (a.x - a.y) * kRsqrt2)
                 : make_float2((a.y - a.x) * kRsqrt2, -(a.x + a.y) * kRsqrt2);
}
// a * (c + S j s)
template <int S>
__device__ __forceinline__ float2 mul_cs(float2 a, float c, float s) {
    return S > 0 ? make_float2(fmaf(a.x, c, -a.y * s), fmaf(a.x, s, a.y * c))
                 : make_float2(fmaf(a.x, c, a.y * s), fmaf(a.y, c, -a.x * s));
}

// ---------------------------------------------------------------- small DFTs
template <int S>
__device__ __forceinline__ void dft2(float2& a, float2& b) {
    const float2 t = a;
    a = cadd(t, b);
    b = csub(t, b);
}

template <int S>
__device__ __forceinline__ void dft4(float2& x0, float2& x1, float2& x2, float2& x3) {
    const float2 a0 = cadd(x0, x2), a1 = csub(x0, x2);
    const float2 b0 = cadd(x1, x3), b1 = mul_sj<S>(csub(x1, x3));
    x0 = cadd(a0, b0);
    x2 = csub(a0, b0);
    x1 = cadd(a1, b1);
    x3 = csub(a1, b1);
}

// outputs 0 and 1 of dft4 only (x2, x3 are left unspecified)
template <int S>
__device__ __forceinline__ void dft4_low(float2& x0, float2& x1, float2& x2, float2& x3) {
    const float2 a0 = cadd(x0, x2), a1 = csub(x0, x2);
    const float2 b0 = cadd(x1, x3), b1 = mul_sj<S>(csub(x1, x3));
    x0 = cadd(a0, b0);
    x1 = cadd(a1, b1);
}

template <int S>
__device__ __forceinline__ void dft8(float2 (&u)[8]) {
    float2 e0 = u[0], e1 = u[2], e2 = u[4], e3 = u[6];
    float2 o0 = u[1], o1 = u[3], o2 = u[5], o3 = u[7];
    dft4<S>(e0, e1, e2, e3);
    dft4<S>(o0, o1, o2, o3);
    o1 = mul_w8<S>(o1);
    o2 = mul_sj<S>(o2);
    o3 = mul_w8_3<S>(o3);
    u[0] = cadd(e0, o0); u[4] = csub(e0, o0);
    u[1] = cadd(e1, o1); u[5] = csub(e1, o1);
    u[2] = cadd(e2, o2); u[6] = csub(e2, o2);
    u[3] = cadd(e3, o3); u[7] = csub(e3, o3);
}

// 16-point DFT as 4 x 4: X[k1 + 4 k2] = sum_n2 w4^(n2 k2) w16^(n2 k1) sum_n1 x[4 n1 + n2] w4^(n1 k1)
template <int S>
__device__ __forceinline__ void dft16(float2 (&u)[16]) {
#pragma unroll
    for (int n2 = 0; n2 < 4; ++n2) dft4<S>(u[n2], u[n2 + 4], u[n2 + 8], u[n2 + 12]);
    // after the first stage, u[n2 + 4 k1] holds A[n2][k1]; twiddle by w16^(n2 k1)
    u[1 + 4 * 1] = mul_cs<S>(u[1 + 4 * 1], kCos8, kSin8);      // w16^1
    u[1 + 4 * 2] = mul_w8<S>(u[1 + 4 * 2]);                     // w16^2
    u[1 + 4 * 3] = mul_cs<S>(u[1 + 4 * 3], kSin8, kCos8);      // w16^3
    u[2 + 4 * 1] = mul_w8<S>(u[2 + 4 * 1]);                     // w16^2
    u[2 + 4 * 2] = mul_sj<S>(u[2 + 4 * 2]);                     // w16^4
    u[2 + 4 * 3] = mul_w8_3<S>(u[2 + 4 * 3]);                   // w16^6
    u[3 + 4 * 1] = mul_cs<S>(u[3 + 4 * 1], kSin8, kCos8);      // w16^3
    u[3 + 4 * 2] = mul_w8_3<S>(u[3 + 4 * 2]);                   // w16^6
    u[3 + 4 * 3] = mul_cs<S>(u[3 + 4 * 3], -kCos8, -kSin8);    // w16^9
    // second stage over n2 for each k1; result X[k1 + 4 k2]
    float2 r[16];
#pragma unroll
    for (int k1 = 0; k1 < 4; ++k1) {
        float2 a0 = u[0 + 4 * k1], a1 = u[1 + 4 * k1], a2 = u[2 + 4 * k1], a3 = u[3 + 4 * k1];
        dft4<S>(a0, a1, a2, a3);
        r[k1 + 0] = a0;
        r[k1 + 4] = a1;
        r[k1 + 8] = a2;
        r[k1 + 12] = a3;
    }
#pragma unroll
    for (int i = 0; i < 16; ++i) u[i] = r[i];
}

template <int R, int S>
__device__ __forceinline__ void dft_r(float2 (&u)[R]) {
    if constexpr (R == 2) {
        dft2<S>(u[0], u[1]);
    } else if constexpr (R == 4) {
        dft4<S>(u[0], u[1], u[2], u[3]);
    } else if constexpr (R == 8) {
        dft8<S>(u);
    } else {
        static_assert(R == 16, "radix");
        dft16<S>(u);
    }
}

// ---------------------------------------------------------------- LDS exchange
__device__ __forceinline__ int pad16(int i) { return i + (i >> 4); }

template <int LOGN>
struct Fft {
    static constexpr int N = 1 << LOGN;
    static constexpr int NT = N / 16;                  // threads
    static constexpr int LDS = N + N / 16;             // padded complex elements
    static constexpr int P16 = LOGN / 4;               // radix-16 passes
    static constexpr int RLAST = 1 << (LOGN % 4);      // final radix (1: none)
    static_assert(LOGN >= 8 && LOGN <= 14, "transform size");

    // One Stockham pass on register data: butterflies b = t + q*NT, inputs v[q + r*16/R].
    template <int NS, int R, int S>
    __device__ __forceinline__ static void pass(float2 (&v)[16], const float2* __restrict__ tw, int t) {
        constexpr int NB = 16 / R;
#pragma unroll
        for (int q = 0; q < NB; ++q) {
            float2 u[R];
#pragma unroll
            for (int r = 0; r < R; ++r) u[r] = v[q + r * NB];
            if constexpr (NS > 1) {
                const int j = (t + q * NT) & (NS - 1);
#pragma unroll
                for (int r = 1; r < R; ++r) {
                    float2 w = tw[j * r * (N / (NS * R))];
                    if constexpr (S < 0) w.y = -w.y;
                    u[r] = cmul(u[r], w);
                }
            }
            dft_r<R, S>(u);
#pragma unroll
            for (int r = 0; r < R; ++r) v[q + r * NB] = u[r];
        }
    }

    template <int NS, int R>
    __device__ __forceinline__ static void store(const float2 (&v)[16], float2* lds, int t) {
        constexpr int NB = 16 / R;
#pragma unroll
        for (int q = 0; q < NB; ++q) {
            const int b = t + q * NT;
            const int base = (b / NS) * NS * R + (b & (NS - 1));
#pragma unroll
            for (int r = 0; r < R; ++r) lds[pad16(base + r * NS)] = v[q + r * NB];
        }
    }

    __device__ __forceinline__ static void load(float2 (&v)[16], const float2* lds, int t) {
#pragma unroll
        for (int m = 0; m < 16; ++m) v[m] = lds[pad16(t + m * NT)];
    }

    // Pass number P (0-based) of the sequence, with its span and radix.
    template <int P>
    struct Step {
        static constexpr int NS = 1 << (4 * P);
        static constexpr int R = (P < P16) ? 16 : RLAST;
        static constexpr bool LAST = (P == P16 - 1 && RLAST == 1) || (P == P16);
    };

    template <int P, int S>
    __device__ __forceinline__ static void run_from(float2 (&v)[16], float2* lds,
                                                    const float2* __restrict__ tw, int t) {
        using St = Step<P>;
        pass<St::NS, St::R, S>(v, tw, t);
        if constexpr (!St::LAST) {
            store<St::NS, St::R>(v, lds, t);
            __syncthreads();
            load(v, lds, t);
            __syncthreads();
            run_from<P + 1, S>(v, lds, tw, t);
        }
    }

    // Full transform.  On return every thread has finished reading LDS, so the
    // buffer may be rewritten immediately.
    template <int S>
    __device__ __forceinline__ static void transform(float2 (&v)[16], float2* lds,
                                                     const float2* __restrict__ tw, int t) {
        run_from<0, S>(v, lds, tw, t);
    }
};

}  // namespace dev
}  // namespace acq
