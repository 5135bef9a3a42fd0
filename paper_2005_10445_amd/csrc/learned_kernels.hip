// Kernels of the proposal stage (declarations and conventions in learned.h).
//
//   k_stft            256-point Hann-windowed FFT per frame (hop 128), one wave per
//                     frame, radix-4 Stockham passes exchanged through LDS; the
//                     samples come from a device block or from the synthetic
//                     generator (so training blocks never touch HBM)
//   k_hist/k_select   exact lower median of a block's F*256 powers: radix
//                     selection over the FP32 bit patterns (11 + 10 + 10 bits)
//   k_map             ln(P / median), stored bf16 (or FP32)
//   k_conv_tile       dilated conv layers as implicit GEMMs on bf16 MFMA
//                     (v_mfma_f32_16x16x32_bf16, FP32 accumulation): forward and
//                     input gradient
//   k_conv_dw_taps    weight gradient, all taps of a channel group per workgroup,
//                     on the same MFMA; k_dw_reduce adds the row-chunk sums
//   k_conv_*_ref      the same products in FP32 FMA, one output per thread
//                     (reference arithmetic for tests)
//   k_head            1x1 head, weighted BCE with logits and its gradient
//   k_adam            Adam update of the FP32 master weights, refreshing the
//                     bf16 copies in both operand layouts
//   k_window/k_propose window scores, frames at or above the threshold and the
//                     segment list
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cfloat>

#include "device_fft.h"
#include "learned.h"

namespace acq {
namespace learned {

NetLayout net_layout(int cin0) {
    NetLayout l{};
    int64_t off = 0, bf = 0;
    for (int i = 0; i < kLayers; ++i) {
        l.cin[i] = i == 0 ? cin0 : kCh;
        l.w_off[i] = off;
        off += int64_t(kTaps) * l.cin[i] * kCh;
        l.b_off[i] = off;
        off += kCh;
        l.bf_off[i] = bf;
        bf += int64_t(kTaps) * l.cin[i] * kCh;
    }
    l.wh_off = off;
    off += kCh;
    l.bh_off = off;
    off += 1;
    l.total = off;
    l.bf_total = bf;
    return l;
}

namespace {

using dev::cmul;
using bf16x4 = __attribute__((ext_vector_type(4))) short;
using f32x4 = __attribute__((ext_vector_type(4))) float;

__device__ __forceinline__ uint16_t to_bf16(float f) {
    const uint32_t u = __float_as_uint(f);
    return uint16_t((u + 0x7fffu + ((u >> 16) & 1u)) >> 16);   // nearest even (finite inputs)
}
__device__ __forceinline__ float from_bf16(uint16_t h) { return __uint_as_float(uint32_t(h) << 16); }

// ------------------------------------------------------------------ generator
// Philox4x32-10 (Salmon, Moraes, Dror and Shaw, SC'11).
struct P4 {
    uint32_t a, b, c, d;
};

__device__ __forceinline__ P4 philox10(P4 x, uint32_t k0, uint32_t k1) {
#pragma unroll
    for (int r = 0; r < 10; ++r) {
        const uint64_t p0 = uint64_t(0xD2511F53u) * x.a;
        const uint64_t p1 = uint64_t(0xCD9E8D57u) * x.c;
        x = P4{uint32_t(p1 >> 32) ^ x.b ^ k0, uint32_t(p1), uint32_t(p0 >> 32) ^ x.d ^ k1, uint32_t(p0)};
        k0 += 0x9E3779B9u;
        k1 += 0xBB67AE85u;
    }
    return x;
}

// Sample n of synthetic block b: CN(0,1) noise (Box-Muller on two 24-bit
// uniforms) plus every transmission covering n.
__device__ float2 synth_sample(const BlockSource& s, int b, int64_t n) {
    const int64_t blk = s.block0 + b;
    const P4 r = philox10(P4{uint32_t(n), uint32_t(n >> 32), uint32_t(blk), uint32_t(blk >> 32) ^ 0x4E4F4953u},
                          s.seed_lo, s.seed_hi);
    const float u1 = (float(r.a >> 8) + 0.5f) * (1.0f / 16777216.0f);     // (0, 1)
    const float u2 = float(r.b >> 8) * (1.0f / 16777216.0f);              // [0, 1)
    const float rad = sqrtf(-logf(u1));                                   // sqrt(-2 ln u1) / sqrt(2)
    float sn, cs;
    sincospif(2.0f * u2, &sn, &cs);
    float2 v = make_float2(rad * cs, rad * sn);
    const int nt = s.ntx[b];
    for (int t = 0; t < nt; ++t) {
        const SynthTx tx = s.tx[int64_t(b) * kMaxTx + t];
        const int64_t m = n - tx.delay;
        if (m < 0 || m >= s.chip_len) continue;
        const uint32_t c = uint32_t(m) / uint32_t(s.spc);     // 0 <= m < chip_len < 2^31
        const P4 q = philox10(P4{c >> 7, tx.code, uint32_t(blk), 0x43484950u}, s.seed_lo, s.seed_hi);
        const int w = int(c & 127);
        const uint32_t word = w < 32 ? q.a : w < 64 ? q.b : w < 96 ? q.c : q.d;
        const float chip = ((word >> (w & 31)) & 1u) ? 1.0f : -1.0f;
        double ph = tx.cycles_per_sample * double(n) + double(tx.phase0);
        ph -= floor(ph);
        float s2, c2;
        sincospif(2.0f * float(ph), &s2, &c2);
        v.x = fmaf(tx.amp * chip, c2, v.x);
        v.y = fmaf(tx.amp * chip, s2, v.y);
    }
    return v;
}

// ------------------------------------------------------------------ STFT
// Wave w of workgroup g transforms row 4g + w.  Lane l holds elements
// l + 64 r (r < 4) before and after each radix-4 pass (Stockham: pass with
// sub-transform length Ns reads a[j + 64 r], twiddles input r by
// exp(-j 2 pi r (j mod Ns) / (4 Ns)), and writes output r to
// (j / Ns) 4 Ns + (j mod Ns) + r Ns).
__global__ __launch_bounds__(256) void k_stft(BlockSource src, int nblocks, int64_t F, const float* __restrict__ hann,
                                              const float2* __restrict__ tw, float* __restrict__ P) {
    constexpr int kShared = 3 * kHop + kWin;   // samples of the workgroup's 4 frames
    __shared__ float2 buf[4][kWin];
    __shared__ float2 stw[kWin];
    __shared__ float swin[kWin];
    __shared__ float2 smp[kShared];
    const int tid = int(threadIdx.x), lane = tid & 63, wave = tid >> 6;
    stw[tid] = tw[tid];
    swin[tid] = hann[tid];
    const int64_t total = int64_t(nblocks) * F;
    // generated blocks: when the 4 frames lie in one block, each of their
    // samples is generated once (frames overlap by half) and shared through LDS
    const int64_t row0 = int64_t(blockIdx.x) * 4;
    const int gb = int(row0 / F);
    const int64_t gf = row0 - int64_t(gb) * F;
    const bool shared_gen = !src.x && row0 + 3 < total && gf + 3 < F;    // uniform
    if (shared_gen)
        for (int j = tid; j < kShared; j += 256) smp[j] = synth_sample(src, gb, gf * kHop + j);
    __syncthreads();
    const int64_t row = row0 + wave;
    const bool live = row < total;
    const int64_t rr = live ? row : total - 1;
    const int b = int(rr / F);
    const int64_t f = rr - int64_t(b) * F;
    float2 a[4];
#pragma unroll
    for (int r = 0; r < 4; ++r) {
        const int j = lane + 64 * r;
        const int64_t n = f * kHop + j;
        const float2 x = src.x ? src.x[int64_t(b) * src.stride + n]
                               : shared_gen ? smp[wave * kHop + j] : synth_sample(src, b, n);
        a[r] = make_float2(x.x * swin[j], x.y * swin[j]);
    }
    float2* X = buf[wave];
#pragma unroll
    for (int Ns = 1; Ns < kWin; Ns *= 4) {
        const int k = lane & (Ns - 1);
        const int step = 64 / Ns;
#pragma unroll
        for (int r = 1; r < 4; ++r) a[r] = cmul(a[r], stw[(r * k * step) & (kWin - 1)]);
        dev::dft4<-1>(a[0], a[1], a[2], a[3]);
        if (Ns < 64) {
            const int o = (lane / Ns) * Ns * 4 + k;
#pragma unroll
            for (int r = 0; r < 4; ++r) X[o + r * Ns] = a[r];
            __syncthreads();
#pragma unroll
            for (int r = 0; r < 4; ++r) a[r] = X[lane + 64 * r];
            __syncthreads();
        }
    }
    if (live) {
#pragma unroll
        for (int r = 0; r < 4; ++r) P[row * kWin + lane + 64 * r] = fmaf(a[r].x, a[r].x, a[r].y * a[r].y);
    }
}

// ------------------------------------------------------------------ median
__global__ void k_median_init(MedianState* st, int nblocks, uint32_t rank) {
    const int b = int(blockIdx.x * blockDim.x + threadIdx.x);
    if (b < nblocks) st[b] = MedianState{0u, rank};
}

// pass 0: digit = bits[30:20]; pass 1: bits[19:10] of values whose bits[30:20]
// equal the prefix; pass 2: bits[9:0] of values whose bits[30:10] match.
__global__ __launch_bounds__(256) void k_hist(const float* __restrict__ P, int64_t per_block, int pass,
                                              const MedianState* __restrict__ st, uint32_t* __restrict__ hist) {
    __shared__ uint32_t h[2048];
    for (int i = int(threadIdx.x); i < 2048; i += 256) h[i] = 0u;
    __syncthreads();
    const int b = int(blockIdx.y);
    const uint32_t prefix = st[b].prefix;
    const float* p = P + int64_t(b) * per_block;
    // 8 loads in flight per thread before their histogram updates
    const int64_t stride = int64_t(gridDim.x) * 256;
    for (int64_t i0 = int64_t(blockIdx.x) * 256 + threadIdx.x; i0 < per_block; i0 += 8 * stride) {
        uint32_t u[8];
#pragma unroll
        for (int k = 0; k < 8; ++k) {
            const int64_t i = i0 + k * stride;
            u[k] = i < per_block ? __float_as_uint(p[i]) : 0u;
        }
#pragma unroll
        for (int k = 0; k < 8; ++k) {
            if (i0 + k * stride >= per_block) break;
            uint32_t digit;
            bool match;
            if (pass == 0) {
                digit = u[k] >> 20;
                match = true;
            } else if (pass == 1) {
                digit = (u[k] >> 10) & 1023u;
                match = (u[k] >> 20) == prefix;
            } else {
                digit = u[k] & 1023u;
                match = (u[k] >> 10) == prefix;
            }
            if (match) atomicAdd(&h[digit], 1u);
        }
    }
    __syncthreads();
    for (int i = int(threadIdx.x); i < 2048; i += 256)
        if (h[i]) atomicAdd(&hist[int64_t(b) * 2048 + i], h[i]);
}

// One workgroup per block: find the bucket holding the wanted rank, extend the
// prefix, and clear the histogram for the next pass.
__global__ __launch_bounds__(256) void k_select(uint32_t* __restrict__ hist, int pass, MedianState* __restrict__ st,
                                                float* __restrict__ med) {
    __shared__ uint32_t part[256];
    const int b = int(blockIdx.x), t = int(threadIdx.x);
    const MedianState s = st[b];
    uint32_t* h = hist + int64_t(b) * 2048;
    const int per = pass == 0 ? 8 : 4;
    uint32_t local[8];
    uint32_t sum = 0;
    for (int q = 0; q < per; ++q) {
        local[q] = h[t * per + q];
        sum += local[q];
    }
    part[t] = sum;
    __syncthreads();
    for (int off = 1; off < 256; off <<= 1) {
        const uint32_t v = t >= off ? part[t - off] : 0u;
        __syncthreads();
        part[t] += v;
        __syncthreads();
    }
    const uint32_t incl = part[t], excl = incl - sum;
    if (s.rank >= excl && s.rank < incl) {
        uint32_t c = excl, digit = 0, rank = 0;
        for (int q = 0; q < per; ++q) {
            if (s.rank < c + local[q]) {
                digit = uint32_t(t * per + q);
                rank = s.rank - c;
                break;
            }
            c += local[q];
        }
        const uint32_t prefix = pass == 0 ? digit : (s.prefix << 10) | digit;
        st[b] = MedianState{prefix, rank};
        if (pass == 2) med[b] = __uint_as_float(prefix);
    }
    for (int q = 0; q < per; ++q) h[t * per + q] = 0u;
}

// four values per thread (one block's median when per_block is a multiple of 4)
template <bool BF>
__global__ void k_map(const float* __restrict__ P, int64_t per_block, int64_t total, const float* __restrict__ med,
                      void* __restrict__ out) {
    const int64_t i0 = (int64_t(blockIdx.x) * blockDim.x + threadIdx.x) * 4;
    if (i0 >= total) return;
    auto value = [&](float p, float m) { return m > 0.0f ? logf(fmaxf(p, FLT_MIN) / m) : 0.0f; };
    if (per_block % 4 == 0 && i0 + 4 <= total) {
        const float m = med[i0 / per_block];
        const float4 p = *reinterpret_cast<const float4*>(P + i0);
        const float v0 = value(p.x, m), v1 = value(p.y, m), v2 = value(p.z, m), v3 = value(p.w, m);
        if constexpr (BF)
            *reinterpret_cast<uint2*>(static_cast<uint16_t*>(out) + i0) =
                uint2{uint32_t(to_bf16(v0)) | (uint32_t(to_bf16(v1)) << 16),
                      uint32_t(to_bf16(v2)) | (uint32_t(to_bf16(v3)) << 16)};
        else
            *reinterpret_cast<float4*>(static_cast<float*>(out) + i0) = float4{v0, v1, v2, v3};
        return;
    }
    for (int64_t i = i0; i < i0 + 4 && i < total; ++i) {
        const float v = value(P[i], med[i / per_block]);
        if constexpr (BF)
            static_cast<uint16_t*>(out)[i] = to_bf16(v);
        else
            static_cast<float*>(out)[i] = v;
    }
}

__global__ void k_synth(BlockSource src, int64_t n, float2* __restrict__ out) {
    const int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (i < n) out[i] = synth_sample(src, 0, i);
}

// 1 when at least half of the frame lies inside some transmission: the frame's
// samples covered by the union of the transmissions, as a 256-bit mask.
__global__ void k_labels(const SynthTx* __restrict__ tx, const int32_t* __restrict__ ntx, int64_t rows, int64_t F,
                         int L, float* __restrict__ labels) {
    const int64_t r = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (r >= rows) return;
    const int b = int(r / F);
    const int64_t f0 = (r - int64_t(b) * F) * kHop;
    const int nt = ntx[b];
    constexpr int kWords = kWin / 32;
    uint32_t cov[kWords];
#pragma unroll
    for (int w = 0; w < kWords; ++w) cov[w] = 0u;
    for (int t = 0; t < nt; ++t) {
        const int64_t d = tx[int64_t(b) * kMaxTx + t].delay;
        const int64_t lo = (d > f0 ? d : f0) - f0;                               // [lo, hi) of the frame
        const int64_t hi = (d + L < f0 + kWin ? d + L : f0 + kWin) - f0;
        if (lo >= hi) continue;
#pragma unroll
        for (int w = 0; w < kWords; ++w) {
            const int a = int(lo - 32 * w > 0 ? lo - 32 * w : 0);
            const int e = int(hi - 32 * w < 32 ? hi - 32 * w : 32);
            if (a < e) cov[w] |= (e - a == 32 ? 0xffffffffu : ((1u << (e - a)) - 1u) << a);
        }
    }
    int covered = 0;
#pragma unroll
    for (int w = 0; w < kWords; ++w) covered += __popc(cov[w]);
    labels[r] = covered >= kWin / 2 ? 1.0f : 0.0f;
}

// ------------------------------------------------------------------ conv (MFMA)
// Forward / input gradient as a tiled GEMM on v_mfma_f32_16x16x32_bf16
// (lane l: A[row l%16][k 8(l/16)+e], B[k 8(l/16)+e][col l%16], e < 8;
// D[row 4(l/16)+e][col l%16], e < 4).  A workgroup computes 128 rows x 64
// columns.  The rows it needs for all five taps -- its 128 plus 2d above and
// below -- are staged once in LDS as bf16 ([row][K + 8], the pad spreading
// the 16-byte reads of a wave over the banks); for the input gradient the
// staging applies the ReLU mask to dH and rounds it once.  Each wave takes
// 32 rows (two 16-row tiles) by the 64 columns (four 16-column tiles); the
// weights of the next 32-deep k step are loaded while the current step's
// eight MFMAs run.  A tap row outside its output row's block is zero.
constexpr int kTileRows = 128;

using bf16x8 = __attribute__((__vector_size__(8 * sizeof(__bf16)))) __bf16;

__device__ __forceinline__ bf16x8 as_bf16x8(uint4 v) { return __builtin_bit_cast(bf16x8, v); }

template <bool FWD>
__global__ __launch_bounds__(256) void k_conv_tile(const void* __restrict__ src, const uint16_t* __restrict__ H,
                                                   int K, const uint16_t* __restrict__ Bt,
                                                   const float* __restrict__ bias, void* __restrict__ out,
                                                   int64_t rows, int64_t F, int d) {
    extern __shared__ __align__(16) uint16_t sA[];
    const int tid = int(threadIdx.x), lane = tid & 63, wave = tid >> 6;
    const int pitch = K + 8, halo = 2 * d, srows = kTileRows + 2 * halo;
    const int64_t r0 = int64_t(blockIdx.x) * kTileRows;
    if constexpr (FWD) {
        const int cpr = K / 8;                           // 16-byte chunks per row
        for (int idx = tid; idx < srows * cpr; idx += 256) {
            const int sr = idx / cpr, ch = idx - sr * cpr;
            const int64_t g = r0 - halo + sr;
            uint4 v = {0u, 0u, 0u, 0u};
            if (g >= 0 && g < rows) v = *reinterpret_cast<const uint4*>(static_cast<const uint16_t*>(src) + g * K + ch * 8);
            *reinterpret_cast<uint4*>(&sA[sr * pitch + ch * 8]) = v;
        }
    } else {
        const int cpr = K / 4;                           // 4 values per thread and step
        for (int idx = tid; idx < srows * cpr; idx += 256) {
            const int sr = idx / cpr, ch = idx - sr * cpr;
            const int64_t g = r0 - halo + sr;
            uint2 o = {0u, 0u};
            if (g >= 0 && g < rows) {
                const float4 gv = *reinterpret_cast<const float4*>(static_cast<const float*>(src) + g * K + ch * 4);
                const uint2 hb = *reinterpret_cast<const uint2*>(H + g * K + ch * 4);
                // dA = dH where the layer output is positive
                const float g0 = (hb.x & 0x7fffu) && !(hb.x & 0x8000u) ? gv.x : 0.f;
                const float g1 = (hb.x & 0x7fff0000u) && !(hb.x & 0x80000000u) ? gv.y : 0.f;
                const float g2 = (hb.y & 0x7fffu) && !(hb.y & 0x8000u) ? gv.z : 0.f;
                const float g3 = (hb.y & 0x7fff0000u) && !(hb.y & 0x80000000u) ? gv.w : 0.f;
                o.x = uint32_t(to_bf16(g0)) | (uint32_t(to_bf16(g1)) << 16);
                o.y = uint32_t(to_bf16(g2)) | (uint32_t(to_bf16(g3)) << 16);
            }
            *reinterpret_cast<uint2*>(&sA[sr * pitch + ch * 4]) = o;
        }
    }
    __syncthreads();

    const int ra = lane & 15, kq = 8 * (lane >> 4);
    int64_t frame[2];
    bool live[2];
#pragma unroll
    for (int rt = 0; rt < 2; ++rt) {
        const int64_t orow = r0 + 32 * wave + 16 * rt + ra;
        live[rt] = orow < rows;
        frame[rt] = orow - (orow / F) * F;
    }
    f32x4 acc[2][4];
#pragma unroll
    for (int rt = 0; rt < 2; ++rt)
#pragma unroll
        for (int nt = 0; nt < 4; ++nt) acc[rt][nt] = f32x4{0.f, 0.f, 0.f, 0.f};
    const int ksteps = K / 32, steps = kTaps * ksteps;
    auto bptr = [&](int step, int nt) {
        const int i = step / ksteps, kc = (step - i * ksteps) * 32;
        return Bt + (int64_t(i) * kCh + nt * 16 + ra) * K + kc + kq;
    };
    uint4 bcur[4];
#pragma unroll
    for (int nt = 0; nt < 4; ++nt) bcur[nt] = *reinterpret_cast<const uint4*>(bptr(0, nt));
    for (int step = 0; step < steps; ++step) {
        uint4 bnext[4];
        const int sn = step + 1 < steps ? step + 1 : step;
#pragma unroll
        for (int nt = 0; nt < 4; ++nt) bnext[nt] = *reinterpret_cast<const uint4*>(bptr(sn, nt));
        const int i = step / ksteps, kc = (step - i * ksteps) * 32;
        const int delta = (FWD ? 1 : -1) * d * (i - 2);
        bf16x8 a[2];
#pragma unroll
        for (int rt = 0; rt < 2; ++rt) {
            const int arow = 32 * wave + 16 * rt + ra + halo + delta;
            const uint4 v = *reinterpret_cast<const uint4*>(&sA[arow * pitch + kc + kq]);
            const bool ok = live[rt] && frame[rt] + delta >= 0 && frame[rt] + delta < F;
            a[rt] = as_bf16x8(ok ? v : uint4{0u, 0u, 0u, 0u});
        }
#pragma unroll
        for (int rt = 0; rt < 2; ++rt)
#pragma unroll
            for (int nt = 0; nt < 4; ++nt)
                acc[rt][nt] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[rt], as_bf16x8(bcur[nt]), acc[rt][nt], 0, 0, 0);
#pragma unroll
        for (int nt = 0; nt < 4; ++nt) bcur[nt] = bnext[nt];
    }
#pragma unroll
    for (int rt = 0; rt < 2; ++rt)
#pragma unroll
        for (int nt = 0; nt < 4; ++nt) {
            const int n = nt * 16 + ra;
            const float bn = FWD ? bias[n] : 0.0f;
#pragma unroll
            for (int e = 0; e < 4; ++e) {
                const int64_t row = r0 + 32 * wave + 16 * rt + 4 * (lane >> 4) + e;
                if (row >= rows) continue;
                if constexpr (FWD)
                    static_cast<uint16_t*>(out)[row * kCh + n] = to_bf16(fmaxf(acc[rt][nt][e] + bn, 0.0f));
                else
                    static_cast<float*>(out)[row * kCh + n] = acc[rt][nt][e];
            }
        }
}

__host__ __device__ constexpr size_t conv_tile_lds(int K, int d) {
    return size_t(kTileRows + 4 * d) * size_t(K + 8) * sizeof(uint16_t);
}
constexpr size_t kMaxConvLds = size_t(160) << 10;   // LDS of a gfx950 compute unit

// Weight gradient dW[i][c][o] += sum_r in[r + d(i-2)][c] dA[r][o] (dA = dH where the
// layer output is positive) on v_mfma_f32_16x16x32_bf16 (lane l: A[row l%16][k
// 8(l/16)+e], B[k 8(l/16)+e][col l%16], e < 8; D[row 4(l/16)+e][col l%16], e < 4),
// all five taps of 64 input channels in one workgroup.  Rows come in 64-row
// pieces: the piece's dA rows and the input rows it reaches (2D before, 2D after)
// are staged once in LDS, transposed to [channel][row] so that an operand's 8
// consecutive rows are one read, and every tap reads the input tile at its own
// row shift D*i.  Wave w holds the 16 channels 16w.. of every tap and output
// channel (20 accumulator tiles); the sums stay in registers over the chunk and
// are stored once as the chunk's sums, which k_dw_reduce adds up in a fixed
// order (atomic adds of every chunk's sums cost more than the products).  A pair (r, r + D(i-2)) whose rows lie in different
// blocks contributes nothing: pieces with no block start near them need no
// test, the others clear those operand rows tap by tap.
constexpr int kDwRows = 64;
constexpr int kDwPitchD = 72;    // dA tile row: 64 rows + 8 pad (bf16), 36 dwords = 4 x odd
constexpr int kDwPitchI = 104;   // input tile row: 64 + 4 * 8 rows + 8 pad, 52 dwords = 4 x odd, so
                                 // the 16 channels of an operand read fall on distinct banks
constexpr int kDwXcds = 8;       // workgroups go to the XCDs in turn
constexpr int kDwWgs = 256;      // workgroups per call (one per CU): sets the rows per workgroup
constexpr int kDwBlock = kTaps * 64 * kCh;   // sums of one chunk and 64-channel group

// 8 bf16 of LDS row `p` starting SHIFT elements past a 16-byte boundary
template <int SHIFT>
__device__ __forceinline__ uint4 lds_row8(const uint16_t* p) {
    p += (SHIFT / 8) * 8;
    constexpr int s = SHIFT % 8;
    if constexpr (s == 0) {
        return *reinterpret_cast<const uint4*>(p);
    } else if constexpr (s % 4 == 0) {
        const uint2* q = reinterpret_cast<const uint2*>(p) + s / 4;
        const uint2 a = q[0], b = q[1];
        return uint4{a.x, a.y, b.x, b.y};
    } else if constexpr (s % 2 == 0) {
        const uint32_t* q = reinterpret_cast<const uint32_t*>(p) + s / 2;
        return uint4{q[0], q[1], q[2], q[3]};
    } else {                                     // odd: five dwords, each pair funnel-shifted by 16 bits
        const uint32_t* q = reinterpret_cast<const uint32_t*>(p) + s / 2;
        const uint32_t w0 = q[0], w1 = q[1], w2 = q[2], w3 = q[3], w4 = q[4];
        return uint4{__builtin_amdgcn_alignbit(w1, w0, 16), __builtin_amdgcn_alignbit(w2, w1, 16),
                     __builtin_amdgcn_alignbit(w3, w2, 16), __builtin_amdgcn_alignbit(w4, w3, 16)};
    }
}

template <int D>
__global__ __launch_bounds__(256, 2) void k_conv_dw_taps(const uint16_t* __restrict__ in, int cin,
                                                      const float* __restrict__ dH, const uint16_t* __restrict__ H,
                                                      float* __restrict__ part, float* __restrict__ pdb, int64_t rows,
                                                      int64_t F, int chunk, int nchunks) {
    static_assert(64 + 4 * D + 8 <= kDwPitchI, "input tile row too short for the dilation");
    __shared__ __align__(16) uint16_t sD[64 * kDwPitchD];
    __shared__ __align__(16) uint16_t sI[64 * kDwPitchI];
    __shared__ float sdb[16][64];
    const int tid = int(threadIdx.x), lane = tid & 63, wave = tid >> 6;
    // workgroup -> (chunk, channel group); the groups of one chunk share an XCD and its L2
    const int ngroups = cin / 64;
    const int wg = int(blockIdx.x), s = wg / kDwXcds;
    const int ck = (s / ngroups) * kDwXcds + wg % kDwXcds, c0 = (s % ngroups) * 64;
    if (ck >= nchunks) return;                   // uniform: padding of the grid
    const bool bias = pdb && c0 == 0;
    // staging: thread -> 4 consecutive rows (j) x 4 consecutive channels (q)
    const int j = tid >> 4, q = tid & 15;
    float dbs[4] = {0.f, 0.f, 0.f, 0.f};
    f32x4 acc[kTaps][4];
#pragma unroll
    for (int i = 0; i < kTaps; ++i)
#pragma unroll
        for (int nt = 0; nt < 4; ++nt) acc[i][nt] = f32x4{0.f, 0.f, 0.f, 0.f};
    const int F32 = int(F);
    const int64_t rend = min(rows, int64_t(ck + 1) * chunk);
    // one piece's staging loads, held in registers so that the next piece's are
    // in flight while this one's products run: dA rows rb + 4j + e, channels 4q..;
    // input row groups j and j + 16 (rows rb - 2D + 4jj + e; zero outside [0, rows))
    float4 pg[4];
    uint2 ph[4], px[2][4];
    auto fetch = [&](int64_t rb) {
#pragma unroll
        for (int e = 0; e < 4; ++e) {
            const int64_t r = rb + 4 * j + e;
            pg[e] = float4{0.f, 0.f, 0.f, 0.f};
            ph[e] = uint2{0u, 0u};
            if (r < rend) {
                pg[e] = *reinterpret_cast<const float4*>(dH + r * kCh + 4 * q);
                ph[e] = *reinterpret_cast<const uint2*>(H + r * kCh + 4 * q);
            }
        }
#pragma unroll
        for (int h = 0; h < 2; ++h)
#pragma unroll
            for (int e = 0; e < 4; ++e) {
                const int jj = j + 16 * h;
                const int64_t g = rb - 2 * D + 4 * jj + e;
                px[h][e] = uint2{0u, 0u};
                if (jj < 16 + D && g >= 0 && g < rows)
                    px[h][e] = *reinterpret_cast<const uint2*>(in + g * cin + c0 + 4 * q);
            }
    };
    // dA = dH where the layer output is positive, to bf16, as sD[channel][row];
    // the input as sI[channel][row - (rb - 2D)]
    auto stage = [&]() {
        uint16_t v[4][4];
#pragma unroll
        for (int e = 0; e < 4; ++e) {
            const float4 g = pg[e];
            const uint2 hb = ph[e];
            const float g0 = (hb.x & 0x7fffu) && !(hb.x & 0x8000u) ? g.x : 0.f;
            const float g1 = (hb.x & 0x7fff0000u) && !(hb.x & 0x80000000u) ? g.y : 0.f;
            const float g2 = (hb.y & 0x7fffu) && !(hb.y & 0x8000u) ? g.z : 0.f;
            const float g3 = (hb.y & 0x7fff0000u) && !(hb.y & 0x80000000u) ? g.w : 0.f;
            dbs[0] += g0;
            dbs[1] += g1;
            dbs[2] += g2;
            dbs[3] += g3;
            v[0][e] = to_bf16(g0);
            v[1][e] = to_bf16(g1);
            v[2][e] = to_bf16(g2);
            v[3][e] = to_bf16(g3);
        }
#pragma unroll
        for (int k = 0; k < 4; ++k)
            *reinterpret_cast<uint2*>(&sD[(4 * q + k) * kDwPitchD + 4 * j]) =
                uint2{uint32_t(v[k][0]) | (uint32_t(v[k][1]) << 16), uint32_t(v[k][2]) | (uint32_t(v[k][3]) << 16)};
#pragma unroll
        for (int h = 0; h < 2; ++h) {
            const int jj = j + 16 * h;
            if (jj >= 16 + D) break;
#pragma unroll
            for (int k = 0; k < 4; ++k) {
                const int sh = 16 * (k & 1), w = k >> 1;
                auto half = [&](int e) { return ((w ? px[h][e].y : px[h][e].x) >> sh) & 0xffffu; };
                *reinterpret_cast<uint2*>(&sI[(4 * q + k) * kDwPitchI + 4 * jj]) =
                    uint2{half(0) | (half(1) << 16), half(2) | (half(3) << 16)};
            }
        }
    };
    int64_t rbase = int64_t(ck) * chunk;
    if (rbase < rend) fetch(rbase);
    for (; rbase < rend; rbase += kDwRows) {
        stage();
        __syncthreads();
        if (rbase + kDwRows < rend) fetch(rbase + kDwRows);
        // no block start in (rbase - 2D, rbase + 64 + 2D): every pair of the piece is in one block
        const int f0 = int(rbase % F);
        const bool clean = f0 >= 2 * D && F32 - f0 >= kDwRows + 2 * D;
        const uint16_t* arow = &sI[(16 * wave + (lane & 15)) * kDwPitchI + 8 * (lane >> 4)];
        const uint16_t* brow = &sD[(lane & 15) * kDwPitchD + 8 * (lane >> 4)];
#pragma unroll
        for (int ks = 0; ks < kDwRows; ks += 32) {
            bf16x8 b[4];
#pragma unroll
            for (int nt = 0; nt < 4; ++nt)
                b[nt] = as_bf16x8(*reinterpret_cast<const uint4*>(brow + 16 * nt * kDwPitchD + ks));
            uint4 a[kTaps];
            a[0] = lds_row8<0 * D>(arow + ks);
            a[1] = lds_row8<1 * D>(arow + ks);
            a[2] = lds_row8<2 * D>(arow + ks);
            a[3] = lds_row8<3 * D>(arow + ks);
            a[4] = lds_row8<4 * D>(arow + ks);
            if (!clean) {
                // clear the rows r of this lane (ks + 8(l/16) + e) whose tap row is in another block
                int fr = f0 + ks + 8 * (lane >> 4);
                while (fr >= F32) fr -= F32;
                int frs[8];
#pragma unroll
                for (int e = 0; e < 8; ++e) {
                    frs[e] = fr;
                    fr = fr + 1 == F32 ? 0 : fr + 1;
                }
#pragma unroll
                for (int i = 0; i < kTaps; ++i) {
                    uint32_t m[4];
#pragma unroll
                    for (int h = 0; h < 4; ++h) {
                        const int t0 = frs[2 * h] + D * (i - 2), t1 = frs[2 * h + 1] + D * (i - 2);
                        m[h] = (t0 >= 0 && t0 < F32 ? 0x0000ffffu : 0u) | (t1 >= 0 && t1 < F32 ? 0xffff0000u : 0u);
                    }
                    a[i].x &= m[0];
                    a[i].y &= m[1];
                    a[i].z &= m[2];
                    a[i].w &= m[3];
                }
            }
#pragma unroll
            for (int i = 0; i < kTaps; ++i)
#pragma unroll
                for (int nt = 0; nt < 4; ++nt)
                    acc[i][nt] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(as_bf16x8(a[i]), b[nt], acc[i][nt], 0, 0, 0);
        }
        __syncthreads();                         // the tiles are restaged by the next piece
    }
    // this chunk's sums: [tap][channel of the group][output channel]
    float* P = part + (int64_t(ck) * ngroups + c0 / 64) * kDwBlock;
#pragma unroll
    for (int i = 0; i < kTaps; ++i)
#pragma unroll
        for (int nt = 0; nt < 4; ++nt)
#pragma unroll
            for (int e = 0; e < 4; ++e) {
                const int c = 16 * wave + 4 * (lane >> 4) + e;
                P[(i * 64 + c) * kCh + 16 * nt + (lane & 15)] = acc[i][nt][e];
            }
    if (bias) {                                  // uniform over the workgroup
#pragma unroll
        for (int k = 0; k < 4; ++k) sdb[j][4 * q + k] = dbs[k];
        __syncthreads();
        if (tid < 64) {
            float t = 0.0f;
#pragma unroll
            for (int jj = 0; jj < 16; ++jj) t += sdb[jj][tid];
            pdb[int64_t(ck) * kCh + tid] = t;
        }
    }
}

// dW[i][c][o] += sum over chunks of their sums, and db[o] likewise (the last
// workgroup): workgroup (i, c) takes the 64 outputs of one row, thread (s, o4) the
// chunks s, s + 16, ... of 4 outputs, then the 16 partial sums are added in order.
__global__ __launch_bounds__(256) void k_dw_reduce(const float* __restrict__ part, const float* __restrict__ pdb,
                                                   float* __restrict__ dW, float* __restrict__ db, int cin,
                                                   int nchunks) {
    __shared__ float4 red[16][16];
    const int tid = int(threadIdx.x), s = tid >> 4, o4 = tid & 15;
    const int row = int(blockIdx.x);             // i * cin + c, or the bias row after them
    const int ngroups = cin / 64;
    const bool brow = row == kTaps * cin;
    const float* src;
    int64_t stride;
    if (brow) {
        src = pdb + 4 * o4;
        stride = kCh;
    } else {
        const int i = row / cin, c = row - i * cin;
        src = part + int64_t(c / 64) * kDwBlock + (i * 64 + c % 64) * kCh + 4 * o4;
        stride = int64_t(ngroups) * kDwBlock;
    }
    float4 t = {0.f, 0.f, 0.f, 0.f};
    for (int k = s; k < nchunks; k += 16) {
        const float4 v = *reinterpret_cast<const float4*>(src + k * stride);
        t.x += v.x;
        t.y += v.y;
        t.z += v.z;
        t.w += v.w;
    }
    red[s][o4] = t;
    __syncthreads();
    if (tid < 16) {
        float4 u = red[0][tid];
        for (int k = 1; k < 16; ++k) {
            u.x += red[k][tid].x;
            u.y += red[k][tid].y;
            u.z += red[k][tid].z;
            u.w += red[k][tid].w;
        }
        float* dst = brow ? db + 4 * tid : dW + int64_t(row) * kCh + 4 * tid;
        dst[0] += u.x;
        dst[1] += u.y;
        dst[2] += u.z;
        dst[3] += u.w;
    }
}

// ------------------------------------------------------------------ conv (FP32 reference)
// out[r][o] = relu(b[o] + sum_i sum_c W[i][c][o] in[r + d(i-2)][c]), W FP32 [5][cin][64].
__global__ void k_conv_fwd_ref(const float* __restrict__ in, int cin, const float* __restrict__ W,
                               const float* __restrict__ bias, float* __restrict__ out, int64_t rows, int64_t F,
                               int d) {
    const int64_t t = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (t >= rows * kCh) return;
    const int64_t r = t / kCh;
    const int o = int(t % kCh);
    const int64_t blk = r / F, f = r - blk * F;
    float acc = bias[o];
    for (int i = 0; i < kTaps; ++i) {
        const int64_t fs = f + int64_t(d) * (i - 2);
        if (fs < 0 || fs >= F) continue;
        const float* a = in + (blk * F + fs) * cin;
        for (int c = 0; c < cin; ++c) acc = fmaf(a[c], W[(int64_t(i) * cin + c) * kCh + o], acc);
    }
    out[t] = fmaxf(acc, 0.0f);
}

__global__ void k_conv_dinput_ref(const float* __restrict__ dH, const float* __restrict__ H,
                                  const float* __restrict__ W, float* __restrict__ dprev, int64_t rows, int64_t F,
                                  int d) {
    const int64_t t = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (t >= rows * kCh) return;
    const int64_t r = t / kCh;
    const int c = int(t % kCh);
    const int64_t blk = r / F, f = r - blk * F;
    float acc = 0.0f;
    for (int i = 0; i < kTaps; ++i) {
        const int64_t fs = f - int64_t(d) * (i - 2);
        if (fs < 0 || fs >= F) continue;
        const int64_t sr = blk * F + fs;
        for (int o = 0; o < kCh; ++o) {
            const float g = H[sr * kCh + o] > 0.0f ? dH[sr * kCh + o] : 0.0f;
            acc = fmaf(W[(int64_t(i) * kCh + c) * kCh + o], g, acc);
        }
    }
    dprev[t] = acc;
}

// thread per (i, c, o); the first kCh threads of each tap also form db
__global__ void k_conv_dw_ref(const float* __restrict__ in, int cin, const float* __restrict__ dH,
                              const float* __restrict__ H, float* __restrict__ dW, float* __restrict__ db,
                              int64_t rows, int64_t F, int d) {
    const int64_t t = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (t >= int64_t(kTaps) * cin * kCh) return;
    const int o = int(t % kCh);
    const int c = int((t / kCh) % cin);
    const int i = int(t / (int64_t(kCh) * cin));
    float acc = 0.0f, bacc = 0.0f;
    for (int64_t r = 0; r < rows; ++r) {
        const float g = H[r * kCh + o] > 0.0f ? dH[r * kCh + o] : 0.0f;
        bacc += g;
        const int64_t blk = r / F, f = r - blk * F, fs = f + int64_t(d) * (i - 2);
        if (fs < 0 || fs >= F) continue;
        acc = fmaf(in[(blk * F + fs) * cin + c], g, acc);
    }
    dW[t] += acc;
    if (i == 0 && c == 0) db[o] += bacc;
}

// db[o] += sum_r dA[r][o] (bf16 activations)

// ------------------------------------------------------------------ head and loss
__device__ __forceinline__ float softplus(float x) { return fmaxf(x, 0.0f) + log1pf(expf(-fabsf(x))); }

// Head and loss.  Sixteen lanes share a row, each holding four of its 64
// channels (coalesced reads of the layer output and writes of dH4): the
// logit is a 16-lane sum; the head-weight gradient is kept per lane over the
// workgroup's rows and added over its 16 row slots in LDS at the end.
constexpr int kHeadRows = 256;          // rows per workgroup

template <bool BF>
__global__ __launch_bounds__(256) void k_head(const void* __restrict__ h4, const float* __restrict__ theta,
                                              int64_t wh_off, float* __restrict__ y, const float* __restrict__ labels,
                                              float pw, float inv_rows, float* __restrict__ dH4,
                                              float* __restrict__ grad, float* __restrict__ loss_sum, int64_t rows) {
    __shared__ float sdw[16][kCh + 1];
    __shared__ float sred[2][16];
    const int t = int(threadIdx.x), j = t & 15, slot = t >> 4;
    float w[4];
#pragma unroll
    for (int c = 0; c < 4; ++c) w[c] = theta[wh_off + 4 * j + c];
    const float bias = theta[wh_off + kCh];
    float dw[4] = {0.f, 0.f, 0.f, 0.f};
    float dzs = 0.0f, ls = 0.0f;
    const int64_t rbase = int64_t(blockIdx.x) * kHeadRows;
    for (int rr = 0; rr < kHeadRows; rr += 16) {
        const int64_t r = rbase + rr + slot;
        const bool ok = r < rows;
        float h[4] = {0.f, 0.f, 0.f, 0.f};
        if (ok) {
            if constexpr (BF) {
                const uint2 v = *reinterpret_cast<const uint2*>(static_cast<const uint16_t*>(h4) + r * kCh + 4 * j);
                h[0] = __uint_as_float(v.x << 16);
                h[1] = __uint_as_float(v.x & 0xffff0000u);
                h[2] = __uint_as_float(v.y << 16);
                h[3] = __uint_as_float(v.y & 0xffff0000u);
            } else {
                const float4 v = *reinterpret_cast<const float4*>(static_cast<const float*>(h4) + r * kCh + 4 * j);
                h[0] = v.x; h[1] = v.y; h[2] = v.z; h[3] = v.w;
            }
        }
        float z = fmaf(h[3], w[3], fmaf(h[2], w[2], fmaf(h[1], w[1], h[0] * w[0])));
#pragma unroll
        for (int off = 8; off > 0; off >>= 1) z += __shfl_xor(z, off, 16);
        z += bias;
        if (ok && j == 0) y[r] = z;
        if (!labels) continue;     // uniform: inference
        if (ok) {
            const float lab = labels[r];
            const float sg = 1.0f / (1.0f + expf(-z));
            const float dz = (pw * lab * (sg - 1.0f) + (1.0f - lab) * sg) * inv_rows;
            *reinterpret_cast<float4*>(dH4 + r * kCh + 4 * j) = make_float4(dz * w[0], dz * w[1], dz * w[2], dz * w[3]);
#pragma unroll
            for (int c = 0; c < 4; ++c) dw[c] = fmaf(dz, h[c], dw[c]);
            if (j == 0) {
                dzs += dz;
                ls += pw * lab * softplus(-z) + (1.0f - lab) * softplus(z);
            }
        }
    }
    if (!labels) return;
#pragma unroll
    for (int c = 0; c < 4; ++c) sdw[slot][4 * j + c] = dw[c];
    if (j == 0) {
        sred[0][slot] = dzs;
        sred[1][slot] = ls;
    }
    __syncthreads();
    if (t < kCh) {
        float a = 0.0f;
        for (int q = 0; q < 16; ++q) a += sdw[q][t];
        atomicAdd(&grad[wh_off + t], a);
    } else if (t == kCh) {
        float a = 0.0f, b = 0.0f;
        for (int q = 0; q < 16; ++q) {
            a += sred[0][q];
            b += sred[1][q];
        }
        atomicAdd(&grad[wh_off + kCh], a);
        atomicAdd(loss_sum, b);
    }
}

// ------------------------------------------------------------------ Adam
__global__ void k_adam(float* __restrict__ theta, float* __restrict__ grad, float* __restrict__ m,
                       float* __restrict__ v, int64_t n, float lr, float b1, float b2, float eps, float c1, float c2,
                       NetLayout lay, uint16_t* __restrict__ w_bf, uint16_t* __restrict__ wt_bf, int update) {
    const int64_t p = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (p >= n) return;
    float th = theta[p];
    if (update) {
        const float g = grad[p];
        const float mm = b1 * m[p] + (1.0f - b1) * g;
        const float vv = b2 * v[p] + (1.0f - b2) * g * g;
        m[p] = mm;
        v[p] = vv;
        th -= lr * (mm * c1) / (sqrtf(vv * c2) + eps);
        theta[p] = th;
        grad[p] = 0.0f;
    }
    if (!w_bf) return;
    for (int l = 0; l < kLayers; ++l) {
        const int64_t q = p - lay.w_off[l];
        const int cin = lay.cin[l];
        if (q < 0 || q >= int64_t(kTaps) * cin * kCh) continue;
        const int64_t i = q / (int64_t(cin) * kCh), rem = q % (int64_t(cin) * kCh);
        const int64_t c = rem / kCh, o = rem % kCh;
        const uint16_t hb = to_bf16(th);
        w_bf[lay.bf_off[l] + q] = hb;
        wt_bf[lay.bf_off[l] + (i * kCh + o) * cin + c] = hb;
    }
}

__global__ void k_fill_f32(float* p, int64_t n) {
    const int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (i < n) p[i] = 0.0f;
}
__global__ void k_fill_u32(uint32_t* p, int64_t n) {
    const int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (i < n) p[i] = 0u;
}

// ------------------------------------------------------------------ proposals
__global__ void k_window(const float* __restrict__ y, int64_t F, float* __restrict__ c) {
    const int64_t f = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (f >= F) return;
    float acc = 0.0f;
    for (int i = -(kSpan / 2 - 1); i <= kSpan / 2; ++i) {
        const int64_t g = f + i;
        if (g >= 0 && g < F) acc += y[g];
    }
    c[f] = acc;
}

constexpr int kMaxSegList = 4096;

// One workgroup: every frame whose window score reaches kappa proposes the lags
// [128f + 256 - L, 128f] within [0, n-L]; the segments meeting a proposed range
// are listed in ascending order.  info = {proposed frames, segments}.
__global__ __launch_bounds__(1024) void k_propose(const float* __restrict__ c, int64_t F, float kappa, int64_t n,
                                                  int64_t L, int64_t V, int32_t max_segments,
                                                  int32_t* __restrict__ segs, int32_t* __restrict__ info) {
    __shared__ unsigned char mask[kMaxSegList];
    __shared__ int nprop;
    const int t = int(threadIdx.x);
    if (t == 0) nprop = 0;
    for (int j = t; j < kMaxSegList; j += 1024) mask[j] = 0;
    __syncthreads();
    const int64_t lags = n - L + 1;
    int mine = 0;
    for (int64_t f = t; f < F; f += 1024) {
        if (!(c[f] >= kappa)) continue;
        ++mine;
        const int64_t lo = int64_t(kHop) * f + kWin - L < 0 ? 0 : int64_t(kHop) * f + kWin - L;
        const int64_t hi = int64_t(kHop) * f < lags - 1 ? int64_t(kHop) * f : lags - 1;
        for (int64_t j = lo / V; lo <= hi && j <= hi / V && j < max_segments; ++j) mask[j] = 1;
    }
    if (mine) atomicAdd(&nprop, mine);
    __syncthreads();
    if (t == 0) {
        int ns = 0;
        const int64_t S = (lags + V - 1) / V;
        for (int64_t j = 0; j < S && j < max_segments; ++j)
            if (mask[j]) segs[ns++] = int32_t(j);
        info[0] = nprop;
        info[1] = ns;
    }
}

}  // namespace

// ------------------------------------------------------------------ launchers
static unsigned blocks_for(int64_t n, int per) { return unsigned((n + per - 1) / per); }

hipError_t launch_stft(const BlockSource& src, int nblocks, int64_t F, const float* hann, const float2* tw, float* P,
                       hipStream_t st) {
    const int64_t rows = int64_t(nblocks) * F;
    if (rows <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_stft, dim3(blocks_for(rows, 4)), dim3(256), 0, st, src, nblocks, F, hann, tw, P);
    return hipGetLastError();
}

hipError_t launch_median(const float* P, int nblocks, int64_t per_block, uint32_t* hist, MedianState* state,
                         float* med, hipStream_t st) {
    if (nblocks <= 0 || per_block <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_fill_u32, dim3(blocks_for(int64_t(nblocks) * 2048, 256)), dim3(256), 0, st, hist,
                       int64_t(nblocks) * 2048);
    hipLaunchKernelGGL(k_median_init, dim3(blocks_for(nblocks, 64)), dim3(64), 0, st, state, nblocks,
                       uint32_t((per_block - 1) / 2));
    // at most 64 workgroups per block: each adds its nonzero buckets to the
    // block's histogram with atomics, and the few buckets of the first pass
    // are the same for all of them
    const unsigned chunks = unsigned(per_block / (256 * 16) + 1 < 64 ? per_block / (256 * 16) + 1 : 64);
    for (int pass = 0; pass < 3; ++pass) {
        hipLaunchKernelGGL(k_hist, dim3(chunks, unsigned(nblocks)), dim3(256), 0, st, P, per_block, pass,
                           (const MedianState*)state, hist);
        hipLaunchKernelGGL(k_select, dim3(unsigned(nblocks)), dim3(256), 0, st, hist, pass, state, med);
    }
    return hipGetLastError();
}

hipError_t launch_map(const float* P, int nblocks, int64_t F, const float* med, void* map, bool bf16,
                      hipStream_t st) {
    const int64_t per = F * kWin, total = per * nblocks;
    if (total <= 0) return hipSuccess;
    if (bf16)
        hipLaunchKernelGGL(k_map<true>, dim3(blocks_for(total, 1024)), dim3(256), 0, st, P, per, total, med, map);
    else
        hipLaunchKernelGGL(k_map<false>, dim3(blocks_for(total, 1024)), dim3(256), 0, st, P, per, total, med, map);
    return hipGetLastError();
}

hipError_t launch_synth(const BlockSource& src, int64_t n, float2* out, hipStream_t st) {
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_synth, dim3(blocks_for(n, 256)), dim3(256), 0, st, src, n, out);
    return hipGetLastError();
}

hipError_t launch_labels(const SynthTx* tx, const int32_t* ntx, int nblocks, int64_t F, int L, float* labels,
                         hipStream_t st) {
    const int64_t rows = int64_t(nblocks) * F;
    if (rows <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_labels, dim3(blocks_for(rows, 256)), dim3(256), 0, st, tx, ntx, rows, F, L, labels);
    return hipGetLastError();
}

hipError_t launch_conv_forward(const void* in, int cin, const void* w, const float* bias, void* out, int64_t rows,
                               int64_t F, int d, bool bf16, hipStream_t st) {
    if (rows <= 0) return hipSuccess;
    if (bf16) {
        if (cin % 32 || d < 1) return hipErrorInvalidValue;
        const size_t lds = conv_tile_lds(cin, d);
        if (lds > kMaxConvLds) return hipErrorInvalidValue;
        hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void*>(&k_conv_tile<true>),
                                           hipFuncAttributeMaxDynamicSharedMemorySize, int(lds));
        if (e != hipSuccess) return e;
        hipLaunchKernelGGL(k_conv_tile<true>, dim3(blocks_for(rows, kTileRows)), dim3(256), lds, st, in,
                           (const uint16_t*)nullptr, cin, (const uint16_t*)w, bias, out, rows, F, d);
    } else {
        hipLaunchKernelGGL(k_conv_fwd_ref, dim3(blocks_for(rows * kCh, 256)), dim3(256), 0, st, (const float*)in,
                           cin, (const float*)w, bias, (float*)out, rows, F, d);
    }
    return hipGetLastError();
}

hipError_t launch_conv_dinput(const float* dH, const void* H, const void* w, float* dprev, int64_t rows, int64_t F,
                              int d, bool bf16, hipStream_t st) {
    if (rows <= 0) return hipSuccess;
    if (bf16) {
        if (d < 1) return hipErrorInvalidValue;
        const size_t lds = conv_tile_lds(kCh, d);
        if (lds > kMaxConvLds) return hipErrorInvalidValue;
        hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void*>(&k_conv_tile<false>),
                                           hipFuncAttributeMaxDynamicSharedMemorySize, int(lds));
        if (e != hipSuccess) return e;
        hipLaunchKernelGGL(k_conv_tile<false>, dim3(blocks_for(rows, kTileRows)), dim3(256), lds, st, (const void*)dH,
                           (const uint16_t*)H, kCh, (const uint16_t*)w, (const float*)nullptr, (void*)dprev, rows,
                           F, d);
    } else
        hipLaunchKernelGGL(k_conv_dinput_ref, dim3(blocks_for(rows * kCh, 256)), dim3(256), 0, st, dH,
                           (const float*)H, (const float*)w, dprev, rows, F, d);
    return hipGetLastError();
}

// chunks x groups <= (pieces / k + 1) * groups <= kDwWgs + groups for k = ceil(pieces * groups / kDwWgs)
int64_t dweight_part_elems(int cin) {
    const int64_t ngroups = std::max(cin / 64, 1);
    return (kDwWgs + ngroups) * (kDwBlock + kCh);
}

hipError_t launch_conv_dweight(const void* in, int cin, const float* dH, const void* H, float* dW, float* db,
                               float* part, int64_t part_elems, int64_t rows, int64_t F, int d, bool bf16,
                               hipStream_t st) {
    if (rows <= 0) return hipSuccess;
    if (bf16) {
        if (cin % 64 || cin <= 0 || rows >= (int64_t(1) << 31) || !part) return hipErrorInvalidValue;
        const int64_t ngroups = cin / 64, pieces = (rows + kDwRows - 1) / kDwRows;
        const int64_t chunk = kDwRows * std::max<int64_t>(1, (pieces * ngroups + kDwWgs - 1) / kDwWgs);
        const int nchunks = int((rows + chunk - 1) / chunk);
        if ((nchunks * ngroups) * (kDwBlock + kCh) > part_elems) return hipErrorInvalidValue;
        float* pdb = db ? part + nchunks * ngroups * kDwBlock : nullptr;
        const unsigned grid = unsigned((nchunks + kDwXcds - 1) / kDwXcds * kDwXcds * ngroups);
        auto go = [&](auto kern) {
            hipLaunchKernelGGL(kern, dim3(grid), dim3(256), 0, st, (const uint16_t*)in, cin, dH,
                               (const uint16_t*)H, part, pdb, rows, F, int(chunk), nchunks);
        };
        switch (d) {
        case 1: go(k_conv_dw_taps<1>); break;
        case 2: go(k_conv_dw_taps<2>); break;
        case 4: go(k_conv_dw_taps<4>); break;
        case 8: go(k_conv_dw_taps<8>); break;
        default: return hipErrorInvalidValue;    // the network's dilations only
        }
        hipLaunchKernelGGL(k_dw_reduce, dim3(unsigned(kTaps * cin + (db ? 1 : 0))), dim3(256), 0, st,
                           (const float*)part, (const float*)pdb, dW, db, cin, nchunks);
    } else {
        hipLaunchKernelGGL(k_conv_dw_ref, dim3(blocks_for(int64_t(kTaps) * cin * kCh, 256)), dim3(256), 0, st,
                           (const float*)in, cin, dH, (const float*)H, dW, db, rows, F, d);
    }
    return hipGetLastError();
}

hipError_t launch_head(const void* h4, const float* theta, int64_t wh_off, float* y, const float* labels,
                       float pos_weight, float inv_rows, float* dH4, float* grad, float* loss_sum, int64_t rows,
                       bool bf16, hipStream_t st) {
    if (rows <= 0) return hipSuccess;
    if (bf16)
        hipLaunchKernelGGL(k_head<true>, dim3(blocks_for(rows, kHeadRows)), dim3(256), 0, st, h4, theta, wh_off, y,
                           labels, pos_weight, inv_rows, dH4, grad, loss_sum, rows);
    else
        hipLaunchKernelGGL(k_head<false>, dim3(blocks_for(rows, kHeadRows)), dim3(256), 0, st, h4, theta, wh_off, y,
                           labels, pos_weight, inv_rows, dH4, grad, loss_sum, rows);
    return hipGetLastError();
}

hipError_t launch_adam(float* theta, float* grad, float* m, float* v, int64_t n, float lr, float b1, float b2,
                       float eps, int t, const NetLayout& lay, uint16_t* w_bf, uint16_t* wt_bf, hipStream_t st) {
    // t = 0: refresh the bf16 copies only
    const double c1 = t > 0 ? 1.0 / (1.0 - pow(double(b1), t)) : 1.0;
    const double c2 = t > 0 ? 1.0 / (1.0 - pow(double(b2), t)) : 1.0;
    hipLaunchKernelGGL(k_adam, dim3(blocks_for(n, 256)), dim3(256), 0, st, theta, grad, m, v, n, lr, b1, b2, eps,
                       float(c1), float(c2), lay, w_bf, wt_bf, t > 0 ? 1 : 0);
    return hipGetLastError();
}

hipError_t launch_fill_f32(float* p, int64_t n, hipStream_t st) {
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_fill_f32, dim3(blocks_for(n, 256)), dim3(256), 0, st, p, n);
    return hipGetLastError();
}

hipError_t launch_fill_u32(uint32_t* p, int64_t n, hipStream_t st) {
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_fill_u32, dim3(blocks_for(n, 256)), dim3(256), 0, st, p, n);
    return hipGetLastError();
}

hipError_t launch_window(const float* y, int64_t F, float* c, hipStream_t st) {
    if (F <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_window, dim3(blocks_for(F, 256)), dim3(256), 0, st, y, F, c);
    return hipGetLastError();
}

hipError_t launch_propose(const float* c, int64_t F, float kappa, int64_t n, int64_t L, int64_t V,
                          int32_t max_segments, int32_t* segs, int32_t* out_info, hipStream_t st) {
    if (max_segments > kMaxSegList) return hipErrorInvalidValue;
    hipLaunchKernelGGL(k_propose, dim3(1), dim3(1024), 0, st, c, F, kappa, n, L, V, max_segments, segs, out_info);
    return hipGetLastError();
}

}  // namespace learned
}  // namespace acq
