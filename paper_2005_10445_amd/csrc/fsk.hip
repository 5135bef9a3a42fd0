// FSK searching pipeline of Section 3 (steps 1-8) on gfx950, with the FFT
// methods of Section 4.1.
//
//   k_fsk_front     : one workgroup per overlap-save segment of the composed
//                     filters: int16 -> complex and local-oscillator mix (or,
//                     at plan time, the noise-free continuous-phase replica of
//                     a tag's bits), forward 4096-point transform, products
//                     with the spectra of h_BP * h_1 and h_BP * h_0, two inverse
//                     transforms, demodulation d = (|f1|-|f0|)/(|f1|+|f0|),
//                     u = |f1|-|f0|.  Output d and u (block) or d (replica).
//   k_fsk_pack      : overlap-save segments 2s and 2s+1 of the call (numbered
//                     over its blocks) as the real and imaginary parts of one
//                     complex M-point input (slot s)
//   (forward spectra of the slots and of the templates: launch_forward, the
//    decimation-in-time transform of the acquisition path)
//   k_fsk_correlate : the real cross-correlation of d with each template by
//                     overlap-save.  The template d^(c) is real, so the inverse
//                     transform of Z_g conj(D^(c)) / M holds the correlation of
//                     segment 2g in its real part and of segment 2g+1 in its
//                     imaginary part: one complex transform per two segments.
//                     Two tracking segments with different templates share
//                     a slot too: with Z the slot's spectrum, X_A = (Z[i] +
//                     conj Z[-i]) / 2 and j X_B = (Z[i] - conj Z[-i]) / 2,
//                     so the product is (Z[i] (B_a + B_b) + conj Z[-i]
//                     (B_a - B_b)) / 2 for the conjugate spectra B of the two
//                     templates.  The peak search uses |c|.  An M-point inverse
//                     transform (M up to 2^18) runs as P = M / Msub phases of
//                     an Msub-point transform: for output lag tau = P u + rho,
//                       G_rho[i'] = exp(+j 2 pi i' rho / M)
//                                   sum_a Y[i' + Msub a] exp(+j 2 pi a rho / P),
//                     Y the spectrum product, then an Msub-point inverse
//                     transform of G_rho.  Keys: bits(|Re c|) << 32 | ~tau.
//   k_fsk_refine_*  : FP64 sums over +/-3 lags of the peak from the stored d,
//                     u and template (in parts, added in order), re-maximisation,
//                     parabola, w_c, q, p_c, z.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <new>
#include <string>
#include <vector>

#include "acq.h"
#include "device_common.h"
#include "host_logic.h"
#include "kernels.h"

namespace acq {

using namespace kdev;

namespace {

constexpr int kFrontLog = 12;                 // composed filters applied on 4096-point segments
constexpr int kFrontN = 1 << kFrontLog;
constexpr int kFskMaxGrid = 256;              // workgroups (and scratch slots) of the correlation: one per CU
constexpr int kFskSplitMaxGrid = 2048;        // workgroups of the one-phase-per-workgroup form (no scratch)

// One block of an FSK call: the searching window (tag -1: every template) or
// one tracking task (its tag only).  Front-end segments and correlation
// segments are numbered globally over the call's blocks; slot s holds
// correlation segments 2s and 2s+1, which may belong to different blocks.
struct FskTask {
    const int16_t* iq;          // device [n][2]
    int64_t n;                  // samples
    int64_t lags;               // n - n_t + 1 (<= 0: nothing to search)
    int64_t zoff;               // offset of the block's d and u in the plan's arrays
    int32_t tag;                // -1 searching; else the tracked template
    int32_t fseg0, nfseg;       // front-end segments
    int32_t unit0;              // first correlation segment (global number)
    int32_t nseg;               // overlap-save segments of the correlation
};

struct FskTasks {
    const FskTask* t;           // device [count]
    int32_t count;
    int32_t track;              // 1: tracking tasks (one template each)
};

// block holding global index g of the field (fseg0 or unit0), by binary search
template <int32_t FskTask::*FIRST>
__device__ __forceinline__ int fsk_task_of(const FskTasks& tt, int g) {
    int lo = 0, hi = tt.count - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (tt.t[mid].*FIRST <= g) lo = mid; else hi = mid - 1;
    }
    return lo;
}

struct FrontArgs {
    FskTasks tasks;             // blocks (block mode)
    const uint8_t* bits;        // replica: [T][nbits]
    const double* bit_cyc;      // replica: [T][nbits] carrier phase (cycles, in [0,1)) at each bit start
    const float2* G1;           // [kFrontN] DFT(h_BP * h_1) / kFrontN
    const float2* G0;
    const float2* roots;        // [kFrontN] exp(+j 2 pi m / kFrontN)
    float2* out;                // replica: [T][out_stride] (d, 0)
    float* out_d;               // block: d at the block's zoff
    float* out_u;               // block: u at the block's zoff
    int64_t n_in, n_out, out_stride;     // replica mode
    double lo_cyc;              // f_LO / Fs
    float2 lo_step[16];         // exp(-j 2 pi (f_LO / Fs) (NT m)), m < 16 (FP64, rounded once)
    double f1_cyc, f0_cyc;      // tones, cycles per sample
    int32_t nbits, sps, lg, vf, nseg, replica;   // nseg: segments per replica
};

// One workgroup per (template, segment) of the replicas or per global segment
// of the blocks: outputs s*vf .. s*vf + vf - 1 of the causal convolution with
// the composed filters, from inputs s*vf - (lg-1) ..  Three workgroups per CU
// (at most 168 VGPRs: the forward spectrum stays in registers through the
// first inverse transform; at 128 it spills and runs slower).
__global__ __launch_bounds__(256, 3) void k_fsk_front(FrontArgs a) {
    using E = StockhamEngine<kFrontLog>;
    __shared__ float2 lds[E::LDS];
    E eng;
    eng.init(a.roots, nullptr);
    int s, tag = 0;
    const int16_t* iq = nullptr;
    int64_t n_in = a.n_in, n_out = a.n_out, zoff = 0;
    if (a.replica) {
        s = int(blockIdx.x) % a.nseg;
        tag = int(blockIdx.x) / a.nseg;
    } else {
        const int b = fsk_task_of<&FskTask::fseg0>(a.tasks, int(blockIdx.x));
        const FskTask tk = a.tasks.t[b];
        s = int(blockIdx.x) - tk.fseg0;
        iq = tk.iq;
        n_in = n_out = tk.n;
        zoff = tk.zoff;
    }
    const int64_t base = int64_t(s) * a.vf - (a.lg - 1);
    float2 x[16];
    if (a.replica) {
#pragma unroll
        for (int m = 0; m < 16; ++m) {
            const int64_t p = base + eng.in_index(m);
            float2 v = make_float2(0.f, 0.f);
            if (p >= 0 && p < n_in) {
                const int64_t b = p / a.sps;
                const size_t bi = size_t(tag) * size_t(a.nbits) + size_t(b);
                double cyc = a.bit_cyc[bi] + (a.bits[bi] ? a.f1_cyc : a.f0_cyc) * double(p - b * a.sps);
                cyc -= floor(cyc);                          // exact phase reduction in FP64
                float sn, cs;
                sincospif(2.0f * float(cyc), &sn, &cs);
                v = make_float2(cs, sn);
            }
            x[m] = v;
        }
    } else {
        // LO mix exp(-j 2 pi f_LO p / Fs) at p = p0 + NT m: the phase of p0 is
        // reduced exactly in FP64 once per thread, and register m rotates it
        // by the constant lo_step[m]
        const int64_t p0 = base + eng.in_index(0);
        double cyc = -a.lo_cyc * double(p0);
        cyc -= floor(cyc);
        float sn0, cs0;
        sincospif(2.0f * float(cyc), &sn0, &cs0);
        const float2 e0 = make_float2(cs0, sn0);
#pragma unroll
        for (int m = 0; m < 16; ++m) {
            const int64_t p = base + eng.in_index(m);
            float2 v = make_float2(0.f, 0.f);
            if (p >= 0 && p < n_in) {
                const float2 e = m ? cmul(e0, a.lo_step[m]) : e0;
                v = cmul(make_float2(float(iq[2 * p]), float(iq[2 * p + 1])), e);
            }
            x[m] = v;
        }
    }
    const __amdgpu_buffer_rsrc_t dummy = make_rsrc(a.roots, 8);   // unused by the Stockham engine
    eng.template transform<-1>(x, lds, dummy, nullptr);
    float a1[16];
    float2 w[16];
#pragma unroll
    for (int m = 0; m < 16; ++m) w[m] = cmul(x[m], a.G1[eng.in_index(m)]);
    eng.template transform<+1>(w, lds, dummy, nullptr);
#pragma unroll
    for (int m = 0; m < 16; ++m) a1[m] = sqrtf(fmaf(w[m].x, w[m].x, w[m].y * w[m].y));
#pragma unroll
    for (int m = 0; m < 16; ++m) w[m] = cmul(x[m], a.G0[eng.in_index(m)]);
    eng.template transform<+1>(w, lds, dummy, nullptr);
#pragma unroll
    for (int m = 0; m < 16; ++m) {
        const int idx = eng.in_index(m);                     // natural order in and out
        const int64_t o = int64_t(s) * a.vf + idx - (a.lg - 1);
        if (idx >= a.lg - 1 && o < n_out) {
            const float a0 = sqrtf(fmaf(w[m].x, w[m].x, w[m].y * w[m].y));
            const float sum = a1[m] + a0, dif = a1[m] - a0;
            const float d = sum > 0.f ? dif / sum : 0.f;
            if (a.replica) {
                a.out[size_t(tag) * size_t(a.out_stride) + size_t(o)] = make_float2(d, 0.f);
            } else {
                a.out_d[zoff + o] = d;
                a.out_u[zoff + o] = dif;
            }
        }
    }
}

// zp[s][i] = (d_A[jA V + i], d_B[jB V + i]) for the correlation segments 2s
// (segment jA of block A) and 2s+1 (segment jB of block B; zero if the call
// has no such segment), zero past the end of a block.  256 threads per
// workgroup, each workgroup CHUNK (or M) consecutive i of one slot: the slot,
// and so the block lookups, are uniform over the workgroup and done once.
// Chunks of 4096 when that still gives 512 workgroups, else 1024 (a
// searching window's two slots in 512 workgroups: 7.9 -> 5.6 us; the 32
// slots of 64 tracking tasks keep 4096: with 1024, 23 us against 16).
template <int CHUNK>
__global__ __launch_bounds__(256) void k_fsk_pack(FskTasks tt, const float* __restrict__ d, int64_t V, int64_t M,
                                                  int units, float2* __restrict__ zp) {
    const int64_t chunk = M < CHUNK ? M : CHUNK;
    const int64_t per_slot = M / chunk;
    const int64_t s = int64_t(blockIdx.x) / per_slot;
    const int ua = int(2 * s), ub = int(2 * s + 1);
    const FskTask ta = tt.t[fsk_task_of<&FskTask::unit0>(tt, ua)];
    const bool second = ub < units;
    const FskTask tb = second ? tt.t[fsk_task_of<&FskTask::unit0>(tt, ub)] : ta;
    const float* da = d + ta.zoff;
    const float* dbb = d + tb.zoff;
    const int64_t sa = int64_t(ua - ta.unit0) * V, sb = int64_t(ub - tb.unit0) * V;
    const int64_t i0 = (int64_t(blockIdx.x) - s * per_slot) * chunk;
    for (int64_t i = i0 + threadIdx.x; i < i0 + chunk; i += 256) {
        const float re = sa + i < ta.n ? da[sa + i] : 0.f;
        const float im = (second && sb + i < tb.n) ? dbb[sb + i] : 0.f;
        zp[s * M + i] = make_float2(re, im);
    }
}

// bank[t][i] = conj(X_t[i]) / M in place
__global__ void k_fsk_conj_scale(float2* bank, int64_t count, float scale) {
    const int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (i < count) {
        const float2 v = bank[i];
        bank[i] = make_float2(v.x * scale, -v.y * scale);
    }
}

__global__ void k_fsk_fill(float2* p, int64_t count) {
    const int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (i < count) p[i] = make_float2(0.f, 0.f);
}

struct FskCorrArgs {
    const float2* X;            // [slots][M] spectra of the packed segment pairs
    const float2* bank;         // [T][M] conj(DFT_M(d^(c))) / M
    const float2* rootsM;       // [M]
    const float2* rootsSub;     // [Msub]
    const float2* b1tab;
    float2* scratch;            // [gridDim.x][M]: the P first-step outputs of the workgroup's item
    unsigned long long* keys;   // [T] (searching) or [tasks] (tracking)
    float* dump;                // optional [T][lags]: c at every lag (test hook, searching)
    FskTasks tasks;
    int64_t V;
    int32_t M, Msub, P, T, nslots;      // nslots: slots of the call
    int32_t units;                      // correlation segments of the call
    int32_t split;                      // 1: one phase per work item (set by the launcher)
};

// Work item (template t, slot s), taken with a stride of the grid: searching,
// items t * nslots + s for every template; tracking, item s with the
// templates of its segments' tasks.  Slot s holds correlation segments 2s
// (real part) and 2s+1 (imaginary part).
//   first step, once per item: for each i' < Msub, the spectrum products
//     Y_a = Z_s[i' + Msub a] B_t[i' + Msub a], a < P, B_t = conj(D_t) / M (or
//     the two-template product when the segments' templates differ), and
//     G_rho[i'] = exp(+j 2 pi i' rho / M) sum_a Y_a exp(+j 2 pi a rho / P),
//     written to the workgroup's scratch (each input read once);
//   then, per phase rho, the Msub-point inverse transform of G_rho (lag
//   P u + rho) and each segment's lane maximum of |c| over all phases.
// SPLIT (calls with fewer items than CUs, e.g. a few tracking tasks): work
// item (item, rho) forms its G_rho in registers from the P products, reading
// the spectra once per phase instead of going through the scratch.
// exp(+j 2 pi k / 8), k < 8 (the values FP64 rounds to in FP32)
__device__ __forceinline__ float2 root8(int k) {
    constexpr float h = 0.70710678118654752f;
    switch (k) {
        case 0: return make_float2(1.f, 0.f);
        case 1: return make_float2(h, h);
        case 2: return make_float2(0.f, 1.f);
        case 3: return make_float2(-h, h);
        case 4: return make_float2(-1.f, 0.f);
        case 5: return make_float2(-h, -h);
        case 6: return make_float2(0.f, -1.f);
        default: return make_float2(h, -h);
    }
}

// exp(+j 2 pi k / 8) for a run-time k (selects, no table)
__device__ __forceinline__ float2 root8_rt(int k) {
    constexpr float h = 0.70710678118654752f;
    auto c = [](int kk) {                    // cos(pi kk / 4), kk < 8
        const float mag = (kk & 1) ? h : ((kk & 2) ? 0.0f : 1.0f);
        return (kk >= 3 && kk <= 5) ? -mag : mag;
    };
    return make_float2(c(k & 7), c((k + 6) & 7));
}

// TRACK: tracking calls, whose slots may hold segments of two templates.
template <class E, int PP, bool DUMP, bool SPLIT, bool TRACK>
__global__ __launch_bounds__(E::NT) void k_fsk_correlate(FskCorrArgs a) {
    constexpr int NW = E::NT / 64;
    __shared__ float2 lds[E::LDS];
    __shared__ float2 extra[E::EXTRA];
    __shared__ unsigned long long red[2 * NW];
    E eng;
    eng.init(a.rootsSub, extra);
    const int lane = int(threadIdx.x) & 63, wave = int(threadIdx.x) >> 6;
    const __amdgpu_buffer_rsrc_t b1 = make_rsrc(a.b1tab, E::B1_TABLE * 8);
    const int mmask = a.M - 1;
    float2* G = a.scratch + size_t(blockIdx.x) * size_t(a.M);
    const int items = (a.tasks.track ? a.nslots : a.T * a.nslots) * (SPLIT ? PP : 1);
    // SPLIT with one work item per workgroup: the PP phases of an item read
    // the same spectra, so they run on one XCD (workgroups go to the XCDs in
    // turn) and share its L2.  Within each group of kXcds * PP workgroups,
    // workgroup j takes phase j / kXcds of item j % kXcds of the group.
    constexpr int grp = kXcds * PP;
    const bool xcd_map = SPLIT && int(gridDim.x) >= items;
    // Searching without SPLIT (a grid of whole-XCD multiples): XCD x takes the
    // templates x, x + kXcds, ..., and its workgroups take the slots of one
    // template side by side, so that template's spectrum is read once into
    // the XCD's L2 instead of once per slot on different XCDs.
    const bool tmap = !SPLIT && !TRACK && int(gridDim.x) % kXcds == 0;
    const int xg = int(blockIdx.x) % kXcds, nw = int(gridDim.x) / kXcds;
    const int nloop = tmap ? ((a.T - xg + kXcds - 1) / kXcds) * a.nslots : items;
    for (int ci = tmap ? int(blockIdx.x) / kXcds : int(blockIdx.x); ci < nloop;
         ci += tmap ? nw : int(gridDim.x)) {
        const int wi = tmap ? (xg + kXcds * (ci / a.nslots)) * a.nslots + ci % a.nslots : ci;
        int it = SPLIT ? wi / PP : wi;
        int rho0 = SPLIT ? wi % PP : 0;
        if (xcd_map && wi < items / grp * grp) {
            const int q = wi / grp, j = wi - q * grp;
            it = q * kXcds + j % kXcds;
            rho0 = j / kXcds;
        }
        const int rho1 = SPLIT ? rho0 + 1 : PP;
        const int slot = a.tasks.track ? it : it % a.nslots;
        // the slot's two correlation segments: block, segment within it, template, key
        int bk[2], jseg[2], tg[2], kidx[2];
#pragma unroll
        for (int h = 0; h < 2; ++h) {
            const int u = 2 * slot + h < a.units ? 2 * slot + h : 2 * slot;     // absent: as the first
            bk[h] = fsk_task_of<&FskTask::unit0>(a.tasks, u);
            jseg[h] = 2 * slot + h < a.units ? u - a.tasks.t[bk[h]].unit0 : -1;
            tg[h] = a.tasks.track ? a.tasks.t[bk[h]].tag : it / a.nslots;
            kidx[h] = a.tasks.track ? bk[h] : tg[h];
        }
        const float2* Xj = a.X + size_t(slot) * size_t(a.M);
        const float2* B = a.bank + size_t(tg[0]) * size_t(a.M);
        const float2* Bb = a.bank + size_t(tg[1]) * size_t(a.M);
        const bool two = TRACK && tg[1] != tg[0];              // uniform: tracking segments of two templates
        // first step: P outputs per i' from P products; the P-point DFT uses
        // constant eighth roots of unity, so each i' issues its 2P product
        // loads and P-1 twiddle loads together (one i' at a time keeps them in
        // registers without holding all 16)
        // the P spectrum products of input index ip
        auto products = [&](int ip, float2 (&y)[PP]) {
            if (!two) {
#pragma unroll
                for (int q = 0; q < PP; ++q) y[q] = cmul(Xj[ip + q * a.Msub], B[ip + q * a.Msub]);
            } else {
#pragma unroll
                for (int q = 0; q < PP; ++q) {
                    const int i = ip + q * a.Msub;
                    const float2 z = Xj[i], zm = Xj[(a.M - i) & mmask];
                    const float2 ba = B[i], bb = Bb[i];
                    const float2 s = cadd(ba, bb), d = make_float2(ba.x - bb.x, ba.y - bb.y);
                    const float2 r = cadd(cmul(z, s), cmul(make_float2(zm.x, -zm.y), d));
                    y[q] = make_float2(0.5f * r.x, 0.5f * r.y);
                }
            }
        };
        float2 gs[16];                            // SPLIT: G_rho0 of this thread's inputs
        if constexpr (SPLIT) {
            float2 w[PP];                         // exp(+j 2 pi q rho0 / P)
#pragma unroll
            for (int q = 0; q < PP; ++q) w[q] = root8_rt(q * rho0 * (8 / PP));
#pragma unroll
            for (int m = 0; m < 16; ++m) {
                // opaque index: its address arithmetic is not hoisted out of
                // the item loop for all 16 registers at once
                int ip = eng.in_index(m);
                asm volatile("" : "+v"(ip));
                float2 y[PP];
                products(ip, y);
                float2 acc = y[0];
#pragma unroll
                for (int q = 1; q < PP; ++q) acc = cadd(acc, cmul(y[q], w[q]));
                gs[m] = rho0 ? cmul(acc, a.rootsM[(ip * rho0) & mmask]) : acc;
                asm volatile("" ::: "memory");    // one input index at a time: no hoisting of later loads
            }
        } else {
            // two input indices per pass (one for P = 16), so that their 4P
            // loads are in flight together; the P-point DFT over q is a
            // radix-P butterfly, and the twiddle of phase rho is the rho-th
            // power of exp(+j 2 pi i' / M)
            constexpr int IPP = PP > 8 ? 1 : 2;
#pragma unroll 1
            for (int m = 0; m < 16; m += IPP) {
                float2 y[IPP][PP];
                int ipv[IPP];
#pragma unroll
                for (int h = 0; h < IPP; ++h) {
                    ipv[h] = eng.in_index(m + h);
                    products(ipv[h], y[h]);
                }
#pragma unroll
                for (int h = 0; h < IPP; ++h) {
                    const int ip = ipv[h];
                    if constexpr (PP > 1) dev::dft_r<PP, +1>(y[h]);
                    G[ip] = y[h][0];
                    if constexpr (PP > 1) {
                        const float2 w1 = a.rootsM[ip];
                        float2 tw = w1;
#pragma unroll
                        for (int rho = 1; rho < PP; ++rho) {
                            G[rho * a.Msub + ip] = cmul(y[h][rho], tw);
                            if (rho + 1 < PP) tw = cmul(tw, w1);
                        }
                    }
                }
            }
        }
        if constexpr (!SPLIT) {
            __threadfence_block();
            __syncthreads();
        }
        int ulim[2];
        int64_t sbeg[2];
        unsigned long long best[2] = {0ull, 0ull};
        int vlim[2];                                  // valid lags of each segment
#pragma unroll
        for (int h = 0; h < 2; ++h) {
            const int64_t lags = a.tasks.t[bk[h]].lags;
            sbeg[h] = int64_t(jseg[h]) * a.V;
            vlim[h] = jseg[h] >= 0 ? int(lags - sbeg[h] < a.V ? lags - sbeg[h] : a.V) : 0;
        }
        for (int rho = rho0; rho < rho1; ++rho) {
#pragma unroll
            for (int h = 0; h < 2; ++h) ulim[h] = vlim[h] > rho ? (vlim[h] - rho + PP - 1) / PP : 0;
            const int ob0 = eng.out_base();
            const int omin = eng.out_min();
            const bool hi = omin + E::HI_OFF < max(ulim[0], ulim[1]);
            float2 v[16];
#pragma unroll
            for (int m = 0; m < 16; ++m) {
                if constexpr (SPLIT) v[m] = gs[m];
                else v[m] = G[rho * a.Msub + eng.in_index(m)];
            }
            eng.template transform<+1>(v, lds, b1, extra, hi);
            // output off of this lane is a valid lag of segment h when off < lim[h]
            int lim[2] = {ulim[0] - ob0, ulim[1] - ob0};
            asm volatile("" : "+v"(lim[0]), "+v"(lim[1]));
            // this lane's largest |c| of the phase, in increasing lag (strict
            // comparison: the smallest lag of a tie within the phase); one
            // maximum per segment when tracking, else one over both segments
            // (the first segment's lags come first)
            constexpr int NR = TRACK ? 2 : 1;
            float bp[NR];
            int boff[NR], bh[NR];
#pragma unroll
            for (int k = 0; k < NR; ++k) {
                bp[k] = -1.0f;
                boff[k] = bh[k] = 0;
            }
#pragma unroll
            for (int h = 0; h < 2; ++h) {
                const int k = TRACK ? h : 0;
#pragma unroll
                for (int rr = 0; rr < 16; ++rr) {
                    const int r = E::visit(rr);
                    const int off = E::out_off(r);
                    if (omin + off < ulim[h]) {
                        const float cv = h ? v[r].y : v[r].x;
                        const float pv = fabsf(cv);
                        if constexpr (DUMP) {
                            if (off < lim[h]) {
                                const int64_t tau = sbeg[h] + int64_t(PP) * (ob0 + off) + rho;
                                a.dump[size_t(tg[h]) * size_t(a.tasks.t[bk[h]].lags) + size_t(tau)] = cv;
                            }
                        }
                        const bool take = pv > bp[k] && off < lim[h];
                        boff[k] = take ? off : boff[k];
                        bh[k] = take ? h : bh[k];
                        bp[k] = take ? pv : bp[k];
                    }
                }
            }
#pragma unroll
            for (int k = 0; k < NR; ++k) {
                const unsigned lag = unsigned(sbeg[bh[k]] + rho) + unsigned(ob0 + boff[k]) * unsigned(PP);
                const unsigned long long key = bp[k] >= 0.0f
                    ? (static_cast<unsigned long long>(__float_as_uint(bp[k])) << 32) | static_cast<unsigned long long>(~lag)
                    : 0ull;
                best[k] = key > best[k] ? key : best[k];    // across phases the key order decides ties
            }
        }
        // one key per result: the two segments' maxima combine when they
        // belong to the same result (searching, or one tracking task)
        const bool same = kidx[1] == kidx[0];
        if (same) best[0] = best[1] > best[0] ? best[1] : best[0];
        best[0] = wave_max(best[0]);
        if (!same) best[1] = wave_max(best[1]);
        if (lane == 0) {
            red[wave] = best[0];
            red[NW + wave] = best[1];
        }
        __syncthreads();
        if (threadIdx.x < (same ? 1 : 2)) {
            const int h = int(threadIdx.x);
            unsigned long long m = 0ull;
            for (int q = 0; q < NW; ++q) m = red[h * NW + q] > m ? red[h * NW + q] : m;
            if (m) atomicMax(&a.keys[kidx[h]], m);
        }
        __syncthreads();                     // red[], scratch and LDS are reused by the next item
    }
}

// Results: searching, one item per template of the window; tracking, one item
// per task (its template).
struct FskRefineArgs {
    const float* d;             // the blocks' d (each at its zoff)
    const float* u;
    const float2* tmpl;         // [T][tstride] (d^(c), 0)
    const unsigned long long* keys;     // [items]
    double* partial;            // [items][kFskParts][kFskSums]
    acq_fsk_detection* dets;    // [items]
    int32_t* found;             // [items]
    FskTasks tasks;
    int64_t nt, tstride;
    double theta;
};

struct FskItem {
    int tag, block;
    FskTask tk;
};

__device__ __forceinline__ FskItem fsk_item(const FskRefineArgs& a, int item) {
    FskItem r;
    r.block = a.tasks.track ? item : 0;
    r.tk = a.tasks.t[r.block];
    r.tag = a.tasks.track ? r.tk.tag : item;
    return r;
}

// FP64 sums over lags tau*-3 .. tau*+3 around the peak key: w_c, p_c and q at
// each lag and E_c, enough for the re-maximisation over +/-1 and one
// re-centring.  Each (tag, part) workgroup sums a fixed chunk of the template
// in a fixed order and the parts are added in order: deterministic.
constexpr int kFskWin = 7;
constexpr int kFskParts = 16;
constexpr int kFskSums = 3 * kFskWin + 1;
constexpr int kFskStage = 4608;     // d and u samples of one part staged in LDS (longer parts read global)

__global__ __launch_bounds__(256) void k_fsk_refine_sums(FskRefineArgs a) {
    constexpr int NT = 256, NW = NT / 64;
    const int item = int(blockIdx.x) / kFskParts, part = int(blockIdx.x) % kFskParts;
    const FskItem fi = fsk_item(a, item);
    const int t = int(threadIdx.x), lane = t & 63, wave = t >> 6;
    __shared__ double red[NW][kFskSums];
    double* out = a.partial + (size_t(item) * kFskParts + part) * kFskSums;
    const unsigned long long key = fi.tk.lags > 0 ? a.keys[item] : 0ull;
    if (key == 0ull) {
        if (t < kFskSums) out[t] = 0.0;
        return;
    }
    const int64_t lam0 = int64_t(~unsigned(key & 0xffffffffull)) - kFskWin / 2;
    const float2* dc = a.tmpl + size_t(fi.tag) * size_t(a.tstride);
    const float* db = a.d + fi.tk.zoff;
    const float* ub = a.u + fi.tk.zoff;
    const int64_t ch = (a.nt + kFskParts - 1) / kFskParts;
    const int64_t i0 = int64_t(part) * ch, i1 = min(a.nt, i0 + ch);
    // the part reads block samples k0 .. k0 + span - 1 (zero outside the block),
    // each kFskWin times: stage them in LDS when they fit
    __shared__ float s_d[kFskStage], s_u[kFskStage];
    const int64_t k0 = lam0 + i0;
    const int64_t span = i1 > i0 ? i1 - i0 + kFskWin - 1 : 0;
    const bool staged = span <= kFskStage;
    if (staged) {
        for (int64_t q = t; q < span; q += NT) {
            const int64_t k = k0 + q;
            const bool in = k >= 0 && k < fi.tk.n;
            s_d[q] = in ? db[k] : 0.f;
            s_u[q] = in ? ub[k] : 0.f;
        }
    }
    __syncthreads();
    double wv[kFskWin], pv[kFskWin], qv[kFskWin], ec = 0.0;
#pragma unroll
    for (int w = 0; w < kFskWin; ++w) wv[w] = pv[w] = qv[w] = 0.0;
    for (int64_t i = i0 + t; i < i1; i += NT) {
        const double c = dc[i].x;
        ec += c * c;
#pragma unroll
        for (int w = 0; w < kFskWin; ++w) {
            double zd = 0.0, zu = 0.0;
            if (staged) {                           // zero outside the block, as staged
                zd = s_d[i - i0 + w];
                zu = s_u[i - i0 + w];
            } else {
                const int64_t k = lam0 + w + i;
                if (k >= 0 && k < fi.tk.n) {
                    zd = db[k];
                    zu = ub[k];
                }
            }
            wv[w] += c * zd;
            pv[w] += c * zu;
            qv[w] += zd * zd;
        }
    }
#pragma unroll
    for (int w = 0; w < kFskWin; ++w) {
        const double r0 = wave_sum(wv[w]), r1 = wave_sum(pv[w]), r2 = wave_sum(qv[w]);
        if (lane == 0) {
            red[wave][3 * w] = r0;
            red[wave][3 * w + 1] = r1;
            red[wave][3 * w + 2] = r2;
        }
    }
    const double es = wave_sum(ec);
    if (lane == 0) red[wave][3 * kFskWin] = es;
    __syncthreads();
    if (t < kFskSums) {
        double v = 0.0;
        for (int q = 0; q < NW; ++q) v += red[q][t];
        out[t] = v;
    }
}

// One wave per item: lane k < kFskSums adds sum k over the parts in order;
// lane 0 re-maximises |w_c| over +/-1 lag (one re-centring when it lands on
// the edge), fits the parabola and writes the result.
__global__ __launch_bounds__(64) void k_fsk_refine_final(FskRefineArgs a) {
    const int item = int(blockIdx.x);
    const FskItem fi = fsk_item(a, item);
    const int64_t lags = fi.tk.lags;
    const unsigned long long key = lags > 0 ? a.keys[item] : 0ull;
    const int t = int(threadIdx.x);
    if (key == 0ull) {
        if (t == 0) a.found[item] = 0;
        return;
    }
    __shared__ double S[kFskSums];
    if (t < kFskSums) {
        double v = 0.0;
        for (int p = 0; p < kFskParts; ++p) v += a.partial[(size_t(item) * kFskParts + p) * kFskSums + t];
        S[t] = v;
    }
    __syncthreads();
    if (t != 0) return;
    const int64_t lam0 = int64_t(~unsigned(key & 0xffffffffull)) - kFskWin / 2;
    double A[kFskWin];
    for (int w = 0; w < kFskWin; ++w) {
        const int64_t lam = lam0 + w;
        A[w] = (lam >= 0 && lam < lags) ? fabs(S[3 * w]) : -1.0;
    }
    const double Ec = S[3 * kFskWin];
    int c = kFskWin / 2;
    bool hit = false;
    for (int pass = 0; pass < 2; ++pass) {
        int wb = c;
        for (int w = c - 1; w <= c + 1; ++w)
            if (A[w] > A[wb] || (A[w] == A[wb] && w < wb)) wb = w;
        const int64_t lam = lam0 + wb;
        hit = (wb == c - 1 && lam > 0) || (wb == c + 1 && lam < lags - 1);
        c = wb;
        if (!hit) break;
    }
    const int64_t lam = lam0 + c;
    unsigned flags = hit ? ACQ_DET_WINDOW_EDGE : 0u;
    const double p0 = A[c];
    const double pm = A[c - 1] < 0.0 ? 0.0 : A[c - 1];
    const double pp = A[c + 1] < 0.0 ? 0.0 : A[c + 1];
    double delta = 0.0;
    if (lam == 0 || lam == lags - 1) {
        flags |= ACQ_DET_NEAR_EDGE;
    } else {
        const double den = pm - 2.0 * p0 + pp;
        if (den < 0.0) {
            delta = 0.5 * (pm - pp) / den;
            delta = delta > 0.5 ? 0.5 : (delta < -0.5 ? -0.5 : delta);
        }
    }
    acq_fsk_detection r;
    r.tag = fi.tag;
    r.block = fi.block;
    r.reserved = 0;
    r.flags = flags;
    r.lag = lam;
    r.toa_samples = double(lam) + delta;
    r.xcorr = S[3 * c];
    r.p = S[3 * c + 1];
    r.q = S[3 * c + 2];
    r.z = (r.q > 0.0 && Ec > 0.0) ? r.xcorr * r.xcorr / (r.q * Ec) : 0.0;
    a.dets[item] = r;
    a.found[item] = (a.theta <= 0.0 || r.z >= a.theta) ? 1 : 0;
}

// Results in tag order: one workgroup of 1024 threads, runs of tags per
// thread, a scan of the counts gives each run's output offset.
__global__ __launch_bounds__(1024) void k_fsk_compact(const acq_fsk_detection* __restrict__ dets,
                                                      const int32_t* __restrict__ found, int T,
                                                      acq_fsk_detection* __restrict__ out,
                                                      int32_t* __restrict__ count) {
    __shared__ int scan[1024];
    const int t = int(threadIdx.x);
    const int per = (T + 1023) / 1024;
    const int b0 = min(T, t * per), b1 = min(T, b0 + per);
    int c = 0;
    for (int i = b0; i < b1; ++i) c += found[i] ? 1 : 0;
    scan[t] = c;
    __syncthreads();
    for (int off = 1; off < 1024; off <<= 1) {
        const int v = t >= off ? scan[t - off] : 0;
        __syncthreads();
        scan[t] += v;
        __syncthreads();
    }
    int o = scan[t] - c;
    for (int i = b0; i < b1; ++i)
        if (found[i]) out[o++] = dets[i];
    if (t == 1023) *count = scan[t];
}

template <class E, int PP>
void launch_fsk_corr_ep(const FskCorrArgs& a, int grid, hipStream_t st) {
    const bool track = a.tasks.track != 0;
    // one phase per work item (split) is built for P <= 8 (eighth roots of unity)
    constexpr bool can_split = PP > 1 && PP <= 8;
    if (a.dump)                                          // searching only
        hipLaunchKernelGGL((k_fsk_correlate<E, PP, true, false, false>), dim3(grid), dim3(E::NT), 0, st, a);
    else if (can_split && a.split && track)
        hipLaunchKernelGGL((k_fsk_correlate<E, PP, false, can_split, true>), dim3(grid), dim3(E::NT), 0, st, a);
    else if (can_split && a.split)
        hipLaunchKernelGGL((k_fsk_correlate<E, PP, false, can_split, false>), dim3(grid), dim3(E::NT), 0, st, a);
    else if (track)
        hipLaunchKernelGGL((k_fsk_correlate<E, PP, false, false, true>), dim3(grid), dim3(E::NT), 0, st, a);
    else
        hipLaunchKernelGGL((k_fsk_correlate<E, PP, false, false, false>), dim3(grid), dim3(E::NT), 0, st, a);
}

// M <= 2^14 runs as one phase (P = 1) on the Stockham engine of that size;
// larger M as P = M / 2^14 phases on the 2^14-point engine.
hipError_t launch_fsk_correlate(const FskCorrArgs& a, int grid, int log2_sub, hipStream_t st) {
    if (grid <= 0) return hipSuccess;
    if ((log2_sub < 14 && a.P != 1) || (1 << log2_sub) != a.Msub) return hipErrorInvalidValue;
    switch (log2_sub) {
        case 10: launch_fsk_corr_ep<StockhamEngine<10>, 1>(a, grid, st); break;
        case 11: launch_fsk_corr_ep<StockhamEngine<11>, 1>(a, grid, st); break;
        case 12: launch_fsk_corr_ep<StockhamEngine<12>, 1>(a, grid, st); break;
        case 13: launch_fsk_corr_ep<StockhamEngine<13>, 1>(a, grid, st); break;
        case 14:
            switch (a.P) {
                case 1: launch_fsk_corr_ep<Fft14, 1>(a, grid, st); break;
                case 2: launch_fsk_corr_ep<Fft14, 2>(a, grid, st); break;
                case 4: launch_fsk_corr_ep<Fft14, 4>(a, grid, st); break;
                case 8: launch_fsk_corr_ep<Fft14, 8>(a, grid, st); break;
                case 16: launch_fsk_corr_ep<Fft14, 16>(a, grid, st); break;
                default: return hipErrorInvalidValue;
            }
            break;
        default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

// ------------------------------------------------------------------ host side
struct FskGeometry {
    int64_t lg = 0, nt = 0, M = 0, Msub = 0, V = 0, vf = 0, max_seg = 0, max_front_seg = 0, bytes = 0;
    int64_t slots = 0;          // packed segment pairs a call may use
    int P = 1, log2_sub = 0;
    int max_tasks = 16;         // tracking tasks per call
    int items = 0;              // results per call: max(templates, tasks)
};

int fsk_geometry(const acq_fsk_config* c, FskGeometry* g) {
    if (!c) return fail(ACQ_ERR_INVALID_ARG, "null configuration");
    if (!(c->sample_rate_hz > 0.0) || !std::isfinite(c->lo_hz) || !std::isfinite(c->f1_hz) ||
        !std::isfinite(c->f0_hz) || !std::isfinite(c->threshold))
        return fail(ACQ_ERR_INVALID_ARG, "sample rate must be positive and frequencies finite");
    if (!c->bp_taps || !c->bits) return fail(ACQ_ERR_INVALID_ARG, "null taps or bits");
    if (c->bp_len < 1 || c->bp_len > 1024) return fail(ACQ_ERR_INVALID_ARG, "bp_len outside [1, 1024]");
    if (c->mf_len < 1 || c->mf_len > 64) return fail(ACQ_ERR_INVALID_ARG, "mf_len outside [1, 64]");
    if (c->num_tags < 1 || c->num_bits < 1) return fail(ACQ_ERR_INVALID_ARG, "num_tags and num_bits must be >= 1");
    if (c->max_block_len < 1) return fail(ACQ_ERR_INVALID_ARG, "max_block_len must be >= 1");
    g->lg = int64_t(c->bp_len) + c->mf_len - 1;
    g->nt = int64_t(c->num_bits) * c->mf_len + g->lg - 1;
    g->vf = kFrontN - g->lg + 1;
    constexpr int64_t kMaxM = int64_t(1) << 18;
    int64_t M = c->fft_len;
    if (M == 0) {
        M = 1024;
        while (M <= g->nt && M < kMaxM) M <<= 1;      // smallest power of two > n_t ...
        if (M < kMaxM && M - g->nt + 1 < g->nt / 2) M <<= 1;   // ... doubled when few lags remain
        // ... or, from 2^17 (templates of the paper's length), doubled when
        // that needs fewer transform points for the plan's blocks: one window
        // of max_block_len samples, or, when the plan is sized for tracking
        // tasks, max_track_tasks blocks of equal length
        if (M >= (int64_t(1) << 17) && M > g->nt && 2 * M <= kMaxM) {
            const int64_t tasks = c->max_track_tasks > 0 ? c->max_track_tasks : 1;
            const int64_t len = (c->max_block_len + tasks - 1) / tasks;
            auto points = [&](int64_t m) {
                const int64_t lags = std::max<int64_t>(len - g->nt + 1, 1), v = m - g->nt + 1;
                return tasks * ((lags + v - 1) / v + 1) / 2 * m;       // segments two to a transform
            };
            if (points(2 * M) < points(M)) M *= 2;
        }
    }
    if (M < 1024 || M > kMaxM || (M & (M - 1)))
        return fail(ACQ_ERR_UNSUPPORTED, "fft_len must be a power of two in [2^10, 2^18]");
    if (M <= g->nt) return fail(ACQ_ERR_UNSUPPORTED, "template longer than the correlation segment (at most 2^18 - 1)");
    g->M = M;
    g->Msub = std::min<int64_t>(M, int64_t(1) << 14);
    g->P = int(M / g->Msub);
    g->log2_sub = 0;
    while ((int64_t(1) << g->log2_sub) < g->Msub) ++g->log2_sub;
    g->V = M - g->nt + 1;
    const int64_t lags = c->max_block_len - g->nt + 1;
    g->max_seg = lags > 0 ? (lags + g->V - 1) / g->V : 0;
    g->max_front_seg = (c->max_block_len + g->vf - 1) / g->vf;
    if (c->max_track_tasks < 0 || c->max_track_tasks > 65536)
        return fail(ACQ_ERR_INVALID_ARG, "max_track_tasks outside [0, 65536]");
    g->max_tasks = c->max_track_tasks > 0 ? c->max_track_tasks : 16;
    // a searching window uses ceil(max_seg / 2) slots; tracking blocks of total
    // length <= max_block_len have at most max_block_len / V + one segment per
    // task, two to a slot (the bound below keeps room for one slot per task)
    g->slots = (g->max_seg + 1) / 2 + g->max_tasks + 1;
    g->items = std::max<int>(c->num_tags, g->max_tasks);
    const int64_t T = c->num_tags;
    const int64_t slots = g->slots;
    g->bytes = c->max_block_len * 8 + 2 * slots * M * 8 + std::min<int64_t>(T * slots, kFskMaxGrid) * M * 8 +
               2 * T * M * 8 + T * c->num_bits * 9 + int64_t(g->items) * (kFskParts * kFskSums * 8 + 64) +
               kFrontN * 8 * 3 + M * 8 + g->Msub * 8 + T * (8 + 4 + 2 * int64_t(sizeof(acq_fsk_detection)));
    return ACQ_OK;
}

// composed filter h_BP * h_b, FP64
std::vector<double> composed(const acq_fsk_config* c, double f_hz) {
    const int lb = c->bp_len, lm = c->mf_len;
    std::vector<double> g(size_t(2 * (lb + lm - 1)), 0.0);
    const double two_pi = 6.283185307179586476925286766559;
    for (int k = 0; k < lm; ++k) {
        // h_b[k] = exp(-j 2 pi f (lm-1-k) / Fs), phase reduced in cycles
        double cyc = -f_hz * double(lm - 1 - k) / c->sample_rate_hz;
        cyc -= std::floor(cyc);
        const double hr = std::cos(two_pi * cyc), hi = std::sin(two_pi * cyc);
        for (int i = 0; i < lb; ++i) {
            const double br = c->bp_taps[2 * i], bi = c->bp_taps[2 * i + 1];
            g[size_t(2 * (i + k))] += br * hr - bi * hi;
            g[size_t(2 * (i + k) + 1)] += br * hi + bi * hr;
        }
    }
    return g;
}

// DFT_kFrontN(g) / kFrontN in FP64 (direct sum, exact index reduction), as FP32 pairs
std::vector<float> filter_spectrum(const std::vector<double>& g) {
    const int64_t lg = int64_t(g.size() / 2);
    const std::vector<double> roots = unit_roots64(kFrontN);        // (cos, sin)(2 pi m / N)
    std::vector<float> out(size_t(2 * kFrontN));
    for (int64_t k = 0; k < kFrontN; ++k) {
        double re = 0.0, im = 0.0;
        for (int64_t i = 0; i < lg; ++i) {
            const int64_t e = (i * k) % kFrontN;
            const double cr = roots[size_t(2 * e)], ci = -roots[size_t(2 * e + 1)];   // exp(-j 2 pi i k / N)
            re += g[size_t(2 * i)] * cr - g[size_t(2 * i + 1)] * ci;
            im += g[size_t(2 * i)] * ci + g[size_t(2 * i + 1)] * cr;
        }
        out[size_t(2 * k)] = float(re / kFrontN);
        out[size_t(2 * k + 1)] = float(im / kFrontN);
    }
    return out;
}

}  // namespace
}  // namespace acq

using acq::BlockDesc;
using acq::BlockTable;

struct acq_fsk_plan_s {
    acq_fsk_config cfg{};
    acq::FskGeometry g;
    hipStream_t stream = nullptr;
    float2* d_G1 = nullptr;             // [kFrontN]
    float2* d_G0 = nullptr;
    float2* d_rootsF = nullptr;         // [kFrontN]
    uint8_t* d_bits = nullptr;          // [T][nbits]
    double* d_bitcyc = nullptr;         // [T][nbits]
    float2* d_tmpl = nullptr;           // [T][M] (d^(c), 0), zero beyond n_t
    float2* d_bank = nullptr;           // [T][M] conj(DFT_M(d^(c))) / M
    float* d_d = nullptr;               // [max_block_len] demodulated d
    float* d_u = nullptr;               // [max_block_len] u
    float2* d_zp = nullptr;             // [slots][M] packed segment pairs of d
    float2* d_X = nullptr;              // [slots][M] their spectra
    float2* d_scratch = nullptr;        // [correlation workgroups][M]
    double* d_partial = nullptr;        // [T][parts][sums] refinement partial sums
    int corr_grid = 0;
    float2* d_rootsM = nullptr;
    float2* d_rootsSub = nullptr;
    float2* d_b1tab = nullptr;
    double* d_zero = nullptr;           // [1] residual offset 0 for the forward transform
    BlockDesc* d_tdescs = nullptr;      // [T] templates as blocks of the forward transform
    int32_t* d_tcounts = nullptr;       // [2]
    unsigned long long* d_keys = nullptr;
    acq_fsk_detection* d_dets = nullptr;
    acq_fsk_detection* d_out = nullptr;
    int32_t* d_found = nullptr;
    int32_t* d_count = nullptr;
    acq::FskTask* d_tasks = nullptr;        // [max_tasks] blocks of a call
    acq::FskTask* h_tasks = nullptr;        // pinned [max_tasks]
    acq_fsk_detection* h_out = nullptr;     // pinned [items]
    int32_t* h_count = nullptr;             // pinned [1]
    bool profiling = false;
    hipEvent_t ev[ACQ_FSK_NUM_KERNELS][2] = {};
};

namespace {

#define FSK_HIP(call)                                                                          \
    do {                                                                                       \
        hipError_t e_ = (call);                                                                \
        if (e_ != hipSuccess)                                                                  \
            return acq::fail(e_ == hipErrorOutOfMemory ? ACQ_ERR_OOM : ACQ_ERR_DEVICE,         \
                             std::string(#call) + ": " + hipGetErrorString(e_));               \
    } while (0)

template <typename T>
hipError_t dalloc(T** p, size_t count) {
    return hipMalloc(reinterpret_cast<void**>(p), sizeof(T) * (count ? count : 1));
}

// Event pair around one launch when profiling is on.
struct FskTimer {
    acq_fsk_plan_s* p;
    int id;
    FskTimer(acq_fsk_plan_s* plan, int kernel) : p(plan), id(kernel) {
        if (p->profiling) (void)hipEventRecord(p->ev[id][0], p->stream);
    }
    ~FskTimer() {
        if (p->profiling) (void)hipEventRecord(p->ev[id][1], p->stream);
    }
};

void free_fsk(acq_fsk_plan_s* p) {
    if (!p) return;
    for (auto& pair : p->ev)
        for (hipEvent_t e : pair)
            if (e) (void)hipEventDestroy(e);
    void* dev[] = {p->d_G1, p->d_G0, p->d_rootsF, p->d_bits, p->d_bitcyc, p->d_tmpl, p->d_bank, p->d_d, p->d_u, p->d_zp, p->d_X, p->d_scratch, p->d_partial,
                   p->d_rootsM, p->d_rootsSub, p->d_b1tab, p->d_zero, p->d_tdescs, p->d_tcounts, p->d_keys,
                   p->d_dets, p->d_out, p->d_found, p->d_count};
    for (void* d : dev)
        if (d) (void)hipFree(d);
    if (p->h_out) (void)hipHostFree(p->h_out);
    if (p->h_tasks) (void)hipHostFree(p->h_tasks);
    if (p->d_tasks) (void)hipFree(p->d_tasks);
    if (p->h_count) (void)hipHostFree(p->h_count);
    delete p;
}

// Replica mode writes `out` ([T][M]); block mode processes the call's blocks
// (device task table, fsegs front-end segments in all) into the plan's d, u.
hipError_t launch_front(acq_fsk_plan_s* p, const acq::FskTasks& tasks, int fsegs, bool replica, float2* out) {
    const acq_fsk_config& c = p->cfg;
    acq::FrontArgs a{};
    a.tasks = tasks;
    a.bits = p->d_bits;
    a.bit_cyc = p->d_bitcyc;
    a.G1 = p->d_G1;
    a.G0 = p->d_G0;
    a.roots = p->d_rootsF;
    a.out = out;
    a.out_d = p->d_d;
    a.out_u = p->d_u;
    a.n_in = int64_t(c.num_bits) * c.mf_len;
    a.n_out = p->g.nt;
    a.out_stride = p->g.M;
    a.lo_cyc = c.lo_hz / c.sample_rate_hz;
    {
        using E = acq::kdev::StockhamEngine<acq::kFrontLog>;
        for (int m = 0; m < 16; ++m) {
            double cyc = -a.lo_cyc * double(int64_t(E::NT) * m);
            cyc -= std::floor(cyc);
            a.lo_step[m] = make_float2(float(std::cos(2.0 * M_PI * cyc)), float(std::sin(2.0 * M_PI * cyc)));
        }
    }
    a.f1_cyc = c.f1_hz / c.sample_rate_hz;
    a.f0_cyc = c.f0_hz / c.sample_rate_hz;
    a.nbits = c.num_bits;
    a.sps = c.mf_len;
    a.lg = int(p->g.lg);
    a.vf = int(p->g.vf);
    a.nseg = int((a.n_out + p->g.vf - 1) / p->g.vf);
    a.replica = replica ? 1 : 0;
    const unsigned grid = replica ? unsigned(a.nseg) * unsigned(c.num_tags) : unsigned(fsegs);
    if (grid == 0) return hipSuccess;
    hipLaunchKernelGGL(acq::k_fsk_front, dim3(grid), dim3(256), 0, p->stream, a);
    return hipGetLastError();
}

acq::FwdArgs fwd_args(acq_fsk_plan_s* p, const BlockTable& bt, float2* X, int64_t V) {
    acq::FwdArgs fa{};
    fa.blocks = bt;
    fa.X = X;
    fa.Xh = nullptr;
    fa.exps = nullptr;
    fa.cls_cyc = p->d_zero;
    fa.ncls = 1;
    fa.rootsM = p->d_rootsM;
    fa.rootsSub = p->d_rootsSub;
    fa.b1tab = p->d_b1tab;
    fa.V = V;
    fa.xstride = p->g.M;             // unpadded [slots][M]
    fa.xpad = 0;
    fa.spc = p->g.P;
    fa.M = int(p->g.M);
    fa.Msub = int(p->g.Msub);
    return fa;
}

int build_fsk(acq_fsk_plan_s* p, const acq_fsk_config* cfg) {
    const acq::FskGeometry& g = p->g;
    const acq_fsk_config& c = *cfg;
    const size_t T = size_t(c.num_tags), NB = size_t(c.num_bits), M = size_t(g.M);
    hipStream_t st = p->stream;
    FSK_HIP(dalloc(&p->d_G1, size_t(acq::kFrontN)));
    FSK_HIP(dalloc(&p->d_G0, size_t(acq::kFrontN)));
    FSK_HIP(dalloc(&p->d_rootsF, size_t(acq::kFrontN)));
    FSK_HIP(dalloc(&p->d_bits, T * NB));
    FSK_HIP(dalloc(&p->d_bitcyc, T * NB));
    FSK_HIP(dalloc(&p->d_tmpl, T * M));
    FSK_HIP(dalloc(&p->d_bank, T * M));
    const size_t slots = size_t(g.slots);
    const size_t items = size_t(g.items);
    FSK_HIP(dalloc(&p->d_d, size_t(c.max_block_len)));
    FSK_HIP(dalloc(&p->d_u, size_t(c.max_block_len)));
    FSK_HIP(dalloc(&p->d_zp, slots * M));
    FSK_HIP(dalloc(&p->d_X, slots * M));
    p->corr_grid = int(std::min<size_t>(T * slots, size_t(acq::kFskMaxGrid)));
    FSK_HIP(dalloc(&p->d_tasks, size_t(g.max_tasks)));
    FSK_HIP(hipHostMalloc(reinterpret_cast<void**>(&p->h_tasks), sizeof(acq::FskTask) * size_t(g.max_tasks)));
    FSK_HIP(dalloc(&p->d_scratch, size_t(p->corr_grid) * M));
    FSK_HIP(dalloc(&p->d_rootsM, M));
    FSK_HIP(dalloc(&p->d_rootsSub, size_t(g.Msub)));
    const std::vector<float> b1 = g.log2_sub == 14 ? acq::fft14_b1_table() : std::vector<float>(2, 0.f);
    FSK_HIP(dalloc(&p->d_b1tab, b1.size() / 2));
    FSK_HIP(dalloc(&p->d_zero, 1));
    FSK_HIP(dalloc(&p->d_tdescs, T));
    FSK_HIP(dalloc(&p->d_tcounts, 2));
    FSK_HIP(dalloc(&p->d_keys, items));
    FSK_HIP(dalloc(&p->d_partial, items * size_t(acq::kFskParts) * size_t(acq::kFskSums)));
    FSK_HIP(dalloc(&p->d_dets, items));
    FSK_HIP(dalloc(&p->d_out, items));
    FSK_HIP(dalloc(&p->d_found, items));
    FSK_HIP(dalloc(&p->d_count, 1));
    FSK_HIP(hipHostMalloc(reinterpret_cast<void**>(&p->h_out), sizeof(acq_fsk_detection) * items));
    FSK_HIP(hipHostMalloc(reinterpret_cast<void**>(&p->h_count), sizeof(int32_t)));

    // tables: composed filter spectra, unit roots, replica bit phases (FP64 on the host)
    const std::vector<float> G1 = acq::filter_spectrum(acq::composed(&c, c.f1_hz));
    const std::vector<float> G0 = acq::filter_spectrum(acq::composed(&c, c.f0_hz));
    const std::vector<float> rootsF = acq::unit_roots(acq::kFrontN);
    const std::vector<float> rootsM = acq::unit_roots(g.M);
    const std::vector<float> rootsSub = acq::unit_roots(g.Msub);
    std::vector<double> bitcyc(T * NB);
    std::vector<uint8_t> bits(T * NB);
    for (size_t t = 0; t < T; ++t) {
        long double acc = 0.0L;                   // cycles at the bit start, reduced as it grows
        for (size_t b = 0; b < NB; ++b) {
            const uint8_t bit = c.bits[t * NB + b] ? 1 : 0;
            bits[t * NB + b] = bit;
            bitcyc[t * NB + b] = double(acc);
            acc += (long double)(bit ? c.f1_hz : c.f0_hz) * (long double)c.mf_len / (long double)c.sample_rate_hz;
            acc -= std::floor(acc);
        }
    }
    const double zero = 0.0;
    FSK_HIP(hipMemcpyAsync(p->d_G1, G1.data(), G1.size() * sizeof(float), hipMemcpyHostToDevice, st));
    FSK_HIP(hipMemcpyAsync(p->d_G0, G0.data(), G0.size() * sizeof(float), hipMemcpyHostToDevice, st));
    FSK_HIP(hipMemcpyAsync(p->d_rootsF, rootsF.data(), rootsF.size() * sizeof(float), hipMemcpyHostToDevice, st));
    FSK_HIP(hipMemcpyAsync(p->d_rootsM, rootsM.data(), rootsM.size() * sizeof(float), hipMemcpyHostToDevice, st));
    FSK_HIP(hipMemcpyAsync(p->d_rootsSub, rootsSub.data(), rootsSub.size() * sizeof(float), hipMemcpyHostToDevice,
                           st));
    FSK_HIP(hipMemcpyAsync(p->d_b1tab, b1.data(), b1.size() * sizeof(float), hipMemcpyHostToDevice, st));
    FSK_HIP(hipMemcpyAsync(p->d_bits, bits.data(), bits.size(), hipMemcpyHostToDevice, st));
    FSK_HIP(hipMemcpyAsync(p->d_bitcyc, bitcyc.data(), bitcyc.size() * sizeof(double), hipMemcpyHostToDevice, st));
    FSK_HIP(hipMemcpyAsync(p->d_zero, &zero, sizeof(double), hipMemcpyHostToDevice, st));

    // replica templates d^(c) (zero beyond n_t), then their spectra
    const int64_t tcount = int64_t(T * M);
    hipLaunchKernelGGL(acq::k_fsk_fill, dim3(unsigned((tcount + 255) / 256)), dim3(256), 0, st, p->d_tmpl, tcount);
    FSK_HIP(hipGetLastError());
    FSK_HIP(launch_front(p, acq::FskTasks{}, 0, true, p->d_tmpl));
    std::vector<BlockDesc> descs(T);
    for (size_t t = 0; t < T; ++t) {
        BlockDesc d{};
        d.x = p->d_tmpl + t * M;
        d.n = g.nt;
        d.lags = 1;
        d.seg0 = int32_t(t);
        d.nseg = 1;
        d.tag = -1;
        descs[t] = d;
    }
    const int32_t counts[2] = {int32_t(T), int32_t(T)};
    FSK_HIP(hipMemcpyAsync(p->d_tdescs, descs.data(), T * sizeof(BlockDesc), hipMemcpyHostToDevice, st));
    FSK_HIP(hipMemcpyAsync(p->d_tcounts, counts, sizeof(counts), hipMemcpyHostToDevice, st));
    BlockTable bt{};
    bt.descs = p->d_tdescs;
    bt.counts = p->d_tcounts;
    const acq::FwdArgs fa = fwd_args(p, bt, p->d_bank, g.M);
    FSK_HIP(acq::launch_forward(fa, int(T) * g.P, int(T), g.log2_sub, ACQ_FP32, st));
    hipLaunchKernelGGL(acq::k_fsk_conj_scale, dim3(unsigned((tcount + 255) / 256)), dim3(256), 0, st, p->d_bank, tcount,
                       float(1.0 / double(g.M)));
    FSK_HIP(hipGetLastError());
    FSK_HIP(hipStreamSynchronize(st));
    return ACQ_OK;
}

int check_iq(acq_fsk_plan_s* p, const int16_t* iq, int64_t n) {
    if (!p) return acq::fail(ACQ_ERR_INVALID_ARG, "null plan");
    if (n < 0) return acq::fail(ACQ_ERR_INVALID_ARG, "negative block length");
    if (n > p->cfg.max_block_len) return acq::fail(ACQ_ERR_BLOCK_TOO_LONG, "block longer than max_block_len");
    if (n > 0 && !iq) return acq::fail(ACQ_ERR_INVALID_ARG, "null block");
    if (reinterpret_cast<uintptr_t>(iq) % 4 != 0) return acq::fail(ACQ_ERR_INVALID_ARG, "block must be 4-byte aligned");
    return ACQ_OK;
}

}  // namespace

extern "C" {

int acq_fsk_plan_geometry(const acq_fsk_config* cfg, acq_fsk_geometry* out) {
    if (!out) return acq::fail(ACQ_ERR_INVALID_ARG, "null output");
    acq::FskGeometry g;
    const int rc = acq::fsk_geometry(cfg, &g);
    if (rc != ACQ_OK) return rc;
    out->template_len = g.nt;
    out->fft_len = g.M;
    out->valid_per_segment = g.V;
    out->filter_len = g.lg;
    out->front_fft_len = acq::kFrontN;
    out->device_bytes = g.bytes;
    acq::clear_error();
    return ACQ_OK;
}

int acq_fsk_plan(const acq_fsk_config* cfg, void* stream, acq_fsk_plan_t* out) {
    if (!out) return acq::fail(ACQ_ERR_INVALID_ARG, "null output");
    *out = nullptr;
    acq::FskGeometry g;
    int rc = acq::fsk_geometry(cfg, &g);
    if (rc != ACQ_OK) return rc;
    acq_fsk_plan_s* p = new (std::nothrow) acq_fsk_plan_s();
    if (!p) return acq::fail(ACQ_ERR_OOM, "host allocation failed");
    p->cfg = *cfg;
    p->g = g;
    p->stream = static_cast<hipStream_t>(stream);
    rc = build_fsk(p, cfg);
    p->cfg.bits = nullptr;           // copied to the device; the caller keeps its buffers
    p->cfg.bp_taps = nullptr;
    if (rc != ACQ_OK) {
        free_fsk(p);
        return rc;
    }
    *out = p;
    acq::clear_error();
    return ACQ_OK;
}

int acq_fsk_release(acq_fsk_plan_t p) {
    if (p) {
        (void)hipStreamSynchronize(p->stream);
        free_fsk(p);
    }
    return ACQ_OK;
}

int acq_fsk_demod(acq_fsk_plan_t p, const int16_t* iq, int64_t n, float* d, float* u) {
    int rc = check_iq(p, iq, n);
    if (rc != ACQ_OK) return rc;
    if (n > 0 && (!d || !u)) return acq::fail(ACQ_ERR_INVALID_ARG, "null output");
    if (n == 0) return ACQ_OK;
    acq::FskTask& tk = p->h_tasks[0];
    tk = acq::FskTask{};
    tk.iq = iq;
    tk.n = n;
    tk.tag = -1;
    tk.nfseg = int((n + p->g.vf - 1) / p->g.vf);
    FSK_HIP(hipMemcpyAsync(p->d_tasks, p->h_tasks, sizeof(acq::FskTask), hipMemcpyHostToDevice, p->stream));
    FSK_HIP(launch_front(p, acq::FskTasks{p->d_tasks, 1, 0}, tk.nfseg, false, nullptr));
    FSK_HIP(hipMemcpyAsync(d, p->d_d, sizeof(float) * size_t(n), hipMemcpyDeviceToDevice, p->stream));
    FSK_HIP(hipMemcpyAsync(u, p->d_u, sizeof(float) * size_t(n), hipMemcpyDeviceToDevice, p->stream));
    FSK_HIP(hipStreamSynchronize(p->stream));
    acq::clear_error();
    return ACQ_OK;
}

int acq_fsk_template(acq_fsk_plan_t p, int32_t tag, float* out) {
    if (!p || !out) return acq::fail(ACQ_ERR_INVALID_ARG, "null argument");
    if (tag < 0 || tag >= p->cfg.num_tags) return acq::fail(ACQ_ERR_INVALID_ARG, "tag outside [0, num_tags)");
    FSK_HIP(hipMemcpy2DAsync(out, sizeof(float), p->d_tmpl + size_t(tag) * size_t(p->g.M), sizeof(float2),
                             sizeof(float), size_t(p->g.nt), hipMemcpyDeviceToDevice, p->stream));
    FSK_HIP(hipStreamSynchronize(p->stream));
    acq::clear_error();
    return ACQ_OK;
}

}  // extern "C"

namespace {

// Steps 1-7 and the peak keys on the plan's stream for the call's blocks,
// staged in h_tasks[0 .. nblocks) with iq, n and tag set (tag -1: searching,
// one block).  Fills the rest of each entry, copies the table and launches.
// dump (device [T][lags], searching only) gets c at every lag.  Returns the
// result items (templates or tasks) in *items.
int enqueue_fsk(acq_fsk_plan_s* p, int nblocks, bool track, float* dump, int* items) {
    const acq::FskGeometry& g = p->g;
    const int T = p->cfg.num_tags;
    hipStream_t st = p->stream;
    int64_t zoff = 0;
    int fsegs = 0, units = 0;
    for (int b = 0; b < nblocks; ++b) {
        acq::FskTask& tk = p->h_tasks[b];
        tk.lags = tk.n - g.nt + 1;
        tk.zoff = zoff;
        tk.nseg = tk.lags > 0 ? int((tk.lags + g.V - 1) / g.V) : 0;
        tk.nfseg = tk.lags > 0 ? int((tk.n + g.vf - 1) / g.vf) : 0;
        tk.fseg0 = fsegs;
        tk.unit0 = units;
        zoff += tk.n;
        fsegs += tk.nfseg;
        units += tk.nseg;
    }
    const int slots = (units + 1) / 2;              // correlation segments 2s and 2s+1 share slot s
    if (zoff > p->cfg.max_block_len) return acq::fail(ACQ_ERR_BLOCK_TOO_LONG, "blocks longer than max_block_len in all");
    if (slots > g.slots) return acq::fail(ACQ_ERR_BLOCK_TOO_LONG, "blocks need more segments than the plan holds");
    *items = track ? nblocks : T;
    FSK_HIP(hipMemcpyAsync(p->d_tasks, p->h_tasks, sizeof(acq::FskTask) * size_t(nblocks), hipMemcpyHostToDevice, st));
    acq::FskTasks tt{p->d_tasks, nblocks, track ? 1 : 0};
    FSK_HIP(acq::launch_fill_u64(p->d_keys, *items, st));
    if (slots == 0) return ACQ_OK;
    {
        FskTimer kt(p, ACQ_FSK_KERNEL_FRONT);
        FSK_HIP(launch_front(p, tt, fsegs, false, nullptr));
    }
    const int64_t packed = int64_t(slots) * g.M;      // M is a power of two >= 2^10
    if (packed / 4096 >= 512)
        hipLaunchKernelGGL(acq::k_fsk_pack<4096>, dim3(unsigned(packed / std::min<int64_t>(g.M, 4096))), dim3(256), 0,
                           st, tt, p->d_d, g.V, g.M, units, p->d_zp);
    else
        hipLaunchKernelGGL(acq::k_fsk_pack<1024>, dim3(unsigned(packed / std::min<int64_t>(g.M, 1024))), dim3(256), 0,
                           st, tt, p->d_d, g.V, g.M, units, p->d_zp);
    FSK_HIP(hipGetLastError());
    BlockTable bt{};
    bt.one.x = p->d_zp;
    bt.one.n = packed;
    bt.one.lags = packed;
    bt.one.seg0 = 0;
    bt.one.nseg = slots;
    bt.one.tag = -1;
    const acq::FwdArgs fa = fwd_args(p, bt, p->d_X, g.M);
    {
        FskTimer kt(p, ACQ_FSK_KERNEL_FORWARD);
        FSK_HIP(acq::launch_forward(fa, slots * g.P, slots, g.log2_sub, ACQ_FP32, st));
    }
    acq::FskCorrArgs ca{};
    ca.X = p->d_X;
    ca.bank = p->d_bank;
    ca.rootsM = p->d_rootsM;
    ca.rootsSub = p->d_rootsSub;
    ca.b1tab = p->d_b1tab;
    ca.keys = p->d_keys;
    ca.dump = dump;
    ca.tasks = tt;
    ca.V = g.V;
    ca.M = int(g.M);
    ca.Msub = int(g.Msub);
    ca.P = g.P;
    ca.T = T;
    ca.scratch = p->d_scratch;
    ca.nslots = slots;
    ca.units = units;
    int64_t work = track ? int64_t(slots) : int64_t(T) * slots;
    int grid = int(std::min<int64_t>(work, p->corr_grid));
    if (!dump && g.P > 1 && g.P <= 8 && work < acq::kFskMaxGrid) {   // fewer items than CUs: one phase per workgroup
        ca.split = 1;
        work *= g.P;
        grid = int(std::min<int64_t>(work, acq::kFskSplitMaxGrid));
    }
    {
        FskTimer kt(p, ACQ_FSK_KERNEL_CORRELATE);
        FSK_HIP(acq::launch_fsk_correlate(ca, grid, g.log2_sub, st));
    }
    return ACQ_OK;
}

// Step 8 for the call's result items, compaction and the copy to the host.
int finish_fsk(acq_fsk_plan_s* p, int nblocks, bool track, int items, acq_fsk_detection* out, int32_t capacity,
               int32_t* n_found) {
    const acq::FskGeometry& g = p->g;
    hipStream_t st = p->stream;
    acq::FskRefineArgs ra{};
    ra.d = p->d_d;
    ra.u = p->d_u;
    ra.tmpl = p->d_tmpl;
    ra.keys = p->d_keys;
    ra.partial = p->d_partial;
    ra.dets = p->d_dets;
    ra.found = p->d_found;
    ra.tasks = acq::FskTasks{p->d_tasks, nblocks, track ? 1 : 0};
    ra.nt = g.nt;
    ra.tstride = g.M;
    ra.theta = p->cfg.threshold;
    {
        FskTimer kt(p, ACQ_FSK_KERNEL_REFINE);
        hipLaunchKernelGGL(acq::k_fsk_refine_sums, dim3(unsigned(items) * acq::kFskParts), dim3(256), 0, st, ra);
        FSK_HIP(hipGetLastError());
        hipLaunchKernelGGL(acq::k_fsk_refine_final, dim3(unsigned(items)), dim3(64), 0, st, ra);
        FSK_HIP(hipGetLastError());
    }
    hipLaunchKernelGGL(acq::k_fsk_compact, dim3(1), dim3(1024), 0, st, p->d_dets, p->d_found, items, p->d_out,
                       p->d_count);
    FSK_HIP(hipGetLastError());
    FSK_HIP(hipMemcpyAsync(p->h_count, p->d_count, sizeof(int32_t), hipMemcpyDeviceToHost, st));
    FSK_HIP(hipMemcpyAsync(p->h_out, p->d_out, sizeof(acq_fsk_detection) * size_t(items), hipMemcpyDeviceToHost, st));
    FSK_HIP(hipStreamSynchronize(st));
    const int32_t found = *p->h_count;
    *n_found = found;
    const int32_t ncopy = found < capacity ? found : capacity;
    if (ncopy > 0) std::memcpy(out, p->h_out, sizeof(acq_fsk_detection) * size_t(ncopy));
    if (found > capacity) return acq::fail(ACQ_ERR_TRUNCATED, "more detections than capacity");
    acq::clear_error();
    return ACQ_OK;
}

}  // namespace

extern "C" {

int acq_fsk_set_profiling(acq_fsk_plan_t p, int on) {
    if (!p) return acq::fail(ACQ_ERR_INVALID_ARG, "null plan");
    if (on && !p->ev[0][0])
        for (auto& pair : p->ev)
            for (hipEvent_t& e : pair) FSK_HIP(hipEventCreate(&e));
    p->profiling = on != 0;
    return ACQ_OK;
}

int acq_fsk_last_kernel_times(acq_fsk_plan_t p, double* ms, int32_t n) {
    if (!p || !ms || n < ACQ_FSK_NUM_KERNELS) return acq::fail(ACQ_ERR_INVALID_ARG, "bad arguments");
    if (!p->profiling) return acq::fail(ACQ_ERR_INVALID_ARG, "profiling is off");
    for (int k = 0; k < ACQ_FSK_NUM_KERNELS; ++k) {
        float t = 0.f;
        FSK_HIP(hipEventElapsedTime(&t, p->ev[k][0], p->ev[k][1]));
        ms[k] = t;
    }
    return ACQ_OK;
}

int acq_fsk_xcorr(acq_fsk_plan_t p, const int16_t* iq, int64_t n, float* out) {
    int rc = check_iq(p, iq, n);
    if (rc != ACQ_OK) return rc;
    if (n < p->g.nt) return acq::fail(ACQ_ERR_INVALID_ARG, "block shorter than a template");
    if (!out) return acq::fail(ACQ_ERR_INVALID_ARG, "null output");
    p->h_tasks[0] = acq::FskTask{};
    p->h_tasks[0].iq = iq;
    p->h_tasks[0].n = n;
    p->h_tasks[0].tag = -1;
    int items = 0;
    rc = enqueue_fsk(p, 1, false, out, &items);
    if (rc != ACQ_OK) return rc;
    FSK_HIP(hipStreamSynchronize(p->stream));
    acq::clear_error();
    return ACQ_OK;
}

int acq_fsk_detect(acq_fsk_plan_t p, const int16_t* iq, int64_t n, acq_fsk_detection* out, int32_t capacity,
                   int32_t* n_found) {
    int rc = check_iq(p, iq, n);
    if (rc != ACQ_OK) return rc;
    if (!n_found) return acq::fail(ACQ_ERR_INVALID_ARG, "null n_found");
    if (capacity < 0 || (capacity > 0 && !out)) return acq::fail(ACQ_ERR_INVALID_ARG, "bad output buffer");
    *n_found = 0;
    if (n < p->g.nt) {
        acq::clear_error();
        return ACQ_OK;
    }
    p->h_tasks[0] = acq::FskTask{};
    p->h_tasks[0].iq = iq;
    p->h_tasks[0].n = n;
    p->h_tasks[0].tag = -1;
    int items = 0;
    rc = enqueue_fsk(p, 1, false, nullptr, &items);
    if (rc != ACQ_OK) return rc;
    return finish_fsk(p, 1, false, items, out, capacity, n_found);
}

int acq_fsk_track(acq_fsk_plan_t p, const acq_fsk_task* tasks, int32_t ntasks, acq_fsk_detection* out,
                  int32_t capacity, int32_t* n_found) {
    if (!p) return acq::fail(ACQ_ERR_INVALID_ARG, "null plan");
    if (!tasks || !n_found) return acq::fail(ACQ_ERR_INVALID_ARG, "null argument");
    if (capacity < 0 || (capacity > 0 && !out)) return acq::fail(ACQ_ERR_INVALID_ARG, "bad output buffer");
    if (ntasks < 1 || ntasks > p->g.max_tasks) return acq::fail(ACQ_ERR_INVALID_ARG, "ntasks outside [1, max_track_tasks]");
    int64_t total = 0;
    for (int32_t b = 0; b < ntasks; ++b) {
        const int rc = check_iq(p, tasks[b].iq, tasks[b].n);
        if (rc != ACQ_OK) return rc;
        if (tasks[b].tag < 0 || tasks[b].tag >= p->cfg.num_tags)
            return acq::fail(ACQ_ERR_INVALID_ARG, "task tag outside [0, num_tags)");
        total += tasks[b].n;
    }
    if (total > p->cfg.max_block_len) return acq::fail(ACQ_ERR_BLOCK_TOO_LONG, "tasks longer than max_block_len in all");
    *n_found = 0;
    for (int32_t b = 0; b < ntasks; ++b) {
        p->h_tasks[b] = acq::FskTask{};
        p->h_tasks[b].iq = tasks[b].iq;
        p->h_tasks[b].n = tasks[b].n;
        p->h_tasks[b].tag = tasks[b].tag;
    }
    int items = 0;
    const int rc = enqueue_fsk(p, ntasks, true, nullptr, &items);
    if (rc != ACQ_OK) return rc;
    return finish_fsk(p, ntasks, true, items, out, capacity, n_found);
}

}  // extern "C"
