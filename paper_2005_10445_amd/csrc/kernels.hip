// HIP kernels of the acquisition path (gfx950).
//
//   k_block_power  : FP64 partial sums of |x|^2 (mean block power Pxhat)
//   k_forward_*    : overlap-save segment j, X_j = DFT_M(x[jV .. jV+M)) with a zero
//                    tail, as spc decimated Msub-point transforms (one workgroup
//                    each) combined by one radix-spc decimation-in-time step
//   k_bank         : replica spectra conj(DFT_Msub(chip code)) / M, plan time
//   k_correlate    : the hot loop, in correlate.hip
//   k_refine_*     : FP64 re-correlation around each tag's peak, re-maximisation,
//                    parabolic vertex, z and energy
//   k_compact      : detections in tag order
//
#include <hip/hip_runtime.h>

#include <algorithm>

#include "device_common.h"
#include "host_logic.h"
#include "kernels.h"

namespace acq {

using namespace kdev;

namespace {

// ------------------------------------------------------------------ block power
// Partial sums of block b in parts[b][*]: part p sums the p-th chunk of the
// block (chunks of at least kPowerMinChunk samples, so a block of n samples
// fills the first power_parts(n) <= kPowerParts parts and no more are read).
// Item p * blocks + b, p < the parts of the longest block the plan takes;
// workgroups stride over the items, and every item is summed in the same
// order whichever workgroup takes it, so the sums are deterministic.
constexpr int kPowerMaxGrid = 4096;
constexpr int64_t kPowerMinChunk = 4096;

__host__ __device__ __forceinline__ int64_t power_chunk(int64_t n) {
    const int64_t c = (n + kPowerParts - 1) / kPowerParts;
    return c > kPowerMinChunk ? c : kPowerMinChunk;
}

__host__ __device__ __forceinline__ int power_parts(int64_t n) {
    return n > 0 ? int((n + power_chunk(n) - 1) / power_chunk(n)) : 0;
}

__global__ __launch_bounds__(256) void k_block_power(BlockTable bt, double* __restrict__ parts, int max_parts) {
    __shared__ double red[4];
    const int nb = bt.nblocks();
    const int items = nb * max_parts;
    // part-major order: the low parts of every block come first and spread
    // over distinct workgroups
    for (int it = int(blockIdx.x); it < items; it += int(gridDim.x)) {
        const int b = it % nb, part = it / nb;
        const BlockDesc d = bt.get(b);
        const int64_t chunk = power_chunk(d.n);
        const int64_t beg = int64_t(part) * chunk;
        if (beg >= d.n) continue;                    // uniform: past this block's parts
        const int64_t end = beg + chunk < d.n ? beg + chunk : d.n;
        double acc = 0.0;
        for (int64_t i = beg + threadIdx.x; i < end; i += 256) {
            const float2 v = d.x[i];
            acc += double(v.x) * double(v.x) + double(v.y) * double(v.y);
        }
        acc = wave_sum(acc);
        if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = acc;
        __syncthreads();
        if (threadIdx.x == 0) parts[size_t(b) * kPowerParts + part] = (red[0] + red[1]) + (red[2] + red[3]);
        __syncthreads();
    }
}

__global__ void k_fill_u64(unsigned long long* p, int64_t count) {
    const int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (i < count) p[i] = 0ull;
}

__global__ void k_fill_i32(int* p, int64_t count) {
    const int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (i < count) p[i] = 0;
}

// mean block power from the fixed-order partial sums
__device__ __forceinline__ double block_mean_power(const double* __restrict__ parts, int64_t n) {
    // the parts are added in index order; loads go out 32 at a time so that a
    // single thread does not wait for each one in turn
    constexpr int kBatch = 32;
    double s = 0.0;
    const int np = power_parts(n);
    int i = 0;
    for (; i + kBatch <= np; i += kBatch) {
        double v[kBatch];
#pragma unroll
        for (int j = 0; j < kBatch; ++j) v[j] = parts[i + j];
#pragma unroll
        for (int j = 0; j < kBatch; ++j) s += v[j];
    }
    for (; i < np; ++i) s += parts[i];
    return n > 0 ? s / double(n) : 0.0;
}

// ------------------------------------------------------------------ per-block statistics
// From the block power, for every block b of the table: the power-of-two
// prescale of 16-bit storage, 2^-e with e = round(log2(sqrt(M * Pxhat))) (so
// typical |X| is near 1); the power at the detection threshold, theta * L *
// Pxhat (the z >= theta test on FP32 powers); and whether the block holds a
// non-finite sample (then Pxhat is not finite: |x|^2 of a finite complex64
// value cannot overflow FP64 and every term is >= 0, so no cancellation).
// Workgroup 0 strides over the blocks and counts the non-finite ones; every
// workgroup of the launch also clears a share of the search's peak keys and
// crossing counts.
constexpr int kStatsThreads = 256;

__global__ __launch_bounds__(kStatsThreads) void k_block_stats(BlockTable bt, const double* __restrict__ parts, int M,
                                                               int64_t L, int* __restrict__ exps,
                                                               float* __restrict__ pthr, int32_t* __restrict__ bad,
                                                               int32_t* __restrict__ nbad,
                                                               unsigned long long* __restrict__ keys,
                                                               unsigned* __restrict__ cross, int64_t nclear) {
    __shared__ int s_bad;
    for (int64_t i = int64_t(blockIdx.x) * kStatsThreads + threadIdx.x; i < nclear;
         i += int64_t(gridDim.x) * kStatsThreads) {
        keys[i] = 0ull;
        cross[i] = 0u;
    }
    if (blockIdx.x != 0) return;             // workgroup 0 forms the statistics
    if (threadIdx.x == 0) s_bad = 0;
    __syncthreads();
    const int nb = bt.nblocks();
    for (int b = int(threadIdx.x); b < nb; b += kStatsThreads) {
        const BlockDesc d = bt.get(b);
        const double px = block_mean_power(parts + size_t(b) * kPowerParts, d.n);
        const bool fin = isfinite(px);
        exps[b] = fin && px > 0.0 ? int(rint(0.5 * log2(double(M) * px))) : 0;
        const double th = d.theta * double(L) * px;
        pthr[b] = fin && px > 0.0 && th <= 3.0e38 ? float(th) : __builtin_huge_valf();
        bad[b] = fin ? 0 : 1;
        if (!fin) atomicAdd(&s_bad, 1);
    }
    __syncthreads();
    if (threadIdx.x == 0) nbad[0] = s_bad;
}

// ------------------------------------------------------------------ forward spectra
// One workgroup per global segment g (looping when the grid is smaller):
// X_g = DFT_M of the segment held in slot g (segment g - seg0 of its block, or
// the listed segment when only some segments are searched), in two kernels:
//
// k_forward_sub: work item (g, r), r < spc: the Msub-point DFT of the decimated
//   samples x[base + spc*i + r] (zero beyond the block), F_r, written to
//   X_g[r*Msub + i].  One workgroup per item (a loop over items for batches).
// k_forward_combine: the radix-spc decimation-in-time step, in place per i:
//   X_g[i + q*Msub] = F_0[i] + sum_{r>=1} exp(-j 2 pi (i + q*Msub) r / M) F_r[i],
//   accumulated in FP32 in increasing r; 16-bit plans store the result scaled
//   and packed in the 16-bit copy instead.  Each spectrum sits at offset xpad
//   of its slot, with its last xpad entries copied before it and its first
//   xpad after it (rotated reads need no wrap-around).
// LDS position of transform output i for the natural-order staging: bits 0-3
// XOR-ed with a function of bits 4-7 and 10-11, so that both the engine-order
// writes and the lane-consecutive reads hit 16 distinct 8-byte banks per
// 16 lanes (a permutation of [0, N)).
__device__ __forceinline__ int out_swizzle(int i) { return i ^ (((i >> 4) + 4 * (i >> 10)) & 15); }

template <class E>
__global__ __launch_bounds__(E::NT) void k_forward_sub(FwdArgs a) {
    __shared__ float2 lds[E::LDS];
    __shared__ float2 extra[E::EXTRA];
    E eng;
    eng.init(a.rootsSub, extra);
    const __amdgpu_buffer_rsrc_t b1 = make_rsrc(a.b1tab, E::B1_TABLE * 8);
    const int per_seg = a.ncls * a.spc;
    const int items = a.blocks.total_seg() * per_seg;
    // the per_seg items of a segment read interleaved samples of one input
    // range: with one item per workgroup, place them on one XCD (workgroups
    // go to the XCDs in turn), so that its L2 fetches the range once.  Within
    // each group of kXcds * per_seg workgroups, workgroup j takes item
    // k = j / kXcds of segment j % kXcds of the group.
    const int grp = kXcds * per_seg;
    const bool xcd_map = int(gridDim.x) >= items && per_seg > 1;
    for (int b = int(blockIdx.x); b < items; b += int(gridDim.x)) {
        int it = b;
        if (xcd_map && b < items / grp * grp) {
            const int q = b / grp, j = b - q * grp;
            it = (q * kXcds + j % kXcds) * per_seg + j / kXcds;
        }
        const int g = it / per_seg, rem = it - g * per_seg, c = rem / a.spc, r = rem - c * a.spc;
        const int bi = a.blocks.block_of_segment(g);
        const BlockDesc d = a.blocks.get(bi);
        const int64_t base = int64_t(a.blocks.segment(g, d)) * a.V;
        const double cyc = a.cls_cyc[c];          // residual offset of the class (exact bins)
        float2 v[16];
#pragma unroll
        for (int m = 0; m < 16; ++m) {
            const int64_t idx = base + int64_t(a.spc) * eng.in_index(m) + r;
            v[m] = idx < d.n ? d.x[idx] : make_float2(0.f, 0.f);
            if (cyc != 0.0) {                      // x * exp(-j 2 pi cyc idx), phase reduced in FP64
                double ph = cyc * double(idx);
                ph -= floor(ph);
                float sn, cs;
                sincospif(2.0f * float(ph), &sn, &cs);
                v[m] = make_float2(fmaf(v[m].x, cs, v[m].y * sn), fmaf(v[m].y, cs, -v[m].x * sn));
            }
        }
        eng.template transform<-1>(v, lds, b1, extra);
        float2* F = a.X + (size_t(g) * size_t(a.ncls) + size_t(c)) * size_t(a.xstride) + size_t(a.xpad) +
                    size_t(r) * size_t(a.Msub);
        // outputs leave in the engine's order: put them in natural order in LDS
        // (XOR-swizzled, conflict-free both ways), then store whole lines
        const int ob = eng.out_base();
        __syncthreads();                 // every wave is done with the transform's LDS
#pragma unroll
        for (int m = 0; m < 16; ++m) lds[out_swizzle(ob + E::out_off(m))] = v[m];
        __syncthreads();
#pragma unroll
        for (int m = 0; m < 16; ++m) {
            const int i = eng.in_index(m);
            F[i] = lds[out_swizzle(i)];
        }
        __syncthreads();                 // LDS is reused by the next item
    }
}

// 256 threads per workgroup, one i per thread; a workgroup's 256 i lie in one
// slot (Msub is a multiple of 256).  Workgroups past the slots in use exit.
// SPC (= a.spc) is a template argument so the spc inputs stay in registers.
// The twiddle of phase r is the r-th power of exp(-j 2 pi io / M): one table
// load per output, then products (exact table values for spc <= 2).
template <int PREC, int SPC>
__global__ __launch_bounds__(256) void k_forward_combine(FwdArgs a) {
    using St = dev::Storage<PREC>;
    const int per_slot = a.Msub / 256;
    const int g = int(blockIdx.x) / per_slot;           // spectra slot: segment * ncls + class
    if (g >= a.blocks.total_seg() * a.ncls) return;
    const int i = (int(blockIdx.x) - g * per_slot) * 256 + int(threadIdx.x);
    float2* X = a.X + size_t(g) * size_t(a.xstride) + size_t(a.xpad);
    float xs = 1.0f;
    if constexpr (PREC != ACQ_FP32) xs = ldexpf(1.0f, -a.exps[a.blocks.block_of_segment(g / a.ncls)]);
    float2 F[SPC];
#pragma unroll
    for (int r = 0; r < SPC; ++r) F[r] = X[r * a.Msub + i];
    // 16 phases (the FSK path's 2^18-point segments): X[i + q Msub] is the
    // 16-point DFT over r of F_r[i] exp(-j 2 pi i r / M)
    if constexpr (SPC == 16) {
        const float2 w1 = a.rootsM[i];
        float2 w = w1;
#pragma unroll
        for (int r = 1; r < SPC; ++r) {
            F[r] = cmulc(F[r], w);
            if (r + 1 < SPC) w = cmul(w, w1);
        }
        dev::dft16<-1>(F);
    }
#pragma unroll
    for (int q = 0; q < SPC; ++q) {
        const int io = i + q * a.Msub;
        float2 c = F[0];
        if constexpr (SPC == 16) {
            c = F[q];
        } else if constexpr (SPC > 1) {
            const float2 w1 = a.rootsM[io];
            float2 w = w1;
#pragma unroll
            for (int r = 1; r < SPC; ++r) {
                c = cadd(c, cmulc(F[r], w));
                if (r + 1 < SPC) w = cmul(w, w1);
            }
        }
        // the spectrum, and its wrap-around copy when io is within xpad of an end
        if constexpr (PREC == ACQ_FP32) {
            X[io] = c;
            if (io < a.xpad) X[a.M + io] = c;
            if (io >= a.M - a.xpad) X[io - a.M] = c;
        } else {
            typename St::T* Xh = reinterpret_cast<typename St::T*>(a.Xh) + size_t(g) * size_t(a.xstride) +
                                 size_t(a.xpad);
            const typename St::T h = St::pack(make_float2(c.x * xs, c.y * xs));
            Xh[io] = h;
            if (io < a.xpad) Xh[a.M + io] = h;
            if (io >= a.M - a.xpad) Xh[io - a.M] = h;
        }
    }
}

// ------------------------------------------------------------------ replica bank
// bank[t][i] = 2^bank_exp * conj(DFT_Msub(chips_t))[i] / M in the storage format
template <class E, int PREC>
__global__ __launch_bounds__(E::NT) void k_bank(const int8_t* __restrict__ chips, int C,
                                                void* __restrict__ bank,
                                                const float2* __restrict__ rootsSub,
                                                const float2* __restrict__ b1tab, int M, int bank_exp) {
    using St = dev::Storage<PREC>;
    __shared__ float2 lds[E::LDS];
    __shared__ float2 extra[E::EXTRA];
    E eng;
    eng.init(rootsSub, extra);
    const __amdgpu_buffer_rsrc_t b1 = make_rsrc(b1tab, E::B1_TABLE * 8);
    const int tag = blockIdx.x;
    float2 v[16];
#pragma unroll
    for (int m = 0; m < 16; ++m) {
        const int ip = eng.in_index(m);
        v[m] = make_float2(ip < C ? float(chips[size_t(tag) * C + ip]) : 0.f, 0.f);
    }
    eng.template transform<-1>(v, lds, b1, extra);
    const float s = ldexpf(1.0f, bank_exp) / float(M);   // exact: powers of two
    const int ob = eng.out_base();
    typename St::T* out = reinterpret_cast<typename St::T*>(bank) + size_t(tag) * bank_stride(E::N);
#pragma unroll
    for (int m = 0; m < 16; ++m) {
        const int i = ob + E::out_off(m);
        if (i <= E::N / 2) out[i] = St::pack(make_float2(v[m].x * s, -v[m].y * s));   // the rest is the mirror
    }
}

// ------------------------------------------------------------------ refine
constexpr int kMaxWin = 2 * kMaxRefineRadius + 3;

// FP64 refinement of each (block, tag) peak key, in two passes of two
// kernels.  The first pass takes the window of W = 2R + 3 lags centred on the
// key's lag; k_refine_sums adds, in kRefineParts workgroups per item, the re-
// and im-sums of the mixed samples against the tag's replica and the sample
// energy under it for every lag of the window; k_refine_decide (one wave per
// item) adds the parts in order, re-maximises over the inner 2R+1 lags and
// either writes the detection or, when the maximum sits on the inner edge,
// records a re-centred window for the second pass, which repeats both steps
// once.
// The mix exp(-j 2 pi m_k i / M) is an FP64 table entry at (m_k i) mod M (M a
// power of two, so the reduction is exact), or the exact bin's FP64 phase.
struct RefineItem {
    int bi, tag;
    size_t slot;
    BlockDesc d;
};

__device__ __forceinline__ bool refine_item(const RefineArgs& a, int item, RefineItem* r) {
    const int per = a.track ? 1 : a.T;
    r->bi = item / per;
    if (r->bi >= a.blocks.nblocks()) return false;
    r->d = a.blocks.get(r->bi);
    r->tag = a.track ? r->d.tag : item % per;
    if (r->tag < 0 || r->tag >= a.T) return false;
    r->slot = size_t(r->bi) * a.T + r->tag;
    return true;
}

constexpr int kRefineChipsLds = 4096;     // chips of one part staged in LDS (else read from global)

template <int WMAX>
__global__ __launch_bounds__(256) void k_refine_sums(RefineArgs a, int pass) {
    constexpr int NT = 256, NW = NT / 64;
    const int item = int(blockIdx.x) / kRefineParts, part = int(blockIdx.x) % kRefineParts;
    RefineItem it;
    if (!refine_item(a, item, &it)) return;
    const BlockDesc& d = it.d;
    const unsigned long long key = d.lags > 0 ? a.keys[it.slot] : 0ull;
    if (key == 0ull) return;
    const unsigned idx = ~unsigned(key & 0xffffffffull);
    const int k = int(idx % unsigned(a.K));
    const int64_t center = pass == 0 ? int64_t(idx / unsigned(a.K)) : a.center[item];
    if (center < 0) return;
    const int R = a.radius;
    const int W = 2 * R + 3;
    if (W > WMAX) return;                    // the launcher picks WMAX >= W
    const int t = int(threadIdx.x), lane = t & 63, wave = t >> 6;
    const int64_t lam0 = center - R - 1;
    // samples of the window inside the block, split into parts
    const int64_t e_lo = lam0 < 0 ? -lam0 : 0;
    const int64_t e_hi = min(int64_t(a.L) + W - 1, d.n - lam0);
    const int64_t ch = (e_hi - e_lo + kRefineParts - 1) / kRefineParts;
    const int64_t p0 = e_lo + int64_t(part) * ch, p1 = min(e_hi, p0 + ch);
    // the part's chips (replica samples e - w, w < W) in LDS when they fit
    __shared__ int8_t s_chips[kRefineChipsLds];
    const int8_t* chips = a.chips + size_t(it.tag) * size_t(a.C);
    const int64_t c0 = max(int64_t(0), (p0 - W + 1) >> a.log2_spc);
    const int64_t c1 = min(int64_t(a.C), ((p1 - 1) >> a.log2_spc) + 1);
    const bool lds = c1 - c0 <= kRefineChipsLds;
    if (lds) {
        for (int64_t q = c0 + t; q < c1; q += NT) s_chips[q - c0] = chips[q];
    }
    __syncthreads();
    const int64_t mrot = a.rot_signed[k];
    const int64_t mmask = int64_t(a.M) - 1;
    const double fk = a.cyc[k];
    double cr[WMAX], ci[WMAX], en[WMAX];
#pragma unroll
    for (int w = 0; w < WMAX; ++w) cr[w] = ci[w] = en[w] = 0.0;
    for (int64_t e = p0 + t; e < p1; e += NT) {
        const int64_t i = lam0 + e;
        const float2 xv = d.x[i];
        const double xr = xv.x, xi = xv.y;
        double2 cs;
        if (a.exact) {                          // exp(-j 2 pi (f_k / Fs) i), phase reduced in FP64
            double ph = fk * double(i);
            ph -= floor(ph);
            sincospi(2.0 * ph, &cs.y, &cs.x);
        } else {
            cs = a.roots64[(mrot * i) & mmask];
        }
        const double mr = xr * cs.x + xi * cs.y;      // x * exp(-j 2 pi m i / M)
        const double mi = xi * cs.x - xr * cs.y;
        const double pw = xr * xr + xi * xi;
#pragma unroll
        for (int w = 0; w < WMAX; ++w) {
            const int64_t nn = e - w;
            if (w < W && nn >= 0 && nn < a.L) {
                const int64_t c = nn >> a.log2_spc;
                const double sg = double(lds ? s_chips[c - c0] : chips[c]);
                cr[w] += mr * sg;
                ci[w] += mi * sg;
                en[w] += pw;
            }
        }
    }
    __shared__ double red[NW][3 * WMAX];
#pragma unroll
    for (int w = 0; w < WMAX; ++w) {
        const double r0 = wave_sum(cr[w]), r1 = wave_sum(ci[w]), r2 = wave_sum(en[w]);
        if (lane == 0) {
            red[wave][3 * w] = r0;
            red[wave][3 * w + 1] = r1;
            red[wave][3 * w + 2] = r2;
        }
    }
    __syncthreads();
    if (t < 3 * W) {
        double v = 0.0;
        for (int q = 0; q < NW; ++q) v += red[q][t];
        a.partial[(size_t(item) * kRefineParts + part) * size_t(3 * WMAX) + t] = v;
    }
}

// One wave per item: lane s < 3W adds sum s over the parts in order, lane 0
// decides.
template <int WMAX>
__global__ __launch_bounds__(64) void k_refine_decide(RefineArgs a, int pass) {
    const int item = int(blockIdx.x);
    RefineItem it;
    if (!refine_item(a, item, &it)) return;
    const BlockDesc& d = it.d;
    const int t = int(threadIdx.x);
    const unsigned long long key = d.lags > 0 ? a.keys[it.slot] : 0ull;
    if (key == 0ull) {                       // no valid lag was searched for this tag
        if (pass == 0 && t == 0) {
            a.found[it.slot] = 0;
            a.center[item] = -1;
        }
        return;
    }
    const unsigned idx = ~unsigned(key & 0xffffffffull);
    const int k = int(idx % unsigned(a.K));
    const int64_t center = pass == 0 ? int64_t(idx / unsigned(a.K)) : a.center[item];
    if (center < 0) return;
    const int R = a.radius;
    const int W = 2 * R + 3;
    if (W > WMAX) return;
    __shared__ double sums[3 * WMAX];
    if (t < 3 * W) {
        double v = 0.0;
        for (int q = 0; q < kRefineParts; ++q) v += a.partial[(size_t(item) * kRefineParts + q) * size_t(3 * WMAX) + t];
        sums[t] = v;
    }
    __syncthreads();
    if (t != 0) return;
    const int64_t lam0 = center - R - 1;
    double P[WMAX], E[WMAX];
    for (int w = 0; w < W; ++w) {
        const double re = sums[3 * w], im = sums[3 * w + 1];
        E[w] = sums[3 * w + 2];
        const int64_t lam = lam0 + w;
        P[w] = (lam >= 0 && lam < d.lags) ? re * re + im * im : -1.0;
    }
    int wb = R + 1;
    for (int w = 1; w <= W - 2; ++w)
        if (P[w] > P[wb] || (P[w] == P[wb] && w < wb)) wb = w;
    const int64_t lam = lam0 + wb;
    const bool hit = (wb == 1 && lam > 0) || (wb == W - 2 && lam < d.lags - 1);
    if (pass == 0) {
        a.center[item] = hit ? lam : -1;
        if (hit) return;                     // the second pass re-centres on lam
    }
    unsigned flags = hit ? ACQ_DET_WINDOW_EDGE : 0u;
    const double p0 = P[wb];
    const double pm = P[wb - 1] < 0.0 ? 0.0 : P[wb - 1];
    const double pp = P[wb + 1] < 0.0 ? 0.0 : P[wb + 1];
    double delta = 0.0;
    if (lam == 0 || lam == d.lags - 1) {
        flags |= ACQ_DET_NEAR_EDGE;
    } else {
        const double den = pm - 2.0 * p0 + pp;
        if (den < 0.0) {
            delta = 0.5 * (pm - pp) / den;
            delta = delta > 0.5 ? 0.5 : (delta < -0.5 ? -0.5 : delta);
        }
    }
    const double px = block_mean_power(a.parts + size_t(it.bi) * kPowerParts, d.n);
    const double z = px > 0.0 ? p0 / (double(a.L) * px) : 0.0;
    const bool suppressed = a.check_finite && a.bad[it.bi];
    acq_detection r;
    r.tag = it.tag;
    r.bin = k;
    r.lag = lam;
    r.toa_samples = double(lam) + delta;
    r.freq_hz = a.freqs[k];
    r.peak_power = p0;
    r.z = z;
    r.energy = E[wb];
    r.block_power = px;
    // relative power and SNR (Section 3 step 8's power and SNR sums)
    const double Ld = double(a.L);
    r.power = p0 / (Ld * Ld);
    const double s2 = (E[wb] - p0 / Ld) / Ld;
    r.snr = s2 > 0.0 ? r.power / s2 : __builtin_huge_val();
    r.block = it.bi;
    r.flags = flags;
    r.crossings = int64_t(a.cross[it.slot]);
    a.dets[it.slot] = r;
    a.found[it.slot] = z >= d.theta && !suppressed ? 1 : 0;
}

// Detections in (block, tag) order.  One workgroup: each thread takes a
// contiguous run of candidates, counts its detections, an exclusive scan over
// the threads gives its first output slot, and it copies its run in order.
// Candidates are every (block, tag), or (block, its tag) for tracking tasks.
constexpr int kCompactThreads = 1024;

__global__ __launch_bounds__(kCompactThreads) void k_compact(BlockTable bt, const acq_detection* __restrict__ dets,
                                                             const int32_t* __restrict__ found, int T, int track,
                                                             acq_detection* __restrict__ out, int32_t capacity,
                                                             int32_t* __restrict__ count) {
    __shared__ int scan[kCompactThreads];
    const int t = int(threadIdx.x);
    const int nb = bt.nblocks();
    const int64_t n = track ? int64_t(nb) : int64_t(nb) * T;
    const int64_t per = (n + kCompactThreads - 1) / kCompactThreads;
    const int64_t e0 = min(n, int64_t(t) * per), e1 = min(n, e0 + per);
    auto slot = [&](int64_t e) -> int64_t {
        if (!track) return e;
        const int tag = bt.get(int(e)).tag;
        return tag >= 0 && tag < T ? e * T + tag : -1;
    };
    int c = 0;
    for (int64_t e = e0; e < e1; ++e) {
        const int64_t s = slot(e);
        c += s >= 0 && found[s] ? 1 : 0;
    }
    scan[t] = c;
    __syncthreads();
    for (int off = 1; off < kCompactThreads; off <<= 1) {     // inclusive Hillis-Steele scan
        const int v = t >= off ? scan[t - off] : 0;
        __syncthreads();
        scan[t] += v;
        __syncthreads();
    }
    int o = scan[t] - c;
    for (int64_t e = e0; e < e1 && o < capacity; ++e) {
        const int64_t s = slot(e);
        if (s >= 0 && found[s]) out[o++] = dets[s];
    }
    if (t == kCompactThreads - 1) *count = scan[t];
}

}  // namespace

// ------------------------------------------------------------------ launchers
hipError_t launch_block_power(const BlockTable& bt, int max_blocks, int64_t max_len, double* parts, hipStream_t st) {
    const int mp = std::max(power_parts(max_len), 1);
    const unsigned grid = unsigned(std::min<int64_t>(int64_t(max_blocks) * mp, kPowerMaxGrid));
    hipLaunchKernelGGL(k_block_power, dim3(grid), dim3(256), 0, st, bt, parts, mp);
    return hipGetLastError();
}

hipError_t launch_block_stats(const BlockTable& bt, const double* parts, int M, int64_t L, int* exps, float* pthr,
                              int32_t* bad, int32_t* nbad, unsigned long long* keys, unsigned* cross,
                              int64_t nclear, hipStream_t st) {
    // workgroup 0 forms the statistics; all of them clear, 2048 entries each
    const int64_t grid = std::max<int64_t>(1, std::min<int64_t>(256, (nclear + 2047) / 2048));
    hipLaunchKernelGGL(k_block_stats, dim3(unsigned(grid)), dim3(kStatsThreads), 0, st, bt, parts, M, L, exps, pthr,
                       bad, nbad, keys, cross, nclear);
    return hipGetLastError();
}

hipError_t launch_fill_u64(unsigned long long* p, int64_t count, hipStream_t st) {
    if (count <= 0) return hipSuccess;
    const int64_t blocks = (count + 255) / 256;
    hipLaunchKernelGGL(k_fill_u64, dim3(unsigned(blocks)), dim3(256), 0, st, p, count);
    return hipGetLastError();
}

hipError_t launch_fill_i32(int* p, int64_t count, hipStream_t st) {
    if (count <= 0) return hipSuccess;
    const int64_t blocks = (count + 255) / 256;
    hipLaunchKernelGGL(k_fill_i32, dim3(unsigned(blocks)), dim3(256), 0, st, p, count);
    return hipGetLastError();
}

template <class E>
static hipError_t fwd_e(const FwdArgs& a, int grid, hipStream_t st) {
    hipLaunchKernelGGL((k_forward_sub<E>), dim3(grid), dim3(E::NT), 0, st, a);
    return hipGetLastError();
}

template <int PREC>
static hipError_t combine_p(const FwdArgs& a, dim3 grid, hipStream_t st) {
    if constexpr (PREC == ACQ_FP32) {
        if (a.spc == 16) {                  // the FSK path's 2^18-point segments (16 phases of 2^14)
            hipLaunchKernelGGL((k_forward_combine<PREC, 16>), grid, dim3(256), 0, st, a);
            return hipSuccess;
        }
    }
    switch (a.spc) {
        case 1: hipLaunchKernelGGL((k_forward_combine<PREC, 1>), grid, dim3(256), 0, st, a); break;
        case 2: hipLaunchKernelGGL((k_forward_combine<PREC, 2>), grid, dim3(256), 0, st, a); break;
        case 3: hipLaunchKernelGGL((k_forward_combine<PREC, 3>), grid, dim3(256), 0, st, a); break;
        case 4: hipLaunchKernelGGL((k_forward_combine<PREC, 4>), grid, dim3(256), 0, st, a); break;
        case 5: hipLaunchKernelGGL((k_forward_combine<PREC, 5>), grid, dim3(256), 0, st, a); break;
        case 6: hipLaunchKernelGGL((k_forward_combine<PREC, 6>), grid, dim3(256), 0, st, a); break;
        case 7: hipLaunchKernelGGL((k_forward_combine<PREC, 7>), grid, dim3(256), 0, st, a); break;
        case 8: hipLaunchKernelGGL((k_forward_combine<PREC, 8>), grid, dim3(256), 0, st, a); break;
        default: return hipErrorInvalidValue;
    }
    return hipSuccess;
}

hipError_t launch_forward(const FwdArgs& a, int grid, int combine_slots, int log2_sub, int prec, hipStream_t st) {
    if (grid <= 0 || combine_slots <= 0) return hipSuccess;
    if ((1 << log2_sub) != a.Msub || a.Msub % 256 || a.spc < 1 || (a.spc > 8 && !(a.spc == 16 && prec == ACQ_FP32)))
        return hipErrorInvalidValue;
    if (a.xpad < 0 || a.xpad > a.M / 2 || a.xstride < int64_t(a.M) + 2 * int64_t(a.xpad)) return hipErrorInvalidValue;
    hipError_t e;
    switch (log2_sub) {
        case 10: e = fwd_e<StockhamEngine<10>>(a, grid, st); break;
        case 11: e = fwd_e<StockhamEngine<11>>(a, grid, st); break;
        case 12: e = fwd_e<StockhamEngine<12>>(a, grid, st); break;
        case 13: e = fwd_e<StockhamEngine<13>>(a, grid, st); break;
        case 14: e = fwd_e<Fft14>(a, grid, st); break;
        default: return hipErrorInvalidValue;
    }
    if (e != hipSuccess) return e;
    const dim3 cgrid(unsigned(combine_slots) * unsigned(a.Msub / 256));
    switch (prec) {
        case ACQ_FP32: e = combine_p<ACQ_FP32>(a, cgrid, st); break;
        case ACQ_FP16: e = combine_p<ACQ_FP16>(a, cgrid, st); break;
        case ACQ_BF16: e = combine_p<ACQ_BF16>(a, cgrid, st); break;
        default: return hipErrorInvalidValue;
    }
    if (e != hipSuccess) return e;
    return hipGetLastError();
}

template <class E>
static hipError_t bank_e(const int8_t* chips, int T, int C, void* bank, const float2* rootsSub,
                         const float2* b1tab, int M, int bank_exp, int prec, hipStream_t st) {
    switch (prec) {
        case ACQ_FP32:
            hipLaunchKernelGGL((k_bank<E, ACQ_FP32>), dim3(T), dim3(E::NT), 0, st, chips, C, bank, rootsSub, b1tab, M,
                               bank_exp);
            break;
        case ACQ_FP16:
            hipLaunchKernelGGL((k_bank<E, ACQ_FP16>), dim3(T), dim3(E::NT), 0, st, chips, C, bank, rootsSub, b1tab, M,
                               bank_exp);
            break;
        case ACQ_BF16:
            hipLaunchKernelGGL((k_bank<E, ACQ_BF16>), dim3(T), dim3(E::NT), 0, st, chips, C, bank, rootsSub, b1tab, M,
                               bank_exp);
            break;
        default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

hipError_t launch_bank(const int8_t* chips, int T, int C, void* bank, const float2* rootsSub,
                       const float2* b1tab, int Msub, int M, int bank_exp, int log2_sub, int prec,
                       hipStream_t st) {
    if ((1 << log2_sub) != Msub || C > Msub) return hipErrorInvalidValue;
    switch (log2_sub) {
        case 10: return bank_e<StockhamEngine<10>>(chips, T, C, bank, rootsSub, b1tab, M, bank_exp, prec, st);
        case 11: return bank_e<StockhamEngine<11>>(chips, T, C, bank, rootsSub, b1tab, M, bank_exp, prec, st);
        case 12: return bank_e<StockhamEngine<12>>(chips, T, C, bank, rootsSub, b1tab, M, bank_exp, prec, st);
        case 13: return bank_e<StockhamEngine<13>>(chips, T, C, bank, rootsSub, b1tab, M, bank_exp, prec, st);
        case 14: return bank_e<Fft14>(chips, T, C, bank, rootsSub, b1tab, M, bank_exp, prec, st);
        default: return hipErrorInvalidValue;
    }
}

hipError_t launch_refine(const RefineArgs& a, int max_blocks, hipStream_t st) {
    if (a.radius < 0 || a.radius > kMaxRefineRadius || (a.M & (a.M - 1)) || (1 << a.log2_spc) != a.spc ||
        !a.partial || !a.center)
        return hipErrorInvalidValue;
    const int items = max_blocks * (a.track ? 1 : a.T);
    const dim3 sgrid(unsigned(items) * kRefineParts), dgrid{unsigned(items)};
    for (int pass = 0; pass < 2; ++pass) {
        if (a.radius <= 1) {
            hipLaunchKernelGGL((k_refine_sums<5>), sgrid, dim3(256), 0, st, a, pass);
            hipLaunchKernelGGL((k_refine_decide<5>), dgrid, dim3(64), 0, st, a, pass);
        } else {
            hipLaunchKernelGGL((k_refine_sums<kMaxWin>), sgrid, dim3(256), 0, st, a, pass);
            hipLaunchKernelGGL((k_refine_decide<kMaxWin>), dgrid, dim3(64), 0, st, a, pass);
        }
    }
    return hipGetLastError();
}

hipError_t launch_compact(const BlockTable& bt, const acq_detection* dets, const int32_t* found, int T, int track,
                          acq_detection* out, int32_t capacity, int32_t* count, hipStream_t st) {
    hipLaunchKernelGGL(k_compact, dim3(1), dim3(kCompactThreads), 0, st, bt, dets, found, T, track, out, capacity,
                       count);
    return hipGetLastError();
}

}  // namespace acq
