// The correlation kernel of the acquisition path (gfx950): spectrum product,
// inverse transform, |c|^2 and peak keys for every tag x bin x lag.
//
// Correlation by overlap-save (the FFT identity of Section 4.1 with the
// conjugate on the replica; segmented processing as in Section 4.1's
// overlap-add remark, here overlap-save so each segment yields V = M-L+1 lags):
//
//   c_j[tau] = (1/M) sum_i X_j[(i + m_k) mod M] conj(S_t[i]) exp(+j 2 pi i tau / M)
//
// equals c[t,k,jV+tau] up to a unit-modulus factor for tau < V (the bin's
// frequency shift is the rotation by m_k = f_k M / Fs).  The replica is a
// +/-1 code held spc samples per chip, so its spectrum factors as
// S_t[i] = Chat_t[i mod Msub] * Rect[i], Msub = M / spc, with Chat_t the
// Msub-point spectrum of the chip code and Rect the spectrum of a run of spc
// ones.  Splitting i = i' + Msub*a and the output lag tau = spc*u + rho turns
// the M-point inverse transform into a radix-spc first step that does not
// depend on the tag,
//
//   G_rho[i'] = exp(+j 2 pi i' rho / M) sum_a X_j[(i'+Msub a + m_k) mod M]
//               conj(Rect[i'+Msub a]) exp(+j 2 pi a rho / spc),
//
// followed per tag by an Msub-point inverse transform of conj(Chat_t) G_rho,
// whose output u is the lag spc*u + rho.  One work item is (segment j, bin k,
// phase rho, tile of tags): it forms G_rho once in registers, then for each tag
// multiplies by the stored conj(Chat_t)/M, runs the LDS-resident inverse
// transform, squares, masks invalid lags and max-reduces a 64-bit key per tag:
// key = float_bits(P) << 32 | ~(tau*K + k), so the largest key is the largest
// power with ties going to the smaller lag and then the smaller bin (the
// argmax of Section 3, step 8).  P >= 0, so its bit pattern orders like its
// value.  Each tag also counts its threshold crossings, the (bin, lag) with
// P >= theta * L * Pxhat: each lane counts its own (invalid lags carry
// P = -1), and the wave adds the lanes' counts only when some lane has one.
#include <hip/hip_runtime.h>

#include "device_common.h"
#include "host_logic.h"
#include "kernels.h"

namespace acq {

using namespace kdev;

namespace {

// ------------------------------------------------------------------ correlation
// cos and sin of pi m / 16, m = 0 .. 8 (FP64 values rounded to FP32)
__device__ constexpr float kCos16[9] = {1.0f, 0.98078528040323044913f, 0.92387953251128675613f,
                                         0.83146961230254523708f, 0.70710678118654752440f, 0.55557023301960222474f,
                                         0.38268343236508977173f, 0.19509032201612826785f, 0.0f};

// exp(+j pi m / 16) for a register index m < 16 (a compile-time constant)
__device__ __forceinline__ float2 root32(int m) {
    return m <= 8 ? make_float2(kCos16[m], kCos16[8 - m]) : make_float2(-kCos16[16 - m], kCos16[m - 8]);
}

// First step of the split inverse transform for (global segment slot g, bin k,
// phase rho): G[m] = sum_q X_g[(i + m_k) mod M] W_rho[i], i = in_index(m) +
// q Msub, for the 16 inputs this thread holds.  The spectra are padded, so
// the rotated element is position xpad + i + r_k of the slot (r_k the bin's
// rotation reduced to (-M/2, M/2]); every load is a buffer load whose
// register offset is the same for all 16 registers.  For spc = 2 the weights
// have a closed form: with e = exp(+j 2 pi i / M) (i = in_index(m)), the two
// inputs Xa = X[i + m_k], Xb = X[i + Msub + m_k], S = Xa + Xb, D = Xa - Xb,
//   W_0 = 1 + e, 1 - e   ->  G_0 = S + e D
//   W_1 = e + e^2, e^2 - e  ->  G_1 = e (D + e S)
// and e = exp(+j 2 pi in_index(0) / M) exp(+j pi m / 16) (in_index(m) =
// in_index(0) + m Msub / 16); other spc read W from the table.
template <class E, int PREC>
__device__ __forceinline__ void first_step(const CorrArgs& a, const E& eng, int g, int k, int rho, float gscale,
                                           float2 (&G)[16]) {
    using St = dev::Storage<PREC>;
    constexpr int NT = E::N / 16;
    const size_t slot = size_t(g) * size_t(a.ncls) + size_t(a.cls[k]);
    const __amdgpu_buffer_rsrc_t xr = make_rsrc(static_cast<const char*>(a.X) + slot * size_t(a.xstride) * St::BYTES,
                                                uint32_t(a.xstride) * St::BYTES);
    const int rot = a.rot[k];
    const int rs = rot <= (a.M >> 1) ? rot : rot - a.M;          // |rs| <= xpad
    const int i0 = eng.in_index(0);
    const int xoff = (a.xpad + i0 + rs) * St::BYTES;
    if (a.spc == 2) {
        const float2 e0 = a.rootsM[i0];
        float2 xa[16], xb[16];
#pragma unroll
        for (int m = 0; m < 16; ++m) {
            xa[m] = St::bload(xr, xoff, m * NT * St::BYTES);
            xb[m] = St::bload(xr, xoff, (m * NT + a.Msub) * St::BYTES);
        }
#pragma unroll
        for (int m = 0; m < 16; ++m) {
            const float2 e = m ? cmul(e0, root32(m)) : e0;
            const float2 S = cadd(xa[m], xb[m]);
            const float2 D = make_float2(xa[m].x - xb[m].x, xa[m].y - xb[m].y);
            if (rho == 0) {
                G[m] = cadd(S, cmul(e, D));
            } else {
                G[m] = cmul(e, cadd(D, cmul(e, S)));
            }
        }
    } else {
        const __amdgpu_buffer_rsrc_t wr =
            make_rsrc(a.wts + size_t(rho) * size_t(a.M), uint32_t(a.M) * 8u);
        const int woff = i0 * 8;
#pragma unroll
        for (int m = 0; m < 16; ++m) G[m] = make_float2(0.f, 0.f);
        for (int q = 0; q < a.spc; ++q) {
            const int base = q * a.Msub;
#pragma unroll
            for (int m = 0; m < 16; ++m) {
                const int i = m * NT + base;
                G[m] = cadd(G[m], cmul(St::bload(xr, xoff, i * St::BYTES), bload(wr, woff, i * 8)));
            }
        }
    }
    if constexpr (PREC != ACQ_FP32) {
#pragma unroll
        for (int m = 0; m < 16; ++m) G[m] = make_float2(G[m].x * gscale, G[m].y * gscale);
    }
}

__device__ __forceinline__ unsigned wave_sum_u32(unsigned v) {
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v += unsigned(__shfl_xor(int(v), off, 64));
    return v;
}

// Powers of this lane's valid outputs (ob + out_off < ulim) that reach the
// threshold pth.  Only a lane whose largest power bp reaches it has any, so
// the others skip the count; the powers are formed again exactly as in the
// maximum, and the per-lane test alone decides validity (no wave-uniform
// branches, which would hold a scalar mask per register).
template <class E>
__device__ __forceinline__ unsigned lane_crossings(const float2 (&v)[16], float bp, float pth, int ob, int ulim) {
    unsigned lc = 0;
    if (bp >= pth) {
#pragma unroll
        for (int r = 0; r < 16; ++r) {
            const float p = fmaf(v[r].x, v[r].x, v[r].y * v[r].y);
            lc += (ob + E::out_off(r) < ulim && p >= pth) ? 1u : 0u;
        }
    }
    return lc;
}

// One work item: (tile of tags, global segment g, bin k, phase rho), item index
// wi = ((tile * segments + g) * K + k) * spc + rho.
template <class E, int PREC, bool DUMP>
__device__ __forceinline__ void correlate_item(const CorrArgs& a, const E& eng, int wi, int total_seg,
                                               float2* lds, const float2* extra, unsigned long long* red,
                                               unsigned* cred) {
    using St = dev::Storage<PREC>;
    constexpr int N = E::N;
    constexpr int NW = E::NT / 64;
    int rem = wi;
    const int rho = rem % a.spc;
    rem /= a.spc;
    const int k = rem % a.K;
    rem /= a.K;
    const int g = rem % total_seg;
    const int tile = rem / total_seg;
    const int lane = int(threadIdx.x) & 63, wave = int(threadIdx.x) >> 6;
    const int bi = a.blocks.block_of_segment(g);
    const BlockDesc d = a.blocks.get(bi);
    // a tracking task searches its own tag only (launched with one tile)
    const int tag0 = d.tag >= 0 ? d.tag : tile * a.tile;
    const int ntag = d.tag >= 0 ? 1 : min(a.tile, a.T - tag0);
    const int j = a.blocks.segment(g, d);
    unsigned long long* keys = a.keys + size_t(bi) * a.T;
    const float pth = a.pthr[bi];

    const __amdgpu_buffer_rsrc_t b1 = make_rsrc(a.b1tab, E::B1_TABLE * 8);
    constexpr int NB = bank_stride(N);
    const __amdgpu_buffer_rsrc_t bank =
        make_rsrc(static_cast<const char*>(a.bank) + size_t(tag0) * NB * St::BYTES, uint32_t(ntag) * NB * St::BYTES);
    // stored spectra carry 2^-x_exp (segments) and 2^bank_exp (bank): undo both in G
    float gscale = 1.0f;
    if constexpr (PREC != ACQ_FP32) gscale = ldexpf(1.0f, a.exps[bi] - a.bank_exp);

    // tag-independent first step of the inverse transform
    float2 G[16];
    first_step<E, PREC>(a, eng, g, k, rho, gscale, G);

    // valid outputs: segment lag spc*u + rho < min(V, lags - jV)  <=>  u < ulim
    const int64_t seg0 = int64_t(j) * a.V;
    const int64_t vlim64 = d.lags - seg0 < a.V ? d.lags - seg0 : a.V;
    const int vlim = int(vlim64);
    const int ulim = vlim > rho ? (vlim - rho + a.spc - 1) / a.spc : 0;
    // key index tau*K + k = kbase + u*kstep (fits in 32 bits for valid lags)
    const unsigned kbase = unsigned((seg0 + rho) * a.K + k);
    const unsigned kstep = unsigned(a.spc * a.K);
    const int ob0 = eng.out_base();
    const unsigned idx00 = kbase + unsigned(ob0) * kstep;
    const int omin = eng.out_min(), omax = eng.out_max();   // wave-uniform
    const bool hi = omin + E::HI_OFF < ulim;               // any output of the upper half needed

    // bank element of register m: i = in_index(0) + m*NT, stored for i <= N/2;
    // registers m >= 8 read the mirror N - i = (NT - in_index(0)) + (15-m)*NT
    const int voff = eng.in_index(0) * St::BYTES;
    const int voffm = (E::NT - eng.in_index(0)) * St::BYTES;

    for (int tt = 0; tt < ntag; ++tt) {
        float2 v[16];
#pragma unroll
        for (int m = 0; m < 8; ++m) v[m] = cmul(G[m], St::bload(bank, voff, (tt * NB + m * E::NT) * St::BYTES));
#pragma unroll
        for (int m = 8; m < 16; ++m)
            v[m] = cmulc(G[m], St::bload(bank, voffm, (tt * NB + (15 - m) * E::NT) * St::BYTES));
        eng.template transform<+1>(v, lds, b1, extra, hi);
        // per-register indices and masks are the same for every tag: keep the
        // optimiser from holding all of them across the loop (recomputing is cheap)
        int ob = ob0;
        unsigned idx0 = idx00;
        asm volatile("" : "+v"(ob), "+v"(idx0));
        // this lane's largest valid power; registers are visited in increasing
        // output index, so the strict comparison keeps the smallest lag of a tie
        float bp = -1.0f;
        int boff = 0;
#pragma unroll
        for (int rr = 0; rr < 16; ++rr) {
            const int r = E::visit(rr);
            const int off = E::out_off(r);
            if (omin + off < ulim) {               // wave-uniform: some lane of this register is valid
                float p = fmaf(v[r].x, v[r].x, v[r].y * v[r].y);
                if constexpr (DUMP) {
                    if (ob + off < ulim) {
                        const int64_t tau = seg0 + int64_t(a.spc) * (ob + off) + rho;
                        a.dump[(size_t(tag0 + tt) * a.K + k) * size_t(d.lags) + size_t(tau)] = p;
                    }
                }
                if (omax + off >= ulim && ob + off >= ulim) p = -1.0f;
                boff = p > bp ? off : boff;
                bp = p > bp ? p : bp;
            }
        }
        const unsigned lc = lane_crossings<E>(v, bp, pth, ob, ulim);
        unsigned cross = 0;
        if (__builtin_amdgcn_ballot_w64(lc != 0)) cross = wave_sum_u32(lc);
        unsigned long long best = bp >= 0.0f
            ? (static_cast<unsigned long long>(__float_as_uint(bp)) << 32) |
                  static_cast<unsigned long long>(~(idx0 + unsigned(boff) * kstep))
            : 0ull;
        best = wave_max(best);
        if (lane == 0) {
            red[tt * NW + wave] = best;
            cred[tt * NW + wave] = cross;
        }
    }
    __syncthreads();
    for (int i = int(threadIdx.x); i < ntag; i += E::NT) {
        unsigned long long m = 0ull;
        unsigned c = 0;
        for (int q = 0; q < NW; ++q) {
            m = red[i * NW + q] > m ? red[i * NW + q] : m;
            c += cred[i * NW + q];
        }
        if (m) atomicMax(&keys[tag0 + i], m);
        if (c) atomicAdd(&a.cross[size_t(bi) * a.T + tag0 + i], c);
    }
    __syncthreads();                             // red[] is rewritten by the next item
}

// One tracking work item: (global segment g, tile of bins, phase rho) for the
// block's own tag, item index wi = (g * bin_tiles + tile) * spc + rho, with
// a.tile bins per tile.  Every bin forms its G_rho and runs one inverse
// transform; each lane keeps its largest key over all the item's bins, so one
// wave reduction and one atomic per item remain.
template <class E, int PREC>
__device__ __forceinline__ void track_item(const CorrArgs& a, const E& eng, int wi, float2* lds,
                                           const float2* extra, unsigned long long* red, unsigned* cred) {
    using St = dev::Storage<PREC>;
    constexpr int NW = E::NT / 64;
    const int ntl = (a.K + a.tile - 1) / a.tile;
    int rem = wi;
    const int rho = rem % a.spc;
    rem /= a.spc;
    const int btile = rem % ntl;
    const int g = rem / ntl;
    const int k0 = btile * a.tile, k1 = min(a.K, k0 + a.tile);
    const int lane = int(threadIdx.x) & 63, wave = int(threadIdx.x) >> 6;
    const int bi = a.blocks.block_of_segment(g);
    const BlockDesc d = a.blocks.get(bi);
    const int j = a.blocks.segment(g, d);
    const int tag = d.tag;
    const float pth = a.pthr[bi];

    const __amdgpu_buffer_rsrc_t b1 = make_rsrc(a.b1tab, E::B1_TABLE * 8);
    constexpr int NB = bank_stride(E::N);
    const __amdgpu_buffer_rsrc_t bank =
        make_rsrc(static_cast<const char*>(a.bank) + size_t(tag) * NB * St::BYTES, uint32_t(NB) * St::BYTES);
    float gscale = 1.0f;
    if constexpr (PREC != ACQ_FP32) gscale = ldexpf(1.0f, a.exps[bi] - a.bank_exp);

    const int64_t seg0 = int64_t(j) * a.V;
    const int64_t vlim64 = d.lags - seg0 < a.V ? d.lags - seg0 : a.V;
    const int vlim = int(vlim64);
    const int ulim = vlim > rho ? (vlim - rho + a.spc - 1) / a.spc : 0;
    const unsigned kstep = unsigned(a.spc * a.K);
    const int ob0 = eng.out_base();
    const int omin = eng.out_min(), omax = eng.out_max();
    const bool hi = omin + E::HI_OFF < ulim;
    const int voff = eng.in_index(0) * St::BYTES;              // half bank, as in correlate_item
    const int voffm = (E::NT - eng.in_index(0)) * St::BYTES;

    unsigned long long best = 0ull;
    unsigned lc = 0;                               // this lane's crossings over the item's bins
    // the task's replica spectrum is the same for every bin: read it once
    float2 bk[16];
#pragma unroll
    for (int m = 0; m < 8; ++m) bk[m] = St::bload(bank, voff, (m * E::NT) * St::BYTES);
#pragma unroll
    for (int m = 8; m < 16; ++m) bk[m] = St::bload(bank, voffm, ((15 - m) * E::NT) * St::BYTES);
    for (int k = k0; k < k1; ++k) {
        float2 v[16];
        first_step<E, PREC>(a, eng, g, k, rho, gscale, v);
#pragma unroll
        for (int m = 0; m < 8; ++m) v[m] = cmul(v[m], bk[m]);
#pragma unroll
        for (int m = 8; m < 16; ++m) v[m] = cmulc(v[m], bk[m]);
        eng.template transform<+1>(v, lds, b1, extra, hi);
        int ob = ob0;
        unsigned idx0 = unsigned((seg0 + rho) * a.K + k) + unsigned(ob0) * kstep;
        asm volatile("" : "+v"(ob), "+v"(idx0));
        float bp = -1.0f;
        int boff = 0;
#pragma unroll
        for (int rr = 0; rr < 16; ++rr) {
            const int r = E::visit(rr);
            const int off = E::out_off(r);
            if (omin + off < ulim) {
                float p = fmaf(v[r].x, v[r].x, v[r].y * v[r].y);
                if (omax + off >= ulim && ob + off >= ulim) p = -1.0f;
                lc += p >= pth ? 1u : 0u;
                boff = p > bp ? off : boff;
                bp = p > bp ? p : bp;
            }
        }
        const unsigned long long key = bp >= 0.0f
            ? (static_cast<unsigned long long>(__float_as_uint(bp)) << 32) |
                  static_cast<unsigned long long>(~(idx0 + unsigned(boff) * kstep))
            : 0ull;
        best = key > best ? key : best;
    }
    best = wave_max(best);
    unsigned cross = 0;
    if (__builtin_amdgcn_ballot_w64(lc != 0)) cross = wave_sum_u32(lc);
    if (lane == 0) {
        red[wave] = best;
        cred[wave] = cross;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        unsigned long long m = 0ull;
        unsigned c = 0;
        for (int q = 0; q < NW; ++q) {
            m = red[q] > m ? red[q] : m;
            c += cred[q];
        }
        if (m) atomicMax(&a.keys[size_t(bi) * a.T + tag], m);
        if (c) atomicAdd(&a.cross[size_t(bi) * a.T + tag], c);
    }
    __syncthreads();
}

// Launch forms of the correlation kernel.  Each is its own instantiation so the
// persistent loop's live state does not weigh on the one-item-per-workgroup forms.
enum CorrMode { kCorrGrid = 0, kCorrGridDump = 1, kCorrPersistent = 2, kCorrTrack = 3 };

template <class E, int PREC, int MODE>
__global__ __launch_bounds__(E::NT) void k_correlate(CorrArgs a) {
    constexpr int NW = E::NT / 64;
    constexpr bool DUMP = MODE == kCorrGridDump;
    __shared__ float2 lds[E::LDS];
    __shared__ float2 extra[E::EXTRA];
    __shared__ unsigned long long red[kMaxTagTile * NW];
    __shared__ unsigned cred[kMaxTagTile * NW];
    __shared__ int s_item;
    const int total_seg = a.blocks.total_seg();
    const int total = MODE == kCorrTrack ? total_seg * ((a.K + a.tile - 1) / a.tile) * a.spc
                                         : a.ntiles * total_seg * a.K * a.spc;
    // Workgroups are dealt round-robin to the XCDs; each XCD takes a contiguous
    // range of work items, so items sharing a segment and a tag tile share its L2.
    const int xcd = int(blockIdx.x) % kXcds;
    E eng;
    if constexpr (MODE == kCorrPersistent) {
        eng.init(a.rootsSub, extra);
        const int chunk = (total + kXcds - 1) / kXcds;
        const int begin = xcd * chunk;
        const int end = min(total, begin + chunk);
        for (;;) {
            if (threadIdx.x == 0) s_item = atomicAdd(&a.counters[xcd], 1);
            __syncthreads();
            // uniform by construction; saying so keeps every address derived from
            // the item (bank rows, segment) scalar, with no per-lane resource loops
            const int it = begin + __builtin_amdgcn_readfirstlane(s_item);
            __syncthreads();
            if (it >= end) break;
            correlate_item<E, PREC, false>(a, eng, it, total_seg, lds, extra, red, cred);
        }
    } else {
        // one item per workgroup; the grid may exceed the work (a batch captured
        // for its capacity): the first ceil(total/8) workgroups of each XCD take
        // its contiguous range, the rest exit
        const int per = (total + kXcds - 1) / kXcds;
        const int q = int(blockIdx.x) / kXcds;
        const int wi = xcd * per + q;
        if (q >= per || wi >= total) return;
        eng.init(a.rootsSub, extra);
        if constexpr (MODE == kCorrTrack)
            track_item<E, PREC>(a, eng, wi, lds, extra, red, cred);
        else
            correlate_item<E, PREC, DUMP>(a, eng, wi, total_seg, lds, extra, red, cred);
    }
}

}  // namespace

// ------------------------------------------------------------------ launcher
template <class E, int PREC>
static void corr_ep(const CorrArgs& a, int grid, hipStream_t st) {
    if (a.track)
        hipLaunchKernelGGL((k_correlate<E, PREC, kCorrTrack>), dim3(grid), dim3(E::NT), 0, st, a);
    else if (a.persistent)
        hipLaunchKernelGGL((k_correlate<E, PREC, kCorrPersistent>), dim3(grid), dim3(E::NT), 0, st, a);
    else if (a.dump)
        hipLaunchKernelGGL((k_correlate<E, PREC, kCorrGridDump>), dim3(grid), dim3(E::NT), 0, st, a);
    else
        hipLaunchKernelGGL((k_correlate<E, PREC, kCorrGrid>), dim3(grid), dim3(E::NT), 0, st, a);
}

template <class E>
static hipError_t corr_e(const CorrArgs& a, int grid, int prec, hipStream_t st) {
    switch (prec) {
        case ACQ_FP32: corr_ep<E, ACQ_FP32>(a, grid, st); break;
        case ACQ_FP16: corr_ep<E, ACQ_FP16>(a, grid, st); break;
        case ACQ_BF16: corr_ep<E, ACQ_BF16>(a, grid, st); break;
        default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

hipError_t launch_correlate(const CorrArgs& a, int grid, int log2_sub, int prec, int engine, hipStream_t st) {
    if (grid <= 0) return hipSuccess;
    if ((1 << log2_sub) != a.Msub || a.tile < 1 || a.tile > kMaxTagTile || grid % kXcds) return hipErrorInvalidValue;
    if (a.track && (a.persistent || a.dump)) return hipErrorInvalidValue;
    switch (log2_sub) {
        case 10: return corr_e<StockhamEngine<10>>(a, grid, prec, st);
        case 11: return corr_e<StockhamEngine<11>>(a, grid, prec, st);
        case 12: return corr_e<StockhamEngine<12>>(a, grid, prec, st);
        case 13: return corr_e<StockhamEngine<13>>(a, grid, prec, st);
        case 14:
            return engine == 1 ? corr_e<StockhamEngine<14>>(a, grid, prec, st) : corr_e<Fft14>(a, grid, prec, st);
        default: return hipErrorInvalidValue;
    }
}

}  // namespace acq
