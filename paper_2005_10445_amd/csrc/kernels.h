// Kernel launch interface used by the plan code.
#pragma once

#include <hip/hip_runtime.h>
#include <cstdint>

#include "acq.h"

namespace acq {

// Workgroups of the block-power partial sums, per block.
constexpr int kPowerParts = 256;

// The replica bank keeps half of each tag's Msub-point spectrum: the chip code
// is real, so Chat[Msub - i] = conj(Chat[i]) and entries 0 .. Msub/2 suffice.
// Per-tag stride in elements (padded).
__host__ __device__ constexpr int bank_stride(int msub) { return msub / 2 + 64; }
// Persistent correlation launch: work-item counters, one per XCD.
constexpr int kXcds = 8;

// One block of a launch.
struct BlockDesc {
    const float2* x;            // device, n complex64 samples
    int64_t n;
    int64_t lags;               // n - L + 1 (<= 0: nothing to search)
    int32_t seg0;               // first global segment index
    int32_t nseg;               // overlap-save segments of this block
    double theta;               // detection threshold for this block
    int32_t tag;                // -1: search every tag; >= 0: a tracking task for this one tag
    int32_t reserved;
};

// The blocks of one launch: a single inline descriptor (single-block calls), or
// a device array of descriptors whose count and total segment count are read
// on the device, so one captured graph serves any batch within capacity.
struct BlockTable {
    const BlockDesc* descs;     // device [nblocks] or nullptr (use `one`)
    const int32_t* counts;      // device [2] = {nblocks, total segments} when descs != nullptr
    const int32_t* seg_of;      // device [total segments]: segment of the block searched in global slot g
                                // (a subset of the block's segments), or nullptr: slot g is segment g - seg0
    BlockDesc one;

    __device__ __forceinline__ int nblocks() const { return descs ? counts[0] : 1; }
    __device__ __forceinline__ int total_seg() const { return descs ? counts[1] : one.nseg; }
    __device__ __forceinline__ BlockDesc get(int b) const { return descs ? descs[b] : one; }
    // overlap-save segment (within its block d) held in global slot g
    __device__ __forceinline__ int segment(int g, const BlockDesc& d) const { return seg_of ? seg_of[g] : g - d.seg0; }
    // block holding global segment g (segments are numbered block by block)
    __device__ __forceinline__ int block_of_segment(int g) const {
        if (!descs) return 0;
        int lo = 0, hi = counts[0] - 1;
        while (lo < hi) {
            const int mid = (lo + hi + 1) >> 1;
            if (descs[mid].seg0 <= g) lo = mid; else hi = mid - 1;
        }
        return lo;
    }
};

struct CorrArgs {
    BlockTable blocks;
    const void* X;              // [segments][ncls][xstride] padded spectra (storage format): slot
                                // position xpad + i holds X[i mod M] for -xpad <= i < M + xpad
    const void* bank;           // [T][Msub] 2^bank_exp conj(DFT_Msub(chips)) / M (storage format)
    const int* exps;            // [block] 16-bit storage prescale exponents (16-bit plans)
    const float2* wts;          // [spc][M] W_rho[i] = sum_{r<spc} exp(+j 2 pi i (r + rho) / M)
                                // (read for spc != 2; spc = 2 forms them in closed form)
    const float2* rootsM;       // [M] exp(+j 2 pi m / M)
    const float2* rootsSub;     // [Msub] exp(+j 2 pi m / Msub)
    const float2* b1tab;        // 2^14-point engine twiddle table (else unused)
    const int32_t* rot;         // [K] rotation of bin k, in [0, M)
    const int32_t* cls;         // [K] residual class of bin k (spectra slot g * ncls + cls[k])
    unsigned long long* keys;   // [block][T] packed (power bits, ~(lag*K + k)), max-reduced
    const float* pthr;          // [block] power threshold theta * L * Pxhat (+inf: none)
    unsigned* cross;            // [block][T] count of (bin, lag) with P >= pthr, added to
    float* dump;                // optional [T][K][lags] power (single-block calls)
    int* counters;              // [kXcds] work-item counters (persistent launches)
    int64_t V;                  // valid lags per segment
    int64_t xstride;            // elements per spectra slot
    int32_t xpad;               // wrap-around copies before and after each spectrum
    int32_t K, spc, M, Msub, T, tile, ntiles, bank_exp, ncls;
    int32_t persistent;         // 1: loop over work items from the counters
    int32_t track;              // 1: tracking tasks; `tile` then counts bins per work item
};

struct FwdArgs {
    BlockTable blocks;
    float2* X;                  // [segments][ncls][xstride] FP32 spectra (sub-transforms, then the
                                // result), at offset xpad of each slot with wrap-around copies
    void* Xh;                   // [segments][ncls][xstride] 16-bit copy (FP16/BF16 plans only)
    const int* exps;            // [block] 16-bit storage prescale exponents (16-bit plans)
    const float2* rootsM;
    const float2* rootsSub;
    const float2* b1tab;
    const double* cls_cyc;      // [ncls] residual offset of each class, cycles per sample
    int64_t V;
    int64_t xstride;            // elements per slot (M when unpadded)
    int32_t xpad;               // wrap-around copies before and after each spectrum (0: none)
    int32_t spc, M, Msub, ncls;
};

struct RefineArgs {
    BlockTable blocks;
    const int8_t* chips;        // [T][C]
    const int64_t* rot_signed;  // [K] signed rotation at M
    const double* freqs;        // [K]
    const double2* roots64;     // [M] (cos, sin)(2 pi m / M), FP64
    const double* cyc;          // [K] f_k / Fs (exact bins)
    const unsigned long long* keys;   // [block][T]
    const double* parts;        // [block][kPowerParts]
    const int32_t* bad;         // [block] 1: the block holds a non-finite sample
    const unsigned* cross;      // [block][T] threshold crossings of the correlation pass
    acq_detection* dets;        // [block][T]
    int32_t* found;             // [block][T] 1 if detected
    int64_t L;
    int32_t T, C, K, spc, log2_spc, M, radius, exact;
    int32_t track;              // 1: one candidate per block, the block's own tag
    int32_t check_finite;       // 1: no detection in a block with a non-finite sample
    double* partial;            // [items][kRefineParts][3 * window] FP64 partial sums
    int64_t* center;            // [items] window centre of the second round (-1: none)
};

// Refinement work: items = blocks * (tracking ? 1 : T); each item's sums run in
// kRefineParts workgroups, each writing 3 * WMAX doubles (WMAX = 5 for radius
// <= 1, else 2 * kMaxRefineRadius + 3).
constexpr int kRefineParts = 16;

// partial sums of |x|^2 of every block (blocks of at most max_len samples)
hipError_t launch_block_power(const BlockTable& bt, int max_blocks, int64_t max_len, double* parts, hipStream_t st);
// Per-block quantities derived from the block power, for every block of the
// table: exps[b] = round(log2(sqrt(M * Pxhat_b))) (the 16-bit storage
// prescale), pthr[b] = theta_b * L * Pxhat_b (+inf when Pxhat_b is 0 or not
// finite), bad[b] = 1 when Pxhat_b is not finite (some sample is NaN or
// infinite); nbad[0] receives the number of such blocks (workgroup 0).  The
// same launch also clears the search's per-(block, tag) peak keys and
// crossing counts, nclear of each (two launches fewer per search).
hipError_t launch_block_stats(const BlockTable& bt, const double* parts, int M, int64_t L, int* exps, float* pthr,
                              int32_t* bad, int32_t* nbad, unsigned long long* keys, unsigned* cross,
                              int64_t nclear, hipStream_t st);
hipError_t launch_fill_u64(unsigned long long* p, int64_t count, hipStream_t st);
hipError_t launch_fill_i32(int* p, int64_t count, hipStream_t st);
// grid: workgroups of the sub-transforms (items = segments * spc); combine_slots:
// segment slots the combine step covers (>= the segments in use)
hipError_t launch_forward(const FwdArgs& a, int grid, int combine_slots, int log2_sub, int prec, hipStream_t st);
hipError_t launch_bank(const int8_t* chips, int T, int C, void* bank, const float2* rootsSub,
                       const float2* b1tab, int Msub, int M, int bank_exp, int log2_sub, int prec,
                       hipStream_t st);
// engine: 0 = the library's choice for the size, 1 = Stockham passes (any size)
hipError_t launch_correlate(const CorrArgs& a, int grid, int log2_sub, int prec, int engine, hipStream_t st);
hipError_t launch_refine(const RefineArgs& a, int max_blocks, hipStream_t st);
// track: one candidate per block (its tag), else T per block
// capacity: records written to out (the rest are counted only)
hipError_t launch_compact(const BlockTable& bt, const acq_detection* dets, const int32_t* found, int T, int track,
                          acq_detection* out, int32_t capacity, int32_t* count, hipStream_t st);

}  // namespace acq
