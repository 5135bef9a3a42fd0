// Kernel launch interface used by the plan code.
#pragma once

#include <hip/hip_runtime.h>
#include <cstdint>

#include "acq.h"

namespace acq {

// Workgroups of the block-power partial sums.
constexpr int kPowerParts = 256;

struct CorrArgs {
    const void* X;              // [S][M] forward spectra of the segments (storage format)
    const void* bank;           // [T][Msub] 2^bank_exp conj(DFT_Msub(chips)) / M (storage format)
    const double* parts;        // [kPowerParts] partial sums of |x|^2 (16-bit storage scale)
    const float2* rect;         // [M] sum_{r<spc} exp(+j 2 pi i r / M)
    const float2* rootsM;       // [M] exp(+j 2 pi m / M)
    const float2* rootsSub;     // [Msub] exp(+j 2 pi m / Msub)
    const float2* b1tab;        // 2^14-point engine twiddle table (else unused)
    const int32_t* rot;         // [K] rotation of bin k, in [0, M)
    unsigned long long* keys;   // [T] packed (power bits, ~(lag*K + k)), max-reduced
    float* dump;                // optional [T][K][lags] power
    int64_t n;                  // block length N
    int64_t lags;               // N - L + 1
    int64_t V;                  // valid lags per segment
    int32_t S, K, spc, M, Msub, T, tile, ntiles, nwork, bank_exp;
};

struct FwdArgs {
    const float2* x;            // [N] block
    float2* X;                  // [S][M] FP32 spectra (accumulator)
    void* Xh;                   // [S][M] 16-bit copy (FP16/BF16 plans only)
    const double* parts;        // [kPowerParts] partial sums of |x|^2
    const float2* rootsM;
    const float2* rootsSub;
    const float2* b1tab;
    int64_t n, V;
    int32_t S, spc, M, Msub;
};

struct RefineArgs {
    const float2* x;
    const int8_t* chips;        // [T][C]
    const int64_t* rot_signed;  // [K] signed rotation at M
    const double* freqs;        // [K]
    const unsigned long long* keys;
    const double* parts;        // [kPowerParts] partial sums of |x|^2
    acq_detection* dets;        // [T]
    int32_t* found;             // [T] 1 if detected
    int64_t n, L, lags;
    double theta;
    int32_t T, C, K, spc, M, radius;
};

hipError_t launch_block_power(const float2* x, int64_t n, double* parts, hipStream_t st);
hipError_t launch_fill_u64(unsigned long long* p, int64_t count, hipStream_t st);
hipError_t launch_forward(const FwdArgs& a, int log2_sub, int prec, hipStream_t st);
hipError_t launch_bank(const int8_t* chips, int T, int C, void* bank, const float2* rootsSub,
                       const float2* b1tab, int Msub, int M, int bank_exp, int log2_sub, int prec,
                       hipStream_t st);
hipError_t launch_correlate(const CorrArgs& a, int log2_sub, int prec, hipStream_t st);
hipError_t launch_refine(const RefineArgs& a, hipStream_t st);
hipError_t launch_compact(const acq_detection* dets, const int32_t* found, int T,
                          acq_detection* out, int32_t* count, hipStream_t st);

}  // namespace acq
