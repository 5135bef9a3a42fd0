// Host-side logic shared by the plan code: configuration checks, overlap-save
// geometry, snapped carrier-offset grid, transform tables, error reporting.
// Nothing here touches the GPU.
#pragma once

#include <cstdint>
#include <string>
#include <vector>

#include "acq.h"

namespace acq {

// Smallest and largest per-tag inverse transform handled on one compute unit.
constexpr int kMinSubLog2 = 10;   // 1024 points, 64 threads x 16
constexpr int kMaxSubLog2 = 14;   // 16384 points = 128 KiB of complex64 in LDS
constexpr int kMaxRefineRadius = 8;
constexpr int kMaxTagTile = 64;

struct Geometry {
    int64_t L = 0;          // template length C * spc
    int64_t m_min = 0;      // 2^ceil(log2(L + 1))
    int64_t M = 0;          // overlap-save segment length
    int64_t Msub = 0;       // M / spc
    int     log2_sub = 0;   // log2(Msub)
    int64_t V = 0;          // M - L + 1
    int64_t max_segments = 0;
    double  q = 0;          // Fs / m_min
    int64_t centre_q = 0;   // snapped centre in quanta
    int64_t step_q = 0;     // snapped step in quanta
    int     tag_tile = 0;
    int     max_blocks = 1;         // blocks per batch call
    int64_t max_batch_samples = 0;  // samples per batch call
    int64_t max_total_segments = 0; // segment spectra allocated
    std::vector<double>  freqs_hz;   // K bin frequencies (snapped unless exact)
    std::vector<int32_t> rot;        // per-bin rotation of the M-point spectrum, in [0, M)
    std::vector<int64_t> rot_signed; // per-bin signed rotation at M
    // Segment spectra are stored padded: a slot of xstride elements holds
    // X[(i - xpad) mod M] at position i, i < M + 2 xpad, so that the rotated
    // read X[(i + r) mod M] of any bin (|r| <= xpad, r the rotation reduced to
    // (-M/2, M/2]) is position xpad + i + r, with no wrap-around.
    int64_t xpad = 0;
    int64_t xstride = 0;             // M + 2 xpad rounded up to 64 elements
    bool exact = false;              // ACQ_FLAG_EXACT_BINS
    int ncls = 1;                    // distinct residual offsets (sets of segment spectra)
    std::vector<int32_t> cls;        // per-bin residual class
    std::vector<double>  cls_cyc;    // per-class residual offset, cycles per sample
    std::vector<double>  cyc;        // per-bin f_k / Fs
    int64_t device_bytes = 0;
};

// Thread-local last-error message.
void set_error(const std::string& msg);
void clear_error();
const char* last_error();
int fail(int status, const std::string& msg);

// Validate `cfg` and fill `g`.  Returns ACQ_OK or a negative acq_status (with message).
int derive_geometry(const acq_config* cfg, Geometry* g);

// Default detection threshold for a block of n samples: ln(T K (n-L+1) / 1e-3).
double default_threshold(int64_t num_tags, int64_t num_bins, int64_t n, int64_t L);

// exp(+j 2 pi m / n) for m in [0, n), computed in FP64 with exact quadrant
// symmetry and rounded to FP32; interleaved (re, im).
std::vector<float> unit_roots(int64_t n);
// The same roots in FP64: [2n] = (cos, sin)(2 pi m / n).
std::vector<double> unit_roots64(int64_t n);

// Twiddles of the 2^14-point workgroup transform, laid out [w][k2a][l] with
// entry exp(+j 2 pi l (w + 16 k2a) / 2^14), w, k2a < 16, l < 64.
std::vector<float> fft14_b1_table();

// Weights of the tag-independent first step of the split inverse transform:
// W_rho[i] = conj(Rect[i]) exp(+j 2 pi i rho / M) = sum_{r<spc} exp(+j 2 pi i (r + rho) / M)
// for rho in [0, spc), i in [0, M), with Rect the M-point spectrum of a run of
// spc ones.  Layout [rho][i], interleaved FP32 rounded once from FP64.
std::vector<float> phase_weights(int64_t M, int spc);

}  // namespace acq
