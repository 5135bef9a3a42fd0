// Host-side checks and derived quantities of an acquisition plan (no GPU calls).
#include "host_logic.h"

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <limits>

namespace acq {

namespace {
thread_local std::string g_last_error;

bool is_pow2(int64_t v) { return v > 0 && (v & (v - 1)) == 0; }

int ilog2(int64_t v) {
    int r = 0;
    while ((int64_t(1) << r) < v) ++r;
    return r;
}

// Cost model used to choose M when the caller leaves it open: inverse transform
// points processed for a block of n samples, weighted by the transform depth.
double transform_cost(int64_t n, int64_t L, int64_t M, int spc) {
    const int64_t lags = n - L + 1;
    if (lags <= 0) return 0.0;
    const int64_t V = M - L + 1;
    const int64_t S = (lags + V - 1) / V;
    const double msub = double(M / spc);
    return double(S) * spc * msub * std::log2(msub);
}
}  // namespace

void set_error(const std::string& msg) { g_last_error = msg; }
void clear_error() { g_last_error.clear(); }
const char* last_error() { return g_last_error.c_str(); }
int fail(int status, const std::string& msg) {
    set_error(msg);
    return status;
}

double default_threshold(int64_t num_tags, int64_t num_bins, int64_t n, int64_t L) {
    int64_t lags = n - L + 1;
    if (lags < 1) lags = 1;
    return std::log(double(num_tags) * double(num_bins) * double(lags) / 1e-3);
}

int derive_geometry(const acq_config* cfg, Geometry* g) {
    if (!cfg || !g) return fail(ACQ_ERR_INVALID_ARG, "null config or output");
    if (!(cfg->sample_rate_hz > 0.0) || !std::isfinite(cfg->sample_rate_hz))
        return fail(ACQ_ERR_INVALID_ARG, "sample_rate_hz must be positive and finite");
    if (cfg->num_tags < 1) return fail(ACQ_ERR_INVALID_ARG, "num_tags must be >= 1");
    if (cfg->num_chips < 1) return fail(ACQ_ERR_INVALID_ARG, "num_chips must be >= 1");
    const int spc = cfg->samples_per_chip;
    if (!(spc == 1 || spc == 2 || spc == 4 || spc == 8))
        return fail(ACQ_ERR_UNSUPPORTED, "samples_per_chip must be 1, 2, 4 or 8");
    if (cfg->num_bins < 1 || cfg->num_bins % 2 == 0)
        return fail(ACQ_ERR_INVALID_ARG, "num_bins must be odd and >= 1");
    if (!cfg->chips) return fail(ACQ_ERR_INVALID_ARG, "chips is null");
    if (cfg->max_block_len < 1) return fail(ACQ_ERR_INVALID_ARG, "max_block_len must be >= 1");
    if (!std::isfinite(cfg->bin_center_hz) || !std::isfinite(cfg->bin_step_hz) ||
        !std::isfinite(cfg->threshold))
        return fail(ACQ_ERR_INVALID_ARG, "non-finite frequency or threshold");
    if (cfg->num_bins > 1 && !(cfg->bin_step_hz > 0.0))
        return fail(ACQ_ERR_INVALID_ARG, "bin_step_hz must be > 0 when num_bins > 1");
    if (cfg->precision != ACQ_FP32 && cfg->precision != ACQ_FP16 && cfg->precision != ACQ_BF16)
        return fail(ACQ_ERR_INVALID_ARG, "unknown precision");
    if (cfg->refine_radius < 0 || cfg->refine_radius > kMaxRefineRadius)
        return fail(ACQ_ERR_INVALID_ARG, "refine_radius must be in [0, 8]");
    if (cfg->tag_tile < 0) return fail(ACQ_ERR_INVALID_ARG, "tag_tile must be >= 0");
    if ((cfg->flags & ~(ACQ_FLAG_GRAPH | ACQ_FLAG_EXACT_BINS | ACQ_FLAG_ASYNC | ACQ_FLAG_CHECK_FINITE)) != 0)
        return fail(ACQ_ERR_INVALID_ARG, "unknown flags");
    if (cfg->max_batch_blocks < 0 || cfg->max_batch_samples < 0)
        return fail(ACQ_ERR_INVALID_ARG, "negative batch capacity");

    const int64_t T = cfg->num_tags, C = cfg->num_chips, K = cfg->num_bins;
    for (int64_t i = 0; i < T * C; ++i)
        if (cfg->chips[i] != 1 && cfg->chips[i] != -1)
            return fail(ACQ_ERR_INVALID_ARG, "chips must be +1 or -1");

    Geometry G;
    G.L = C * spc;
    G.m_min = int64_t(1) << ilog2(G.L + 1);
    G.q = cfg->sample_rate_hz / double(G.m_min);

    // choose / check the segment length M
    const int64_t m_lo = G.m_min;
    const int64_t m_hi = int64_t(spc) << kMaxSubLog2;
    if (cfg->fft_len != 0) {
        const int64_t M = cfg->fft_len;
        if (!is_pow2(M) || M < m_lo)
            return fail(ACQ_ERR_INVALID_ARG, "fft_len must be a power of two >= 2^ceil(log2(L+1))");
        if (M > m_hi || (M / spc) < (int64_t(1) << kMinSubLog2))
            return fail(ACQ_ERR_UNSUPPORTED, "fft_len / samples_per_chip must be in [2^10, 2^14]");
        G.M = M;
    } else {
        int64_t best = 0;
        double best_cost = std::numeric_limits<double>::infinity();
        for (int64_t M = m_lo; M <= m_hi; M *= 2) {
            if (M / spc < (int64_t(1) << kMinSubLog2)) continue;
            double c = transform_cost(cfg->max_block_len, G.L, M, spc);
            if (c < best_cost * (1.0 - 1e-9)) {
                best_cost = c;
                best = M;
            }
        }
        if (best == 0)
            return fail(ACQ_ERR_UNSUPPORTED, "template too long for the on-chip inverse transform");
        G.M = best;
    }
    G.Msub = G.M / spc;
    G.log2_sub = ilog2(G.Msub);
    G.V = G.M - G.L + 1;
    const int64_t lags_max = cfg->max_block_len - G.L + 1;
    G.max_segments = lags_max > 0 ? (lags_max + G.V - 1) / G.V : 0;
    if (lags_max > 0 && double(lags_max) * double(K) >= 4294967295.0)
        return fail(ACQ_ERR_UNSUPPORTED, "(max_block_len - L + 1) * num_bins must be < 2^32");

    // snapped grid
    G.centre_q = int64_t(std::llround(cfg->bin_center_hz / G.q));
    if (K > 1) {
        int64_t s = int64_t(std::llround(cfg->bin_step_hz / G.q));
        G.step_q = s < 1 ? 1 : s;
    }
    const int64_t half = (K - 1) / 2;
    const int64_t ratio = G.M / G.m_min;
    G.freqs_hz.resize(size_t(K));
    G.rot.resize(size_t(K));
    G.rot_signed.resize(size_t(K));
    G.exact = (cfg->flags & ACQ_FLAG_EXACT_BINS) != 0;
    G.cls.assign(size_t(K), 0);
    G.cyc.resize(size_t(K));
    G.cls_cyc.clear();
    if (!G.exact) G.cls_cyc.push_back(0.0);
    const double qM = cfg->sample_rate_hz / double(G.M);       // rotation quantum at M
    for (int64_t k = 0; k < K; ++k) {
        int64_t m;
        if (G.exact) {
            const double f = cfg->bin_center_hz + double(k - half) * cfg->bin_step_hz;
            G.freqs_hz[size_t(k)] = f;
            m = int64_t(std::llround(f / qM));                  // nearest rotation at M
            const double resid = (f - double(m) * qM) / cfg->sample_rate_hz;   // cycles per sample
            // residual classes: bins whose residuals agree to 1e-12 cycles per sample share spectra
            int c = -1;
            for (size_t j = 0; j < G.cls_cyc.size() && c < 0; ++j)
                if (std::fabs(G.cls_cyc[j] - resid) <= 1e-12) c = int(j);
            if (c < 0) {
                G.cls_cyc.push_back(resid);
                c = int(G.cls_cyc.size()) - 1;
            }
            G.cls[size_t(k)] = c;
        } else {
            const int64_t fq = G.centre_q + (k - half) * G.step_q;   // frequency in quanta
            G.freqs_hz[size_t(k)] = double(fq) * G.q;
            m = fq * ratio;                                          // rotation at M
        }
        G.cyc[size_t(k)] = G.freqs_hz[size_t(k)] / cfg->sample_rate_hz;
        G.rot_signed[size_t(k)] = m;
        int64_t r = m % G.M;
        if (r < 0) r += G.M;
        G.rot[size_t(k)] = int32_t(r);
    }
    G.ncls = int(G.cls_cyc.size());
    G.xpad = 0;
    for (int64_t k = 0; k < K; ++k) {
        const int64_t r = G.rot[size_t(k)];
        const int64_t rs = r <= G.M / 2 ? r : r - G.M;
        G.xpad = std::max<int64_t>(G.xpad, rs < 0 ? -rs : rs);
    }
    G.xstride = (G.M + 2 * G.xpad + 63) / 64 * 64;

    // batch capacity: segments of a batch are bounded by sum(n_b)/V + blocks
    G.max_blocks = cfg->max_batch_blocks > 0 ? cfg->max_batch_blocks : 1;
    G.max_batch_samples = cfg->max_batch_samples > 0 ? cfg->max_batch_samples
                                                     : int64_t(G.max_blocks) * cfg->max_block_len;
    if (G.max_batch_samples < cfg->max_block_len) G.max_batch_samples = cfg->max_block_len;
    G.max_total_segments = G.max_batch_samples / G.V + G.max_blocks;
    if (G.max_total_segments < G.max_segments) G.max_total_segments = G.max_segments;
    if (double(G.max_total_segments) * double(K) * double(spc) * double(T) >= 2147483000.0)
        return fail(ACQ_ERR_UNSUPPORTED, "batch too large for 32-bit work-item indices");

    G.tag_tile = cfg->tag_tile > 0 ? cfg->tag_tile : 16;
    if (G.tag_tile > kMaxTagTile) G.tag_tile = kMaxTagTile;
    if (G.tag_tile > T) G.tag_tile = int(T);

    // device memory: spectra of segments, replica bank, tables, small buffers
    int64_t bytes = 0;
    const int64_t sbytes = cfg->precision == ACQ_FP32 ? 8 : 4;
    bytes += G.max_total_segments * G.ncls * G.xstride * 8;  // forward spectra X[S][classes][xstride] (FP32)
    if (sbytes == 4) bytes += G.max_total_segments * G.ncls * G.xstride * 4;   // their 16-bit copy
    bytes += T * (G.Msub / 2 + 64) * sbytes;  // replica bank [T][M/spc / 2 + 64] (half spectrum)
    bytes += G.M * 8 * (spc + 1) + G.Msub * 8;  // phase weights [spc][M], roots at M and M/spc
    bytes += T * C;                           // chips
    bytes += K * (4 + 8);                     // rotations, frequencies
    bytes += int64_t(G.max_blocks) * (T * (8 + 4 + 2 * int64_t(sizeof(acq_detection))) + 2048 + 64) + 4096;
    const int64_t wmax = cfg->refine_radius <= 1 ? 5 : 2 * kMaxRefineRadius + 3;
    bytes += int64_t(G.max_blocks) * T * (16 * 3 * wmax * 8 + 8);   // refinement partial sums, centres
    G.device_bytes = bytes;
    *g = std::move(G);
    clear_error();
    return ACQ_OK;
}

std::vector<double> unit_roots64(int64_t n) {
    std::vector<double> out(size_t(2 * n));
    const double two_pi = 6.283185307179586476925286766559;
    for (int64_t m = 0; m < n; ++m) {
        // reduce to a quadrant, then to [0, pi/4] by reflection, exactly in integers
        const int64_t q4 = (4 * m) / n;           // quadrant 0..3
        const int64_t r = m - q4 * (n / 4);       // 0 <= r < n/4 (n >= 4)
        double c, s;
        if (2 * r <= n / 4) {
            const double a = two_pi * double(r) / double(n);
            c = std::cos(a);
            s = std::sin(a);
        } else {
            const double a = two_pi * double(n / 4 - r) / double(n);
            c = std::sin(a);
            s = std::cos(a);
        }
        double re = c, im = s;
        for (int64_t k = 0; k < q4; ++k) {       // multiply by j per quadrant
            const double t = re;
            re = -im;
            im = t;
        }
        out[size_t(2 * m)] = re;
        out[size_t(2 * m + 1)] = im;
    }
    return out;
}

std::vector<float> unit_roots(int64_t n) {
    const std::vector<double> r = unit_roots64(n);
    return std::vector<float>(r.begin(), r.end());
}

std::vector<float> fft14_b1_table() {
    const int64_t n = 16384;
    const std::vector<float> roots = unit_roots(n);
    std::vector<float> out(size_t(2 * 16 * 16 * 64));
    size_t o = 0;
    for (int64_t w = 0; w < 16; ++w)
        for (int64_t k2a = 0; k2a < 16; ++k2a)
            for (int64_t l = 0; l < 64; ++l) {
                const int64_t e = (l * (w + 16 * k2a)) % n;
                out[o++] = roots[size_t(2 * e)];
                out[o++] = roots[size_t(2 * e + 1)];
            }
    return out;
}

std::vector<float> phase_weights(int64_t M, int spc) {
    std::vector<float> out(size_t(2 * M * spc));
    const double two_pi = 6.283185307179586476925286766559;
    for (int rho = 0; rho < spc; ++rho)
        for (int64_t i = 0; i < M; ++i) {
            double re = 0.0, im = 0.0;
            for (int r = 0; r < spc; ++r) {
                const int64_t e = (i * (r + rho)) % M;      // exact reduction of the angle
                const double a = two_pi * double(e) / double(M);
                re += std::cos(a);
                im += std::sin(a);
            }
            const size_t o = size_t(2 * (int64_t(rho) * M + i));
            out[o] = float(re);
            out[o + 1] = float(im);
        }
    return out;
}

}  // namespace acq
