// HIP kernels of the acquisition path (gfx950).
//
//   k_block_power  : FP64 partial sums of |x|^2 (mean block power Pxhat)
//   k_forward      : overlap-save segment j, X_j = DFT_M(x[jV .. jV+M)) with a zero
//                    tail, as spc decimated Msub-point transforms combined by one
//                    radix-spc decimation-in-time step
//   k_bank         : replica spectra conj(DFT_Msub(chip code)) / M, plan time
//   k_correlate    : the hot loop, see below
//   k_refine       : FP64 re-correlation around each tag's peak, re-maximisation,
//                    parabolic vertex, z and energy
//   k_compact      : detections in tag order
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
// value.
#include <hip/hip_runtime.h>

#include "device_fft.h"
#include "fft14.h"
#include "storage.h"
#include "host_logic.h"
#include "kernels.h"

namespace acq {

using dev::cadd;
using dev::cmul;
using dev::cmulc;
using dev::Fft;
using dev::dft16;

namespace {

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
    return v;
}

__device__ __forceinline__ unsigned long long wave_max(unsigned long long v) {
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) {
        const unsigned long long o = __shfl_xor(v, off, 64);
        v = o > v ? o : v;
    }
    return v;
}

// ------------------------------------------------------------------ block power
__global__ __launch_bounds__(256) void k_block_power(const float2* __restrict__ x, int64_t n,
                                                     double* __restrict__ parts) {
    const int64_t chunk = (n + kPowerParts - 1) / kPowerParts;
    const int64_t beg = int64_t(blockIdx.x) * chunk;
    const int64_t end = beg + chunk < n ? beg + chunk : n;
    double acc = 0.0;
    for (int64_t i = beg + threadIdx.x; i < end; i += 256) {
        const float2 v = x[i];
        acc += double(v.x) * double(v.x) + double(v.y) * double(v.y);
    }
    acc = wave_sum(acc);
    __shared__ double red[4];
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = acc;
    __syncthreads();
    if (threadIdx.x == 0) parts[blockIdx.x] = (red[0] + red[1]) + (red[2] + red[3]);
}

__global__ void k_fill_u64(unsigned long long* p, int64_t count) {
    const int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (i < count) p[i] = 0ull;
}

// ------------------------------------------------------------------ transform engines
// Both engines take v[m] = a[in_index(m)] and leave output index
// out_base() + out_off(r) in v[r].

// Stockham passes (2^10 .. 2^13 points), see device_fft.h.
template <int LOGN_>
struct StockhamEngine {
    using F = Fft<LOGN_>;
    static constexpr int LOGN = LOGN_;
    static constexpr int N = F::N;
    static constexpr int NT = F::NT;
    static constexpr int LDS = F::LDS;
    static constexpr int EXTRA = 1;
    static constexpr int B1_TABLE = 1;
    int t;
    const float2* roots;
    __device__ __forceinline__ void init(const float2* __restrict__ r, float2*) {
        t = int(threadIdx.x);
        roots = r;
    }
    __device__ __forceinline__ int in_index(int m) const { return t + m * NT; }
    __device__ __forceinline__ int out_base() const { return t; }
    // smallest / largest out_base() over the wave (wave-uniform)
    __device__ __forceinline__ int out_min() const { return __builtin_amdgcn_readfirstlane(t & ~63); }
    __device__ __forceinline__ int out_max() const { return out_min() + 63; }
    static constexpr int out_off(int r) { return r * NT; }
    static constexpr int HI_OFF = 1 << 30;      // no output is ever pruned
    template <int S>
    __device__ __forceinline__ void transform(float2 (&v)[16], float2* lds, __amdgpu_buffer_rsrc_t,
                                              const float2*, bool = true) const {
        int tq = t;
        asm volatile("" : "+v"(tq));            // recompute addressing per call, no hoisting
        F::template transform<S>(v, lds, roots, tq);
    }
};

using dev::bload;
using dev::Fft14;
using dev::make_rsrc;

// ------------------------------------------------------------------ forward spectra
// Power-of-two prescale of the stored segment spectra for 16-bit storage:
// 2^-e with e = round(log2(sqrt(M * Pxhat))), so typical |X| is near 1.
__device__ __forceinline__ int spectrum_exponent(const double* __restrict__ parts, int64_t n, int M) {
    __shared__ int s_e;
    if (threadIdx.x == 0) {
        double s = 0.0;
        for (int i = 0; i < kPowerParts; ++i) s += parts[i];
        const double px = s / double(n);
        s_e = px > 0.0 ? int(rint(0.5 * log2(double(M) * px))) : 0;
    }
    __syncthreads();
    return s_e;
}

template <class E, int PREC>
__global__ __launch_bounds__(E::NT) void k_forward(FwdArgs a) {
    using St = dev::Storage<PREC>;
    __shared__ float2 lds[E::LDS];
    __shared__ float2 extra[E::EXTRA];
    E eng;
    eng.init(a.rootsSub, extra);
    const __amdgpu_buffer_rsrc_t b1 = make_rsrc(a.b1tab, E::B1_TABLE * 8);
    const int j = blockIdx.x;
    const int64_t base = int64_t(j) * a.V;
    float2* Xj = a.X + size_t(j) * size_t(a.M);
    const int mmask = a.M - 1;
    float xs = 1.0f;
    if constexpr (PREC != ACQ_FP32) xs = ldexpf(1.0f, -spectrum_exponent(a.parts, a.n, a.M));
    for (int r = 0; r < a.spc; ++r) {
        float2 v[16];
#pragma unroll
        for (int m = 0; m < 16; ++m) {
            const int64_t idx = base + int64_t(a.spc) * eng.in_index(m) + r;
            v[m] = idx < a.n ? a.x[idx] : make_float2(0.f, 0.f);
        }
        eng.template transform<-1>(v, lds, b1, extra);
        // X[i] += exp(-j 2 pi i r / M) F_r[i mod Msub], accumulated in FP32
        const int ob = eng.out_base();
        const bool last = r == a.spc - 1;
#pragma unroll
        for (int m = 0; m < 16; ++m) {
            const int ip = ob + E::out_off(m);
            for (int q = 0; q < a.spc; ++q) {
                const int i = ip + q * a.Msub;
                float2 c = v[m];
                if (r) c = cmulc(c, a.rootsM[(int)((int64_t(i) * r) & mmask)]);
                if (r) c = cadd(Xj[i], c);
                if constexpr (PREC == ACQ_FP32) {
                    Xj[i] = c;
                } else {
                    if (last)
                        reinterpret_cast<typename St::T*>(a.Xh)[size_t(j) * size_t(a.M) + i] =
                            St::pack(make_float2(c.x * xs, c.y * xs));
                    else
                        Xj[i] = c;
                }
            }
        }
        __syncthreads();
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
    typename St::T* out = reinterpret_cast<typename St::T*>(bank) + size_t(tag) * E::N;
#pragma unroll
    for (int m = 0; m < 16; ++m) out[ob + E::out_off(m)] = St::pack(make_float2(v[m].x * s, -v[m].y * s));
}

// ------------------------------------------------------------------ correlation
template <class E, int PREC, bool DUMP>
__global__ __launch_bounds__(E::NT) void k_correlate(CorrArgs a) {
    using St = dev::Storage<PREC>;
    constexpr int N = E::N;
    constexpr int NW = E::NT / 64;
    __shared__ float2 lds[E::LDS];
    __shared__ float2 extra[E::EXTRA];
    __shared__ unsigned long long red[kMaxTagTile * NW];

    // Workgroups are dealt round-robin to the 8 XCDs; give each XCD a contiguous
    // range of work items so items sharing a segment and a tag tile share its L2.
    const int per = int(gridDim.x) >> 3;
    const int wi = int(blockIdx.x & 7u) * per + int(blockIdx.x >> 3);
    if (wi >= a.nwork) return;
    int rem = wi;
    const int rho = rem % a.spc;
    rem /= a.spc;
    const int k = rem % a.K;
    rem /= a.K;
    const int j = rem % a.S;
    const int tile = rem / a.S;
    const int tag0 = tile * a.tile;
    const int ntag = min(a.tile, a.T - tag0);
    const int lane = int(threadIdx.x) & 63, wave = int(threadIdx.x) >> 6;

    E eng;
    eng.init(a.rootsSub, extra);
    const __amdgpu_buffer_rsrc_t b1 = make_rsrc(a.b1tab, E::B1_TABLE * 8);
    const __amdgpu_buffer_rsrc_t bank =
        make_rsrc(static_cast<const char*>(a.bank) + size_t(tag0) * N * St::BYTES, uint32_t(ntag) * N * St::BYTES);
    // stored spectra carry 2^-x_exp (segments) and 2^bank_exp (bank): undo both in G
    float gscale = 1.0f;
    if constexpr (PREC != ACQ_FP32) gscale = ldexpf(1.0f, spectrum_exponent(a.parts, a.n, a.M) - a.bank_exp);

    // tag-independent first step of the inverse transform
    float2 G[16];
    {
        const typename St::T* Xj = static_cast<const typename St::T*>(a.X) + size_t(j) * size_t(a.M);
        const int rot = a.rot[k];
        const int mmask = a.M - 1;
#pragma unroll
        for (int m = 0; m < 16; ++m) {
            const int ip = eng.in_index(m);
            float2 acc = make_float2(0.f, 0.f);
            for (int q = 0; q < a.spc; ++q) {
                const int i = ip + q * a.Msub;
                float2 xv = cmul(St::unpack(Xj[(i + rot) & mmask]), a.rect[i]);
                const int e = (a.Msub * q * rho) & mmask;
                if (e) xv = cmul(xv, a.rootsM[e]);
                acc = cadd(acc, xv);
            }
            if (rho) acc = cmul(acc, a.rootsM[ip * rho]);
            if constexpr (PREC != ACQ_FP32) acc = make_float2(acc.x * gscale, acc.y * gscale);
            G[m] = acc;
        }
    }

    // valid outputs: segment lag spc*u + rho < min(V, lags - jV)  <=>  u < ulim
    const int64_t seg0 = int64_t(j) * a.V;
    const int64_t vlim64 = a.lags - seg0 < a.V ? a.lags - seg0 : a.V;
    const int vlim = int(vlim64);
    const int ulim = vlim > rho ? (vlim - rho + a.spc - 1) / a.spc : 0;
    // key index tau*K + k = kbase + u*kstep (fits in 32 bits for valid lags)
    const unsigned kbase = unsigned((seg0 + rho) * a.K + k);
    const unsigned kstep = unsigned(a.spc * a.K);
    const int ob = eng.out_base();
    const unsigned idx0 = kbase + unsigned(ob) * kstep;
    const int omin = eng.out_min(), omax = eng.out_max();   // wave-uniform
    const bool hi = omin + E::HI_OFF < ulim;               // any output of the upper half needed

    const int voff = eng.in_index(0) * St::BYTES;   // bank element of register m: in_index(0) + m*NT

    for (int tt = 0; tt < ntag; ++tt) {
        float2 v[16];
#pragma unroll
        for (int m = 0; m < 16; ++m) v[m] = cmul(G[m], St::bload(bank, voff, (tt * N + m * E::NT) * St::BYTES));
        eng.template transform<+1>(v, lds, b1, extra, hi);
        unsigned long long best = 0ull;
#pragma unroll
        for (int r = 0; r < 16; ++r) {
            const int off = E::out_off(r);
            if (omin + off < ulim) {               // wave-uniform: some lane of this register is valid
                const float p = fmaf(v[r].x, v[r].x, v[r].y * v[r].y);
                const unsigned idx = idx0 + unsigned(off) * kstep;
                unsigned long long key = (static_cast<unsigned long long>(__float_as_uint(p)) << 32) |
                                         static_cast<unsigned long long>(~idx);
                if (omax + off >= ulim && ob + off >= ulim) key = 0ull;
                best = key > best ? key : best;
                if constexpr (DUMP) {
                    if (ob + off < ulim) {
                        const int64_t tau = seg0 + int64_t(a.spc) * (ob + off) + rho;
                        a.dump[(size_t(tag0 + tt) * a.K + k) * size_t(a.lags) + size_t(tau)] = p;
                    }
                }
            }
        }
        best = wave_max(best);
        if (lane == 0) red[tt * NW + wave] = best;
    }
    __syncthreads();
    for (int i = int(threadIdx.x); i < ntag; i += E::NT) {
        unsigned long long m = 0ull;
        for (int q = 0; q < NW; ++q) m = red[i * NW + q] > m ? red[i * NW + q] : m;
        if (m) atomicMax(&a.keys[tag0 + i], m);
    }
}

// ------------------------------------------------------------------ refine
constexpr int kMaxWin = 2 * kMaxRefineRadius + 3;

__global__ __launch_bounds__(256) void k_refine(RefineArgs a) {
    const int tag = blockIdx.x;
    const int t = threadIdx.x, lane = t & 63, wave = t >> 6;
    __shared__ double s_px;
    __shared__ double red[4][kMaxWin][3];
    __shared__ long long s_center;
    __shared__ int s_again;

    const unsigned long long key = a.keys[tag];
    if (key == 0ull) {               // no valid lag was searched for this tag
        if (t == 0) a.found[tag] = 0;
        return;
    }
    if (t == 0) {
        double s = 0.0;
        for (int i = 0; i < kPowerParts; ++i) s += a.parts[i];
        s_px = s / double(a.n);
    }
    const unsigned idx = ~unsigned(key & 0xffffffffull);
    const int k = int(idx % unsigned(a.K));
    int64_t center = int64_t(idx / unsigned(a.K));
    const int R = a.radius;
    const int W = 2 * R + 3;
    const int64_t mrot = a.rot_signed[k];
    const int8_t* ch = a.chips + size_t(tag) * size_t(a.C);

    for (int pass = 0; pass < 2; ++pass) {
        const int64_t lam0 = center - R - 1;
        double cr[kMaxWin], ci[kMaxWin], en[kMaxWin];
#pragma unroll
        for (int w = 0; w < kMaxWin; ++w) cr[w] = ci[w] = en[w] = 0.0;
        for (int64_t e = t; e < a.L + W - 1; e += 256) {
            const int64_t i = lam0 + e;
            if (i < 0 || i >= a.n) continue;
            const float2 xv = a.x[i];
            const double xr = xv.x, xi = xv.y;
            int64_t ph = (mrot * i) % a.M;
            if (ph < 0) ph += a.M;
            double sn, cs;
            sincospi(2.0 * double(ph) / double(a.M), &sn, &cs);
            const double mr = xr * cs + xi * sn;      // x * exp(-j 2 pi m i / M)
            const double mi = xi * cs - xr * sn;
            const double pw = xr * xr + xi * xi;
#pragma unroll
            for (int w = 0; w < kMaxWin; ++w) {
                const int64_t nn = e - w;
                if (w < W && nn >= 0 && nn < a.L) {
                    const double sg = double(ch[nn / a.spc]);
                    cr[w] += mr * sg;
                    ci[w] += mi * sg;
                    en[w] += pw;
                }
            }
        }
#pragma unroll
        for (int w = 0; w < kMaxWin; ++w) {
            const double r0 = wave_sum(cr[w]), r1 = wave_sum(ci[w]), r2 = wave_sum(en[w]);
            if (lane == 0 && w < W) {
                red[wave][w][0] = r0;
                red[wave][w][1] = r1;
                red[wave][w][2] = r2;
            }
        }
        __syncthreads();
        if (t == 0) {
            double P[kMaxWin], E[kMaxWin];
            for (int w = 0; w < W; ++w) {
                const double re = (red[0][w][0] + red[1][w][0]) + (red[2][w][0] + red[3][w][0]);
                const double im = (red[0][w][1] + red[1][w][1]) + (red[2][w][1] + red[3][w][1]);
                E[w] = (red[0][w][2] + red[1][w][2]) + (red[2][w][2] + red[3][w][2]);
                const int64_t lam = lam0 + w;
                P[w] = (lam >= 0 && lam < a.lags) ? re * re + im * im : -1.0;
            }
            int wb = R + 1;
            for (int w = 1; w <= W - 2; ++w)
                if (P[w] > P[wb] || (P[w] == P[wb] && w < wb)) wb = w;
            const int64_t lam = lam0 + wb;
            const bool hit = (wb == 1 && lam > 0) || (wb == W - 2 && lam < a.lags - 1);
            if (hit && pass == 0) {
                s_center = lam;
                s_again = 1;
            } else {
                s_again = 0;
                unsigned flags = hit ? ACQ_DET_WINDOW_EDGE : 0u;
                const double p0 = P[wb];
                const double pm = P[wb - 1] < 0.0 ? 0.0 : P[wb - 1];
                const double pp = P[wb + 1] < 0.0 ? 0.0 : P[wb + 1];
                double delta = 0.0;
                if (lam == 0 || lam == a.lags - 1) {
                    flags |= ACQ_DET_NEAR_EDGE;
                } else {
                    const double den = pm - 2.0 * p0 + pp;
                    if (den < 0.0) {
                        delta = 0.5 * (pm - pp) / den;
                        delta = delta > 0.5 ? 0.5 : (delta < -0.5 ? -0.5 : delta);
                    }
                }
                const double px = s_px;
                const double z = px > 0.0 ? p0 / (double(a.L) * px) : 0.0;
                acq_detection d;
                d.tag = tag;
                d.bin = k;
                d.lag = lam;
                d.toa_samples = double(lam) + delta;
                d.freq_hz = a.freqs[k];
                d.peak_power = p0;
                d.z = z;
                d.energy = E[wb];
                d.block_power = px;
                d.block = 0;
                d.flags = flags;
                a.dets[tag] = d;
                a.found[tag] = z >= a.theta ? 1 : 0;
            }
        }
        __syncthreads();
        if (!s_again) break;
        center = s_center;
    }
}

__global__ void k_compact(const acq_detection* __restrict__ dets, const int32_t* __restrict__ found,
                          int T, acq_detection* __restrict__ out, int32_t* __restrict__ count) {
    if (threadIdx.x != 0 || blockIdx.x != 0) return;
    int c = 0;
    for (int i = 0; i < T; ++i)
        if (found[i]) out[c++] = dets[i];
    *count = c;
}

}  // namespace

// ------------------------------------------------------------------ launchers
hipError_t launch_block_power(const float2* x, int64_t n, double* parts, hipStream_t st) {
    hipLaunchKernelGGL(k_block_power, dim3(kPowerParts), dim3(256), 0, st, x, n, parts);
    return hipGetLastError();
}

hipError_t launch_fill_u64(unsigned long long* p, int64_t count, hipStream_t st) {
    if (count <= 0) return hipSuccess;
    const int64_t blocks = (count + 255) / 256;
    hipLaunchKernelGGL(k_fill_u64, dim3(unsigned(blocks)), dim3(256), 0, st, p, count);
    return hipGetLastError();
}

template <class E>
static hipError_t fwd_e(const FwdArgs& a, int prec, hipStream_t st) {
    switch (prec) {
        case ACQ_FP32: hipLaunchKernelGGL((k_forward<E, ACQ_FP32>), dim3(a.S), dim3(E::NT), 0, st, a); break;
        case ACQ_FP16: hipLaunchKernelGGL((k_forward<E, ACQ_FP16>), dim3(a.S), dim3(E::NT), 0, st, a); break;
        case ACQ_BF16: hipLaunchKernelGGL((k_forward<E, ACQ_BF16>), dim3(a.S), dim3(E::NT), 0, st, a); break;
        default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

hipError_t launch_forward(const FwdArgs& a, int log2_sub, int prec, hipStream_t st) {
    if (a.S <= 0) return hipSuccess;
    if ((1 << log2_sub) != a.Msub) return hipErrorInvalidValue;
    switch (log2_sub) {
        case 10: return fwd_e<StockhamEngine<10>>(a, prec, st);
        case 11: return fwd_e<StockhamEngine<11>>(a, prec, st);
        case 12: return fwd_e<StockhamEngine<12>>(a, prec, st);
        case 13: return fwd_e<StockhamEngine<13>>(a, prec, st);
        case 14: return fwd_e<Fft14>(a, prec, st);
        default: return hipErrorInvalidValue;
    }
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

template <class E, int PREC>
static void corr_ep(const CorrArgs& a, int grid, hipStream_t st) {
    if (a.dump)
        hipLaunchKernelGGL((k_correlate<E, PREC, true>), dim3(grid), dim3(E::NT), 0, st, a);
    else
        hipLaunchKernelGGL((k_correlate<E, PREC, false>), dim3(grid), dim3(E::NT), 0, st, a);
}

template <class E>
static hipError_t corr_e(const CorrArgs& a, int prec, hipStream_t st) {
    const int grid = ((a.nwork + 7) / 8) * 8;
    switch (prec) {
        case ACQ_FP32: corr_ep<E, ACQ_FP32>(a, grid, st); break;
        case ACQ_FP16: corr_ep<E, ACQ_FP16>(a, grid, st); break;
        case ACQ_BF16: corr_ep<E, ACQ_BF16>(a, grid, st); break;
        default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

hipError_t launch_correlate(const CorrArgs& a, int log2_sub, int prec, hipStream_t st) {
    if (a.nwork <= 0) return hipSuccess;
    if ((1 << log2_sub) != a.Msub || a.tile < 1 || a.tile > kMaxTagTile) return hipErrorInvalidValue;
    switch (log2_sub) {
        case 10: return corr_e<StockhamEngine<10>>(a, prec, st);
        case 11: return corr_e<StockhamEngine<11>>(a, prec, st);
        case 12: return corr_e<StockhamEngine<12>>(a, prec, st);
        case 13: return corr_e<StockhamEngine<13>>(a, prec, st);
        case 14: return corr_e<Fft14>(a, prec, st);
        default: return hipErrorInvalidValue;
    }
}

hipError_t launch_refine(const RefineArgs& a, hipStream_t st) {
    if (a.radius < 0 || a.radius > kMaxRefineRadius) return hipErrorInvalidValue;
    hipLaunchKernelGGL(k_refine, dim3(a.T), dim3(256), 0, st, a);
    return hipGetLastError();
}

hipError_t launch_compact(const acq_detection* dets, const int32_t* found, int T, acq_detection* out,
                          int32_t* count, hipStream_t st) {
    hipLaunchKernelGGL(k_compact, dim3(1), dim3(64), 0, st, dets, found, T, out, count);
    return hipGetLastError();
}

}  // namespace acq
