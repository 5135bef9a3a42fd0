// C ABI of the acquisition library: plan lifecycle, single-block and batched
// searches, tuning and kernel timing.
//
// A plan owns everything that does not change from block to block (Section
// 4.2: allocate once, keep the transformed replicas and transform tables on the
// GPU for the plan's lifetime): the replica spectra, the rectangular-chip
// spectrum, the unit-root tables, the per-bin rotations, the segment-spectra
// workspace (sized for the largest batch), the result buffers and pinned host
// staging.  A search only launches kernels on the plan's stream and copies the
// detections back.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <mutex>
#include <new>
#include <string>
#include <type_traits>
#include <vector>

#include "acq.h"
#include "cnn_internal.h"
#include "host_logic.h"
#include "kernels.h"

using acq::BlockDesc;
using acq::BlockTable;
using acq::Geometry;

// Per-search device buffers: everything a search writes, sized for the
// plan's batch capacity.  They live in one region, the plan's workspace
// (caller-owned, or allocated by acq_plan when the caller passes none).
struct Scratch {
    float2* X = nullptr;                // [segments][classes][M] FP32 segment spectra
    void* Xh = nullptr;                 // [segments][classes][M] 16-bit segment spectra (FP16/BF16 plans)
    unsigned long long* keys = nullptr; // [blocks][T] peak keys
    unsigned* cross = nullptr;          // [blocks][T] threshold crossings
    double* parts = nullptr;            // [blocks][kPowerParts] block-power partial sums
    int* exps = nullptr;                // [blocks] 16-bit storage prescale exponents
    float* pthr = nullptr;              // [blocks] power at the detection threshold
    int32_t* bad = nullptr;             // [blocks] 1: a non-finite sample
    acq_detection* dets = nullptr;      // [blocks][T] candidates
    acq_detection* out = nullptr;       // [blocks][T] detections, compacted
    int32_t* found = nullptr;           // [blocks][T]
    double* refpart = nullptr;          // refinement partial sums [blocks * T][parts][3 * window]
    int64_t* refcenter = nullptr;       // [blocks * T] refinement re-centring
    int32_t* count = nullptr;           // [2]: detections, blocks holding a non-finite sample
    int* counters = nullptr;            // [kXcds] persistent-launch work counters
    BlockDesc* descs = nullptr;         // [blocks]
    int32_t* counts = nullptr;          // [2] = {blocks, segments} of a batch
    int32_t* seglist = nullptr;         // segments searched by a proposal search
};

struct acq_plan_s {
    acq_config cfg{};
    Geometry g;
    hipStream_t stream = nullptr;
    int device = 0;
    int cus = 256;                      // compute units (persistent grid size)
    int engine = 0;                     // acq_tuning.engine
    int tile = 16;                      // acq_tuning.tag_tile
    int batch_launch = ACQ_BATCH_GRID;  // acq_tuning.batch_launch
    int track_bins = 0;                 // acq_tuning.track_bins (0: chosen per launch)

    Scratch ws;                         // per-search buffers in the workspace
    void* own_ws = nullptr;             // the workspace when acq_plan allocated it
    int32_t* d_cls = nullptr;           // [K] residual class of each bin
    double* d_cls_cyc = nullptr;        // [classes] residual offsets, cycles per sample
    double* d_cyc = nullptr;            // [K] f_k / Fs
    void* d_bank = nullptr;             // [T][bank_stride(Msub)]: spectrum entries 0 .. Msub/2, storage format
    int bank_exp = 0;                   // power-of-two prescale of the stored bank
    float2* d_wts = nullptr;            // [spc][M] first-step weights of the split inverse transform
    float2* d_rootsM = nullptr;         // [M]
    float2* d_rootsSub = nullptr;       // [Msub]
    double2* d_roots64 = nullptr;       // [M] FP64 unit roots (refinement mix)
    float2* d_b1tab = nullptr;          // 2^14-point engine table (or a 1-entry stub)
    int8_t* d_chips = nullptr;          // [T][C]
    int32_t* d_rot = nullptr;           // [K]
    int64_t* d_rot_signed = nullptr;    // [K]
    double* d_freqs = nullptr;          // [K]
    acq_detection* h_out = nullptr;     // pinned [blocks][T]
    int32_t* h_count = nullptr;         // pinned [2]
    BlockDesc* h_descs = nullptr;       // pinned [blocks]
    int32_t* h_counts = nullptr;        // pinned [2]
    int32_t* h_iota = nullptr;          // pinned [max_segments] 0, 1, 2, ... (full-search lists)
    hipEvent_t desc_ev = nullptr;       // after the last upload of h_descs / h_counts
    bool desc_pending = false;

    bool profiling = false;
    int profile_mode = ACQ_PROFILE_OFF;
    unsigned profile_mask = 0;            // bit k: time kernel ACQ_KERNEL_k
    bool capturing = false;             // capturing the plan's own batch graph
    bool ext_capture = false;           // the plan's stream is being captured by the caller
    hipEvent_t ev[ACQ_NUM_KERNELS][2] = {};
    bool ev_used[ACQ_NUM_KERNELS] = {};

    void* scratch = nullptr;            // this device's address of the static search scratch
                                        // (acq_detect_noalloc), resolved by acq_plan

    hipStream_t cap_stream = nullptr;   // private stream the batch graphs are captured on
    hipGraph_t graph = nullptr;         // searching batch
    hipGraphExec_t gexec = nullptr;
    hipGraph_t tgraph = nullptr;        // tracking batch
    hipGraphExec_t tgexec = nullptr;
};

// Per-search buffers of acq_detect_noalloc, which may allocate nothing: one
// array in the library's code object, so every GPU the library runs on holds
// its own copy (for the life of the process).  In host code the name stands
// for no device address; its device address comes from hipGetSymbolAddress.
constexpr size_t kStaticScratchBytes = size_t(64) << 20;
static __device__ __align__(256) char scratch[kStaticScratchBytes];

namespace {

std::mutex g_scratch_mu;
std::vector<void*> g_scratch_addr;          // per device, once resolved

// Device address of `scratch` on `device` (the current device), resolved once
// per device.
hipError_t static_scratch_address(int device, void** out) {
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (device < 0) return hipErrorInvalidDevice;
    if (size_t(device) >= g_scratch_addr.size()) g_scratch_addr.resize(size_t(device) + 1, nullptr);
    if (!g_scratch_addr[size_t(device)]) {
        void* ptr = nullptr;
        const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return e;
        g_scratch_addr[size_t(device)] = ptr;
    }
    *out = g_scratch_addr[size_t(device)];
    return hipSuccess;
}

std::string hip_msg(const char* what, hipError_t e) {
    return std::string(what) + ": " + hipGetErrorString(e);
}

#define ACQ_HIP(call)                                                            \
    do {                                                                         \
        hipError_t e_ = (call);                                                  \
        if (e_ != hipSuccess) {                                                  \
            return acq::fail(e_ == hipErrorOutOfMemory ? ACQ_ERR_OOM : ACQ_ERR_DEVICE, \
                             hip_msg(#call, e_));                                \
        }                                                                        \
    } while (0)

template <typename T>
hipError_t dalloc(T** p, size_t count) {
    return hipMalloc(reinterpret_cast<void**>(p), sizeof(T) * (count ? count : 1));
}

void drop_graph(acq_plan_s* p) {
    if (p->gexec) (void)hipGraphExecDestroy(p->gexec);
    if (p->graph) (void)hipGraphDestroy(p->graph);
    if (p->tgexec) (void)hipGraphExecDestroy(p->tgexec);
    if (p->tgraph) (void)hipGraphDestroy(p->tgraph);
    p->gexec = nullptr;
    p->graph = nullptr;
    p->tgexec = nullptr;
    p->tgraph = nullptr;
}

void free_plan(acq_plan_s* p) {
    if (!p) return;
    drop_graph(p);
    void* dev[] = {p->own_ws, p->d_cls, p->d_cls_cyc, p->d_cyc, p->d_bank, p->d_wts, p->d_rootsM, p->d_rootsSub,
                   p->d_roots64, p->d_b1tab, p->d_chips, p->d_rot, p->d_rot_signed, p->d_freqs};
    for (void* d : dev)
        if (d) (void)hipFree(d);
    void* host[] = {p->h_out, p->h_count, p->h_descs, p->h_counts, p->h_iota};
    for (void* h : host)
        if (h) (void)hipHostFree(h);
    for (auto& pair : p->ev)
        for (hipEvent_t e : pair)
            if (e) (void)hipEventDestroy(e);
    if (p->desc_ev) (void)hipEventDestroy(p->desc_ev);
    if (p->cap_stream) (void)hipStreamDestroy(p->cap_stream);
    delete p;
}

constexpr size_t kWsAlign = 256;

// Carve the per-search buffers of `blocks` blocks and `segments` segment
// spectra (and a proposal list of `seglist` entries) out of `base`, each
// aligned to kWsAlign bytes.  Returns the bytes used; with base == nullptr
// only the size is computed.
size_t layout_scratch(const Geometry& g, const acq_config& c, int64_t blocks, int64_t segments, int64_t seglist,
                      char* base, Scratch* s) {
    size_t off = 0;
    auto take = [&](auto*& ptr, size_t bytes) {
        using P = std::remove_reference_t<decltype(ptr)>;
        ptr = base ? reinterpret_cast<P>(base + off) : nullptr;
        off += (std::max<size_t>(bytes, 1) + kWsAlign - 1) / kWsAlign * kWsAlign;
    };
    const size_t T = size_t(c.num_tags), B = size_t(blocks), S = size_t(std::max<int64_t>(segments, 1));
    const size_t spectra = S * size_t(g.ncls) * size_t(g.xstride);
    const size_t wmax = c.refine_radius <= 1 ? 5 : size_t(2 * acq::kMaxRefineRadius + 3);
    take(s->X, spectra * sizeof(float2));
    if (c.precision != ACQ_FP32) take(s->Xh, spectra * 4);
    else s->Xh = nullptr;
    take(s->keys, B * T * sizeof(unsigned long long));
    take(s->cross, B * T * sizeof(unsigned));
    take(s->parts, B * size_t(acq::kPowerParts) * sizeof(double));
    take(s->exps, B * sizeof(int));
    take(s->pthr, B * sizeof(float));
    take(s->bad, B * sizeof(int32_t));
    take(s->dets, B * T * sizeof(acq_detection));
    take(s->out, B * T * sizeof(acq_detection));
    take(s->found, B * T * sizeof(int32_t));
    take(s->refpart, B * T * size_t(acq::kRefineParts) * 3 * wmax * sizeof(double));
    take(s->refcenter, B * T * sizeof(int64_t));
    take(s->count, 2 * sizeof(int32_t));
    take(s->counters, size_t(acq::kXcds) * sizeof(int));
    take(s->descs, B * sizeof(BlockDesc));
    take(s->counts, 2 * sizeof(int32_t));
    take(s->seglist, size_t(std::max<int64_t>(seglist, 1)) * sizeof(int32_t));
    return off;
}

size_t workspace_bytes(const Geometry& g, const acq_config& c) {
    Scratch s;
    return layout_scratch(g, c, g.max_blocks, std::max<int64_t>(g.max_total_segments, 1),
                          std::max<int64_t>({g.max_segments, g.max_total_segments, 1}), nullptr, &s);
}

// Device memory a plan holds besides its workspace: replica bank and tables.
size_t own_bytes(const Geometry& g, const acq_config& c) {
    const size_t T = size_t(c.num_tags), K = size_t(c.num_bins);
    const size_t half = c.precision != ACQ_FP32 ? 4 : 8;
    size_t b = T * size_t(acq::bank_stride(int(g.Msub))) * half;
    b += size_t(g.M) * size_t(c.samples_per_chip) * 8 + size_t(g.M) * 8 + size_t(g.Msub) * 8 + size_t(g.M) * 16;
    b += (g.log2_sub == 14 ? size_t(16 * 16 * 64) : 1) * 8;
    b += T * size_t(c.num_chips) + K * (4 + 8 + 8 + 8 + 4) + size_t(g.ncls) * 8;
    return b;
}

int build_plan(acq_plan_s* p, void* workspace, size_t ws_bytes) {
    const Geometry& g = p->g;
    const acq_config& c = p->cfg;
    const size_t T = size_t(c.num_tags), C = size_t(c.num_chips), K = size_t(c.num_bins);
    const size_t B = size_t(g.max_blocks);
    const bool half = c.precision != ACQ_FP32;
    const size_t ncls = size_t(g.ncls);
    const size_t need = workspace_bytes(g, c);
    char* base = static_cast<char*>(workspace);
    if (!base) {
        ACQ_HIP(hipMalloc(&p->own_ws, need));
        base = static_cast<char*>(p->own_ws);
    } else if (ws_bytes < need) {
        return acq::fail(ACQ_ERR_WORKSPACE_TOO_SMALL, "workspace smaller than acq_workspace_size");
    }
    layout_scratch(g, c, g.max_blocks, std::max<int64_t>(g.max_total_segments, 1),
                   std::max<int64_t>({g.max_segments, g.max_total_segments, 1}), base, &p->ws);
    ACQ_HIP(dalloc(&p->d_cls, K));
    ACQ_HIP(dalloc(&p->d_cls_cyc, ncls));
    ACQ_HIP(dalloc(&p->d_cyc, K));
    ACQ_HIP(hipMalloc(&p->d_bank, T * size_t(acq::bank_stride(int(g.Msub))) * (half ? 4 : 8)));
    // 16-bit banks are stored with rms magnitude near 1: 2^round(log2(M / sqrt(C)))
    p->bank_exp = half ? int(std::lrint(std::log2(double(g.M) / std::sqrt(double(C))))) : 0;
    ACQ_HIP(dalloc(&p->d_wts, size_t(g.M) * size_t(c.samples_per_chip)));
    ACQ_HIP(dalloc(&p->d_rootsM, size_t(g.M)));
    ACQ_HIP(dalloc(&p->d_rootsSub, size_t(g.Msub)));
    ACQ_HIP(dalloc(&p->d_roots64, size_t(g.M)));
    const std::vector<float> b1 = g.log2_sub == 14 ? acq::fft14_b1_table() : std::vector<float>(2, 0.f);
    ACQ_HIP(dalloc(&p->d_b1tab, b1.size() / 2));
    ACQ_HIP(dalloc(&p->d_chips, T * C));
    ACQ_HIP(dalloc(&p->d_rot, K));
    ACQ_HIP(dalloc(&p->d_rot_signed, K));
    ACQ_HIP(dalloc(&p->d_freqs, K));
    ACQ_HIP(hipHostMalloc(reinterpret_cast<void**>(&p->h_iota), sizeof(int32_t) * size_t(std::max<int64_t>(g.max_segments, 1))));
    for (int64_t j = 0; j < g.max_segments; ++j) p->h_iota[j] = int32_t(j);
    ACQ_HIP(hipHostMalloc(reinterpret_cast<void**>(&p->h_out), sizeof(acq_detection) * B * T));
    ACQ_HIP(hipHostMalloc(reinterpret_cast<void**>(&p->h_count), sizeof(int32_t) * 2));
    ACQ_HIP(hipHostMalloc(reinterpret_cast<void**>(&p->h_descs), sizeof(BlockDesc) * B));
    ACQ_HIP(hipHostMalloc(reinterpret_cast<void**>(&p->h_counts), sizeof(int32_t) * 2));
    ACQ_HIP(hipEventCreateWithFlags(&p->desc_ev, hipEventDisableTiming));

    const std::vector<float> rootsM = acq::unit_roots(g.M);
    const std::vector<float> rootsSub = acq::unit_roots(g.Msub);
    const std::vector<double> roots64 = acq::unit_roots64(g.M);
    const std::vector<float> wts = acq::phase_weights(g.M, c.samples_per_chip);
    hipStream_t st = p->stream;
    // nothing has been searched yet: results read before the first search are empty
    ACQ_HIP(acq::launch_fill_i32(p->ws.count, 2, st));
    ACQ_HIP(hipMemcpyAsync(p->d_rootsM, rootsM.data(), rootsM.size() * sizeof(float), hipMemcpyHostToDevice, st));
    ACQ_HIP(hipMemcpyAsync(p->d_rootsSub, rootsSub.data(), rootsSub.size() * sizeof(float), hipMemcpyHostToDevice, st));
    ACQ_HIP(hipMemcpyAsync(p->d_roots64, roots64.data(), roots64.size() * sizeof(double), hipMemcpyHostToDevice, st));
    ACQ_HIP(hipMemcpyAsync(p->d_wts, wts.data(), wts.size() * sizeof(float), hipMemcpyHostToDevice, st));
    ACQ_HIP(hipMemcpyAsync(p->d_b1tab, b1.data(), b1.size() * sizeof(float), hipMemcpyHostToDevice, st));
    ACQ_HIP(hipMemcpyAsync(p->d_chips, c.chips, T * C, hipMemcpyHostToDevice, st));
    ACQ_HIP(hipMemcpyAsync(p->d_rot, g.rot.data(), K * sizeof(int32_t), hipMemcpyHostToDevice, st));
    ACQ_HIP(hipMemcpyAsync(p->d_rot_signed, g.rot_signed.data(), K * sizeof(int64_t), hipMemcpyHostToDevice, st));
    ACQ_HIP(hipMemcpyAsync(p->d_freqs, g.freqs_hz.data(), K * sizeof(double), hipMemcpyHostToDevice, st));
    ACQ_HIP(hipMemcpyAsync(p->d_cls, g.cls.data(), K * sizeof(int32_t), hipMemcpyHostToDevice, st));
    ACQ_HIP(hipMemcpyAsync(p->d_cls_cyc, g.cls_cyc.data(), ncls * sizeof(double), hipMemcpyHostToDevice, st));
    ACQ_HIP(hipMemcpyAsync(p->d_cyc, g.cyc.data(), K * sizeof(double), hipMemcpyHostToDevice, st));
    ACQ_HIP(acq::launch_bank(p->d_chips, int(T), int(C), p->d_bank, p->d_rootsSub, p->d_b1tab, int(g.Msub),
                             int(g.M), p->bank_exp, g.log2_sub, c.precision, st));
    ACQ_HIP(hipStreamSynchronize(st));
    return ACQ_OK;
}

// Event pair around one kernel launch when profiling is on (not while capturing).
struct KernelTimer {
    acq_plan_s* p;
    int id;
    bool on;
    KernelTimer(acq_plan_s* plan, int kernel)
        : p(plan), id(kernel),
          on(plan->profiling && ((plan->profile_mask >> kernel) & 1u) && !plan->capturing && !plan->ext_capture) {
        if (on) {
            (void)hipEventRecord(p->ev[id][0], p->stream);
            p->ev_used[id] = true;
        }
    }
    ~KernelTimer() {
        if (on) (void)hipEventRecord(p->ev[id][1], p->stream);
    }
};

void reset_timers(acq_plan_s* p) {
    for (bool& u : p->ev_used) u = false;
}

double threshold_for(const acq_plan_s* p, int64_t n) {
    const acq_config& c = p->cfg;
    return c.threshold > 0.0 ? c.threshold : acq::default_threshold(c.num_tags, c.num_bins, n, p->g.L);
}

// Where a search leaves its results: the compacted detections (at most
// `capacity` records) and their count, in device memory, optionally copied to
// the plan's pinned staging.
struct ResultDest {
    acq_detection* out;
    int32_t capacity;
    int32_t* count;             // [1]
    bool to_host;
};

ResultDest workspace_dest(const acq_plan_s* p, bool to_host) {
    return ResultDest{p->ws.out, int32_t(std::min<int64_t>(int64_t(p->g.max_blocks) * p->cfg.num_tags, INT32_MAX)),
                      p->ws.count, to_host};
}

// Launch sequence of a search on stream st, in the buffers of `w`.  `bt`
// holds one inline block (single-block calls: plain grids sized on the host)
// or the plan's device block table (batches: persistent grids that do not
// depend on the batch, so the sequence can be captured once and replayed).
// track: every block is a tracking task searched for its own tag only.
int enqueue_search(acq_plan_s* p, const Scratch& w, const BlockTable& bt, bool batch, int total_seg_host, float* dump,
                   bool refine, hipStream_t st, bool track, const ResultDest& dst) {
    const Geometry& g = p->g;
    const acq_config& c = p->cfg;
    const int nb_grid = batch ? g.max_blocks : 1;
    {
        KernelTimer kt(p, ACQ_KERNEL_BLOCK_POWER);
        ACQ_HIP(acq::launch_block_power(bt, nb_grid, c.max_block_len, w.parts, st));
    }
    // block statistics; the same launch clears the peak keys and crossing counts
    ACQ_HIP(acq::launch_block_stats(bt, w.parts, int(g.M), g.L, w.exps, w.pthr, w.bad, w.count + 1, w.keys, w.cross,
                                    int64_t(nb_grid) * c.num_tags, st));

    acq::FwdArgs fa{};
    fa.blocks = bt;
    fa.X = w.X;
    fa.Xh = w.Xh;
    fa.exps = w.exps;
    fa.cls_cyc = p->d_cls_cyc;
    fa.ncls = g.ncls;
    fa.rootsM = p->d_rootsM;
    fa.rootsSub = p->d_rootsSub;
    fa.b1tab = p->d_b1tab;
    fa.V = g.V;
    fa.xstride = g.xstride;
    fa.xpad = int(g.xpad);
    fa.spc = c.samples_per_chip;
    fa.M = int(g.M);
    fa.Msub = int(g.Msub);
    {
        KernelTimer kt(p, ACQ_KERNEL_FORWARD);
        // one workgroup per item (so that a segment's items can share an XCD);
        // a captured batch sizes both steps for the plan's capacity and the
        // surplus workgroups exit
        const int slots = (batch && p->capturing ? int(g.max_total_segments) : total_seg_host) * g.ncls;
        const int grid = slots * c.samples_per_chip;
        ACQ_HIP(acq::launch_forward(fa, grid, slots, g.log2_sub, c.precision, st));
    }

    acq::CorrArgs ca{};
    ca.blocks = bt;
    ca.X = c.precision == ACQ_FP32 ? static_cast<const void*>(w.X) : w.Xh;
    ca.bank = p->d_bank;
    ca.exps = w.exps;
    ca.wts = p->d_wts;
    ca.rootsM = p->d_rootsM;
    ca.rootsSub = p->d_rootsSub;
    ca.b1tab = p->d_b1tab;
    ca.rot = p->d_rot;
    ca.cls = p->d_cls;
    ca.ncls = g.ncls;
    ca.keys = w.keys;
    ca.pthr = w.pthr;
    ca.cross = w.cross;
    ca.dump = dump;
    ca.counters = w.counters;
    ca.V = g.V;
    ca.xstride = g.xstride;
    ca.xpad = int(g.xpad);
    ca.K = c.num_bins;
    ca.spc = c.samples_per_chip;
    ca.M = int(g.M);
    ca.Msub = int(g.Msub);
    ca.T = c.num_tags;
    ca.tile = p->tile;
    ca.ntiles = (c.num_tags + p->tile - 1) / p->tile;
    ca.bank_exp = p->bank_exp;
    ca.persistent = batch && !track && p->batch_launch == ACQ_BATCH_PERSISTENT ? 1 : 0;
    ca.track = track ? 1 : 0;
    int grid;
    if (track) {
        // bins per work item: enough items to give every compute unit about
        // two, each amortising its setup (the task's replica spectrum, the
        // item's addressing) over as many bins as that allows (256 tasks x 21
        // bins: all 21 bins per item, 0.421 ms; four items per CU gave 7 bins
        // per item and 0.430 ms, 11 bins 0.437 ms).  The choice follows this batch's
        // segments (for a captured graph, those of the batch it was captured
        // on), while a captured graph sizes its grid for the plan's capacity.
        const int64_t segs = p->capturing ? int64_t(g.max_total_segments) : int64_t(total_seg_host);
        int bins = p->track_bins;
        if (bins <= 0) {
            const int64_t per_bin = int64_t(total_seg_host) * c.samples_per_chip;
            const int64_t want = int64_t(2) * p->cus;
            bins = int(std::max<int64_t>(1, std::min<int64_t>(c.num_bins, per_bin * c.num_bins / want)));
            const int ntl = (c.num_bins + bins - 1) / bins;      // even tiles
            bins = (c.num_bins + ntl - 1) / ntl;
        }
        bins = std::min(bins, c.num_bins);
        ca.tile = bins;
        ca.ntiles = 1;
        const int64_t nwork = segs * ((c.num_bins + bins - 1) / bins) * c.samples_per_chip;
        if (nwork >= (int64_t(1) << 31) - 8) return acq::fail(ACQ_ERR_UNSUPPORTED, "too many work items");
        grid = int((nwork + acq::kXcds - 1) / acq::kXcds) * acq::kXcds;
    } else if (ca.persistent) {
        ACQ_HIP(acq::launch_fill_i32(w.counters, acq::kXcds, st));
        grid = p->cus;
    } else {
        // batches captured into a graph size the grid for the plan's capacity;
        // the kernel reads the real item count from the block table
        const int64_t segs = batch && p->capturing ? int64_t(g.max_total_segments) : int64_t(total_seg_host);
        const int64_t nwork = int64_t(ca.ntiles) * segs * c.num_bins * c.samples_per_chip;
        if (nwork >= (int64_t(1) << 31) - 8) return acq::fail(ACQ_ERR_UNSUPPORTED, "too many work items");
        grid = int((nwork + acq::kXcds - 1) / acq::kXcds) * acq::kXcds;
    }
    {
        KernelTimer kt(p, ACQ_KERNEL_CORRELATE);
        ACQ_HIP(acq::launch_correlate(ca, grid, g.log2_sub, c.precision, p->engine, st));
    }
    if (!refine) return ACQ_OK;

    acq::RefineArgs ra{};
    ra.blocks = bt;
    ra.chips = p->d_chips;
    ra.rot_signed = p->d_rot_signed;
    ra.freqs = p->d_freqs;
    ra.keys = w.keys;
    ra.parts = w.parts;
    ra.bad = w.bad;
    ra.cross = w.cross;
    ra.check_finite = (c.flags & ACQ_FLAG_CHECK_FINITE) ? 1 : 0;
    ra.dets = w.dets;
    ra.found = w.found;
    ra.L = g.L;
    ra.T = c.num_tags;
    ra.C = c.num_chips;
    ra.K = c.num_bins;
    ra.spc = c.samples_per_chip;
    ra.log2_spc = c.samples_per_chip == 1 ? 0 : c.samples_per_chip == 2 ? 1 : c.samples_per_chip == 4 ? 2 : 3;
    ra.roots64 = p->d_roots64;
    ra.cyc = p->d_cyc;
    ra.exact = g.exact ? 1 : 0;
    ra.M = int(g.M);
    ra.radius = c.refine_radius > 0 ? c.refine_radius : 1;
    ra.track = track ? 1 : 0;
    ra.partial = w.refpart;
    ra.center = w.refcenter;
    {
        KernelTimer kt(p, ACQ_KERNEL_REFINE);
        ACQ_HIP(acq::launch_refine(ra, nb_grid, st));
    }
    {
        KernelTimer kt(p, ACQ_KERNEL_COMPACT);
        ACQ_HIP(acq::launch_compact(bt, w.dets, w.found, c.num_tags, track ? 1 : 0, dst.out, dst.capacity, dst.count,
                                    st));
    }
    if (!dst.to_host) return ACQ_OK;
    ACQ_HIP(hipMemcpyAsync(p->h_count, w.count, 2 * sizeof(int32_t), hipMemcpyDeviceToHost, st));
    // at most one detection per (block, tag), per task when tracking
    const size_t most = size_t(nb_grid) * size_t(track ? 1 : c.num_tags);
    ACQ_HIP(hipMemcpyAsync(p->h_out, w.out, sizeof(acq_detection) * most, hipMemcpyDeviceToHost, st));
    return ACQ_OK;
}

int check_block(acq_plan_s* p, const void* block, int64_t n) {
    if (!p) return acq::fail(ACQ_ERR_INVALID_ARG, "null plan");
    if (n < 0) return acq::fail(ACQ_ERR_INVALID_ARG, "negative block length");
    if (n > p->cfg.max_block_len) return acq::fail(ACQ_ERR_BLOCK_TOO_LONG, "block longer than max_block_len");
    if (n > 0 && !block) return acq::fail(ACQ_ERR_INVALID_ARG, "null block");
    if (reinterpret_cast<uintptr_t>(block) % 8 != 0)
        return acq::fail(ACQ_ERR_INVALID_ARG, "block must be 8-byte aligned");
    return ACQ_OK;
}

BlockDesc single_desc(const acq_plan_s* p, const void* block, int64_t n) {
    BlockDesc d{};
    d.x = static_cast<const float2*>(block);
    d.n = n;
    d.lags = n - p->g.L + 1;
    d.seg0 = 0;
    d.nseg = d.lags > 0 ? int((d.lags + p->g.V - 1) / p->g.V) : 0;
    d.theta = threshold_for(p, n);
    d.tag = -1;
    return d;
}

bool async_mode(const acq_plan_s* p) { return (p->cfg.flags & ACQ_FLAG_ASYNC) != 0; }

// The host-side descriptor staging may be rewritten once the previous upload
// from it has run (asynchronous plans return before their searches run).
int wait_descriptors(acq_plan_s* p) {
    if (p->desc_pending) {
        ACQ_HIP(hipEventSynchronize(p->desc_ev));
        p->desc_pending = false;
    }
    return ACQ_OK;
}

// Copies the staged descriptors and runs a batch search: eagerly, or by
// replaying the plan's captured graph for this kind of batch (captured on
// first use with grids sized for the plan's capacity).
int launch_batch(acq_plan_s* p, int32_t seg, bool track) {
    BlockTable bt{};
    bt.descs = p->ws.descs;
    bt.counts = p->ws.counts;
    const size_t desc_bytes = sizeof(BlockDesc) * size_t(p->g.max_blocks);
    const ResultDest dst = workspace_dest(p, !async_mode(p));
    if (p->cfg.flags & ACQ_FLAG_GRAPH) {
        hipGraph_t& graph_ref = track ? p->tgraph : p->graph;
        hipGraphExec_t& exec_ref = track ? p->tgexec : p->gexec;
        if (!exec_ref) {
            if (!p->cap_stream) ACQ_HIP(hipStreamCreateWithFlags(&p->cap_stream, hipStreamNonBlocking));
            ACQ_HIP(hipStreamBeginCapture(p->cap_stream, hipStreamCaptureModeThreadLocal));
            p->capturing = true;
            int rc = ACQ_OK;
            hipError_t e = hipMemcpyAsync(p->ws.descs, p->h_descs, desc_bytes, hipMemcpyHostToDevice, p->cap_stream);
            if (e == hipSuccess)
                e = hipMemcpyAsync(p->ws.counts, p->h_counts, 2 * sizeof(int32_t), hipMemcpyHostToDevice,
                                   p->cap_stream);
            // grids follow the plan's capacity while capturing; the capturing
            // batch's segment count only guides the bins per tracking item
            if (e == hipSuccess)
                rc = enqueue_search(p, p->ws, bt, true, seg, nullptr, true, p->cap_stream, track, dst);
            p->capturing = false;
            hipGraph_t graph = nullptr;
            const hipError_t e2 = hipStreamEndCapture(p->cap_stream, &graph);
            if (e != hipSuccess || rc != ACQ_OK || e2 != hipSuccess) {
                if (graph) (void)hipGraphDestroy(graph);
                if (rc != ACQ_OK) return rc;
                return acq::fail(ACQ_ERR_DEVICE, hip_msg("graph capture", e != hipSuccess ? e : e2));
            }
            graph_ref = graph;
            ACQ_HIP(hipGraphInstantiate(&exec_ref, graph_ref, nullptr, nullptr, 0));
        }
        ACQ_HIP(hipGraphLaunch(exec_ref, p->stream));
        ACQ_HIP(hipEventRecord(p->desc_ev, p->stream));
        p->desc_pending = true;
    } else {
        ACQ_HIP(hipMemcpyAsync(p->ws.descs, p->h_descs, desc_bytes, hipMemcpyHostToDevice, p->stream));
        ACQ_HIP(hipMemcpyAsync(p->ws.counts, p->h_counts, 2 * sizeof(int32_t), hipMemcpyHostToDevice, p->stream));
        ACQ_HIP(hipEventRecord(p->desc_ev, p->stream));
        p->desc_pending = true;
        const int rc = enqueue_search(p, p->ws, bt, true, seg, nullptr, true, p->stream, track, dst);
        if (rc != ACQ_OK) return rc;
    }
    return ACQ_OK;
}

// Detections staged on the host after a synchronous search (or read back by
// acq_collect): copied to out, then the status.  Blocks holding non-finite
// samples (ACQ_FLAG_CHECK_FINITE) take precedence over truncation.
int deliver(acq_plan_s* p, acq_detection* out, int32_t capacity, int32_t* n_found, int32_t* block_of = nullptr) {
    const int32_t found = p->h_count[0];
    const int32_t nbad = p->h_count[1];
    *n_found = found;
    const int32_t ncopy = found < capacity ? found : capacity;
    if (ncopy > 0) std::memcpy(out, p->h_out, sizeof(acq_detection) * size_t(ncopy));
    if (block_of)
        for (int32_t i = 0; i < ncopy; ++i) block_of[i] = out[i].block;
    if ((p->cfg.flags & ACQ_FLAG_CHECK_FINITE) && nbad > 0)
        return acq::fail(ACQ_ERR_NON_FINITE, std::to_string(nbad) + " block(s) hold non-finite samples");
    if (found > capacity) return acq::fail(ACQ_ERR_TRUNCATED, "more detections than capacity");
    acq::clear_error();
    return ACQ_OK;
}

// Output arguments of a result-returning call: required unless the plan is
// asynchronous (its results stay on the device).
int check_outputs(const acq_plan_s* p, const acq_detection* out, int32_t capacity, const int32_t* n_found) {
    if (async_mode(p)) return ACQ_OK;
    if (!n_found) return acq::fail(ACQ_ERR_INVALID_ARG, "null n_found");
    if (capacity < 0 || (capacity > 0 && !out)) return acq::fail(ACQ_ERR_INVALID_ARG, "bad output buffer");
    return ACQ_OK;
}

// Note whether the caller is capturing the plan's stream into a graph (the
// plan's kernel timers stay off then).
int note_capture(acq_plan_s* p) {
    hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
    ACQ_HIP(hipStreamIsCapturing(p->stream, &cs));
    p->ext_capture = cs != hipStreamCaptureStatusNone;
    return ACQ_OK;
}

// End of a result-returning search: synchronous plans wait and deliver,
// asynchronous ones leave the results on the device.
int finish(acq_plan_s* p, acq_detection* out, int32_t capacity, int32_t* n_found, int32_t* block_of = nullptr) {
    if (async_mode(p)) {
        if (n_found) *n_found = 0;
        acq::clear_error();
        return ACQ_OK;
    }
    ACQ_HIP(hipStreamSynchronize(p->stream));
    return deliver(p, out, capacity, n_found, block_of);
}

// A call with nothing to search: the results are empty (device too, so that a
// later acq_collect or device read sees them).
int finish_empty(acq_plan_s* p, int32_t* n_found) {
    if (n_found) *n_found = 0;
    if (async_mode(p)) ACQ_HIP(acq::launch_fill_i32(p->ws.count, 2, p->stream));
    acq::clear_error();
    return ACQ_OK;
}

}  // namespace

extern "C" {

int acq_plan_geometry(const acq_config* cfg, acq_geometry* out) {
    if (!out) return acq::fail(ACQ_ERR_INVALID_ARG, "null output");
    Geometry g;
    const int rc = acq::derive_geometry(cfg, &g);
    if (rc != ACQ_OK) return rc;
    out->template_len = g.L;
    out->min_fft_len = g.m_min;
    out->fft_len = g.M;
    out->sub_fft_len = g.Msub;
    out->valid_per_segment = g.V;
    out->max_segments = g.max_segments;
    out->freq_quantum_hz = g.q;
    out->bin_center_hz = double(g.centre_q) * g.q;
    out->bin_step_hz = double(g.step_q) * g.q;
    out->workspace_bytes = int64_t(workspace_bytes(g, *cfg));
    out->device_bytes = int64_t(own_bytes(g, *cfg)) + out->workspace_bytes;
    return ACQ_OK;
}

int acq_workspace_size(const acq_config* cfg, size_t* bytes) {
    if (!bytes) return acq::fail(ACQ_ERR_INVALID_ARG, "null output");
    Geometry g;
    const int rc = acq::derive_geometry(cfg, &g);
    if (rc != ACQ_OK) return rc;
    *bytes = workspace_bytes(g, *cfg);
    return ACQ_OK;
}

int acq_bin_frequencies(const acq_config* cfg, double* freqs_hz, int32_t n) {
    if (!freqs_hz) return acq::fail(ACQ_ERR_INVALID_ARG, "null output");
    Geometry g;
    const int rc = acq::derive_geometry(cfg, &g);
    if (rc != ACQ_OK) return rc;
    if (n < cfg->num_bins) return acq::fail(ACQ_ERR_INVALID_ARG, "output shorter than num_bins");
    for (int32_t k = 0; k < cfg->num_bins; ++k) freqs_hz[k] = g.freqs_hz[size_t(k)];
    return ACQ_OK;
}

int acq_plan(const acq_config* cfg, void* workspace, size_t workspace_bytes_, void* stream, acq_plan_t* out) {
    if (!out) return acq::fail(ACQ_ERR_INVALID_ARG, "null output");
    *out = nullptr;
    if (workspace && reinterpret_cast<uintptr_t>(workspace) % kWsAlign != 0)
        return acq::fail(ACQ_ERR_INVALID_ARG, "workspace must be 256-byte aligned");
    Geometry g;
    int rc = acq::derive_geometry(cfg, &g);
    if (rc != ACQ_OK) return rc;
    if (workspace && workspace_bytes_ < workspace_bytes(g, *cfg))
        return acq::fail(ACQ_ERR_WORKSPACE_TOO_SMALL, "workspace of " + std::to_string(workspace_bytes_) +
                                                          " bytes, the plan needs " +
                                                          std::to_string(workspace_bytes(g, *cfg)));
    acq_plan_s* p = new (std::nothrow) acq_plan_s();
    if (!p) return acq::fail(ACQ_ERR_OOM, "host allocation failed");
    p->cfg = *cfg;                   // chips are read by build_plan only
    p->g = std::move(g);
    p->tile = p->g.tag_tile;
    p->stream = static_cast<hipStream_t>(stream);
    if (hipGetDevice(&p->device) != hipSuccess) {
        delete p;
        return acq::fail(ACQ_ERR_DEVICE, "no HIP device");
    }
    int cus = 0;
    if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, p->device) == hipSuccess && cus >= 8)
        p->cus = cus / acq::kXcds * acq::kXcds;
    rc = build_plan(p, workspace, workspace_bytes_);
    p->cfg.chips = nullptr;          // copied to the device; the caller keeps its buffer
    if (rc != ACQ_OK) {
        free_plan(p);
        return rc;
    }
    // the static scratch of acq_detect_noalloc on this device; a failure here
    // only disables that entry point, which then reports it
    if (static_scratch_address(p->device, &p->scratch) != hipSuccess) {
        (void)hipGetLastError();
        p->scratch = nullptr;
    }
    *out = p;
    acq::clear_error();
    return ACQ_OK;
}

int acq_detect(acq_plan_t p, const void* block, int64_t n, acq_detection* out, int32_t capacity,
               int32_t* n_found) {
    int rc = check_block(p, block, n);
    if (rc != ACQ_OK) return rc;
    rc = check_outputs(p, out, capacity, n_found);
    if (rc != ACQ_OK) return rc;
    if (n_found) *n_found = 0;
    if (n < p->g.L) return finish_empty(p, n_found);
    rc = note_capture(p);
    if (rc != ACQ_OK) return rc;
    reset_timers(p);
    BlockTable bt{};
    bt.one = single_desc(p, block, n);
    rc = enqueue_search(p, p->ws, bt, false, bt.one.nseg, nullptr, true, p->stream, false,
                        workspace_dest(p, !async_mode(p)));
    if (rc != ACQ_OK) return rc;
    return finish(p, out, capacity, n_found);
}

int acq_detect_batch(acq_plan_t p, const void* const* blocks, const int64_t* lens, int32_t nblocks,
                     acq_detection* out, int32_t capacity, int32_t* n_found, int32_t* block_of) {
    if (!p) return acq::fail(ACQ_ERR_INVALID_ARG, "null plan");
    if (!blocks || !lens) return acq::fail(ACQ_ERR_INVALID_ARG, "null argument");
    int rc = check_outputs(p, out, capacity, n_found);
    if (rc != ACQ_OK) return rc;
    if (nblocks < 1 || nblocks > p->g.max_blocks)
        return acq::fail(ACQ_ERR_INVALID_ARG, "nblocks outside [1, max_batch_blocks]");
    int64_t total = 0;
    for (int32_t b = 0; b < nblocks; ++b) {
        rc = check_block(p, blocks[b], lens[b]);
        if (rc != ACQ_OK) return rc;
        total += lens[b];
    }
    if (total > p->g.max_batch_samples)
        return acq::fail(ACQ_ERR_BLOCK_TOO_LONG, "batch longer than max_batch_samples");
    if (n_found) *n_found = 0;
    rc = wait_descriptors(p);
    if (rc != ACQ_OK) return rc;
    int32_t seg = 0;
    for (int32_t b = 0; b < nblocks; ++b) {
        BlockDesc d = single_desc(p, blocks[b], lens[b]);
        d.seg0 = seg;
        seg += d.nseg;
        p->h_descs[b] = d;
    }
    p->h_counts[0] = nblocks;
    p->h_counts[1] = seg;
    p->ext_capture = false;
    reset_timers(p);

    rc = launch_batch(p, seg, false);
    if (rc != ACQ_OK) return rc;
    return finish(p, out, capacity, n_found, block_of);
}

int acq_track_batch(acq_plan_t p, const acq_track_task* tasks, int32_t ntasks, acq_detection* out,
                    int32_t capacity, int32_t* n_found) {
    if (!p) return acq::fail(ACQ_ERR_INVALID_ARG, "null plan");
    if (!tasks) return acq::fail(ACQ_ERR_INVALID_ARG, "null argument");
    int rc = check_outputs(p, out, capacity, n_found);
    if (rc != ACQ_OK) return rc;
    if (ntasks < 1 || ntasks > p->g.max_blocks)
        return acq::fail(ACQ_ERR_INVALID_ARG, "ntasks outside [1, max_batch_blocks]");
    int64_t total = 0;
    for (int32_t b = 0; b < ntasks; ++b) {
        rc = check_block(p, tasks[b].block, tasks[b].n);
        if (rc != ACQ_OK) return rc;
        if (tasks[b].tag < 0 || tasks[b].tag >= p->cfg.num_tags)
            return acq::fail(ACQ_ERR_INVALID_ARG, "task tag outside [0, num_tags)");
        total += tasks[b].n;
    }
    if (total > p->g.max_batch_samples)
        return acq::fail(ACQ_ERR_BLOCK_TOO_LONG, "batch longer than max_batch_samples");
    if (n_found) *n_found = 0;
    rc = wait_descriptors(p);
    if (rc != ACQ_OK) return rc;
    const acq_config& c = p->cfg;
    int32_t seg = 0;
    for (int32_t b = 0; b < ntasks; ++b) {
        BlockDesc d = single_desc(p, tasks[b].block, tasks[b].n);
        d.seg0 = seg;
        d.tag = tasks[b].tag;
        // one code is tested: K * (n - L + 1) hypotheses
        d.theta = c.threshold > 0.0 ? c.threshold : acq::default_threshold(1, c.num_bins, tasks[b].n, p->g.L);
        seg += d.nseg;
        p->h_descs[b] = d;
    }
    p->h_counts[0] = ntasks;
    p->h_counts[1] = seg;
    p->ext_capture = false;
    reset_timers(p);
    rc = launch_batch(p, seg, true);
    if (rc != ACQ_OK) return rc;
    return finish(p, out, capacity, n_found);
}

int acq_collect(acq_plan_t p, acq_detection* out, int32_t capacity, int32_t* n_found) {
    if (!p) return acq::fail(ACQ_ERR_INVALID_ARG, "null plan");
    if (!n_found || capacity < 0 || (capacity > 0 && !out))
        return acq::fail(ACQ_ERR_INVALID_ARG, "bad output arguments");
    ACQ_HIP(hipStreamSynchronize(p->stream));
    ACQ_HIP(hipMemcpy(p->h_count, p->ws.count, 2 * sizeof(int32_t), hipMemcpyDeviceToHost));
    const int32_t found = p->h_count[0];
    const int32_t ncopy = std::max(0, std::min(found, capacity));
    if (ncopy > 0) ACQ_HIP(hipMemcpy(p->h_out, p->ws.out, sizeof(acq_detection) * size_t(ncopy), hipMemcpyDeviceToHost));
    return deliver(p, out, capacity, n_found);
}

int acq_detect_noalloc(acq_plan_t p, const void* block, int64_t n, acq_detection* out, int32_t capacity,
                       int32_t* count) {
    int rc = check_block(p, block, n);
    if (rc != ACQ_OK) return rc;
    if (!count || capacity < 0 || (capacity > 0 && !out))
        return acq::fail(ACQ_ERR_INVALID_ARG, "bad output arguments");
    if (!p->scratch) return acq::fail(ACQ_ERR_DEVICE, "the static scratch has no address on this device");
    if (n < p->g.L) {
        ACQ_HIP(acq::launch_fill_i32(count, 1, p->stream));
        acq::clear_error();
        return ACQ_OK;
    }
    BlockTable bt{};
    bt.one = single_desc(p, block, n);
    Scratch w;
    const size_t need = layout_scratch(p->g, p->cfg, 1, bt.one.nseg, 1, nullptr, &w);
    if (need > kStaticScratchBytes)
        return acq::fail(ACQ_ERR_WORKSPACE_TOO_SMALL,
                         "acq_detect_noalloc: a block of " + std::to_string(n) + " samples needs " +
                             std::to_string(need) + " bytes of search memory, the static scratch holds " +
                             std::to_string(kStaticScratchBytes));
    layout_scratch(p->g, p->cfg, 1, bt.one.nseg, 1, static_cast<char*>(p->scratch), &w);
    rc = note_capture(p);
    if (rc != ACQ_OK) return rc;
    reset_timers(p);
    rc = enqueue_search(p, w, bt, false, bt.one.nseg, nullptr, true, p->stream, false,
                        ResultDest{out, capacity, count, false});
    if (rc != ACQ_OK) return rc;
    acq::clear_error();
    return ACQ_OK;
}

int acq_device_results(acq_plan_t p, const acq_detection** records, const int32_t** counts) {
    if (!p || !records || !counts) return acq::fail(ACQ_ERR_INVALID_ARG, "null argument");
    *records = p->ws.out;
    *counts = p->ws.count;
    return ACQ_OK;
}

}  // extern "C"

namespace {

// Proposals of one block (n >= L) written to d_segs; on a fallback the full
// list 0 .. nseg-1 instead.  Fills the report and the searched segment count.
int propose_block(acq_plan_s* p, acq_cnn_t cnn, const void* block, int64_t n, const acq_learned_params* lp,
                  int32_t* d_segs, acq_learned_report* rep, int32_t* nseg_out) {
    double floor = 0.0;
    const bool have_floor = acq::cnn_floor(cnn, &floor);
    rep->floor = float(floor);
    const BlockDesc d = single_desc(p, block, n);
    rep->total_segments = d.nseg;
    acq::ProposalResult pr{};
    const int rc = acq::cnn_propose(cnn, block, n, p->g.L, p->g.V, int32_t(p->g.max_segments), lp->kappa, d_segs,
                                    p->stream, &pr);
    if (rc != ACQ_OK) return rc;
    rep->proposals = pr.proposals;
    rep->median = pr.median;
    rep->fallback = ACQ_FALLBACK_NONE;
    if (double(pr.segments) > double(lp->max_fraction) * double(d.nseg))
        rep->fallback = ACQ_FALLBACK_FRACTION;
    else if (lp->floor_db > 0.0f && have_floor && floor > 0.0 && pr.median > 0.0f &&
             std::fabs(10.0 * std::log10(double(pr.median) / floor)) > double(lp->floor_db))
        rep->fallback = ACQ_FALLBACK_FLOOR;
    acq::cnn_update_floor(cnn, double(pr.median));
    if (rep->fallback == ACQ_FALLBACK_NONE) {
        rep->segments = pr.segments;
    } else {
        rep->segments = d.nseg;
        ACQ_HIP(hipMemcpyAsync(d_segs, p->h_iota, sizeof(int32_t) * size_t(d.nseg), hipMemcpyHostToDevice, p->stream));
    }
    *nseg_out = rep->segments;
    return ACQ_OK;
}

}  // namespace

extern "C" {

int acq_detect_learned(acq_plan_t p, acq_cnn_t cnn, const void* block, int64_t n, const acq_learned_params* lp,
                       acq_detection* out, int32_t capacity, int32_t* n_found, acq_learned_report* report) {
    int rc = check_block(p, block, n);
    if (rc != ACQ_OK) return rc;
    if (!cnn || !lp || !n_found) return acq::fail(ACQ_ERR_INVALID_ARG, "null argument");
    if (capacity < 0 || (capacity > 0 && !out)) return acq::fail(ACQ_ERR_INVALID_ARG, "bad output buffer");
    if (!(lp->max_fraction >= 0.0f)) return acq::fail(ACQ_ERR_INVALID_ARG, "bad proposal parameters");
    *n_found = 0;
    acq_learned_report rep{};
    if (n < p->g.L) {
        double floor = 0.0;
        (void)acq::cnn_floor(cnn, &floor);
        rep.floor = float(floor);
        if (report) *report = rep;
        acq::clear_error();
        return ACQ_OK;
    }
    reset_timers(p);
    BlockTable bt{};
    bt.one = single_desc(p, block, n);
    int32_t nseg = 0;
    rc = propose_block(p, cnn, block, n, lp, p->ws.seglist, &rep, &nseg);
    if (rc != ACQ_OK) return rc;
    if (report) *report = rep;
    if (nseg == 0) {
        acq::clear_error();
        return ACQ_OK;
    }
    bt.one.nseg = nseg;
    bt.seg_of = p->ws.seglist;
    p->ext_capture = false;
    rc = enqueue_search(p, p->ws, bt, false, nseg, nullptr, true, p->stream, false, workspace_dest(p, true));
    if (rc != ACQ_OK) return rc;
    ACQ_HIP(hipStreamSynchronize(p->stream));
    return deliver(p, out, capacity, n_found);
}

int acq_detect_batch_learned(acq_plan_t p, acq_cnn_t cnn, const void* const* blocks, const int64_t* lens,
                             int32_t nblocks, const acq_learned_params* lp, acq_detection* out, int32_t capacity,
                             int32_t* n_found, acq_learned_report* reports) {
    if (!p) return acq::fail(ACQ_ERR_INVALID_ARG, "null plan");
    if (!cnn || !lp || !blocks || !lens || !n_found) return acq::fail(ACQ_ERR_INVALID_ARG, "null argument");
    if (capacity < 0 || (capacity > 0 && !out)) return acq::fail(ACQ_ERR_INVALID_ARG, "bad output buffer");
    if (!(lp->max_fraction >= 0.0f)) return acq::fail(ACQ_ERR_INVALID_ARG, "bad proposal parameters");
    if (nblocks < 1 || nblocks > p->g.max_blocks)
        return acq::fail(ACQ_ERR_INVALID_ARG, "nblocks outside [1, max_batch_blocks]");
    int64_t total = 0;
    for (int32_t b = 0; b < nblocks; ++b) {
        const int rc = check_block(p, blocks[b], lens[b]);
        if (rc != ACQ_OK) return rc;
        total += lens[b];
    }
    if (total > p->g.max_batch_samples)
        return acq::fail(ACQ_ERR_BLOCK_TOO_LONG, "batch longer than max_batch_samples");
    *n_found = 0;
    const int wrc = wait_descriptors(p);
    if (wrc != ACQ_OK) return wrc;
    reset_timers(p);
    int32_t seg = 0;
    for (int32_t b = 0; b < nblocks; ++b) {
        BlockDesc d = single_desc(p, blocks[b], lens[b]);
        acq_learned_report rep{};
        int32_t nseg = 0;
        if (lens[b] >= p->g.L) {
            const int rc = propose_block(p, cnn, blocks[b], lens[b], lp, p->ws.seglist + seg, &rep, &nseg);
            if (rc != ACQ_OK) return rc;
        } else {
            double floor = 0.0;
            (void)acq::cnn_floor(cnn, &floor);
            rep.floor = float(floor);
        }
        if (reports) reports[b] = rep;
        d.seg0 = seg;
        d.nseg = nseg;
        seg += nseg;
        p->h_descs[b] = d;
    }
    if (seg == 0) {
        acq::clear_error();
        return ACQ_OK;
    }
    p->h_counts[0] = nblocks;
    p->h_counts[1] = seg;
    BlockTable bt{};
    bt.descs = p->ws.descs;
    bt.counts = p->ws.counts;
    bt.seg_of = p->ws.seglist;
    ACQ_HIP(hipMemcpyAsync(p->ws.descs, p->h_descs, sizeof(BlockDesc) * size_t(nblocks), hipMemcpyHostToDevice,
                           p->stream));
    ACQ_HIP(hipMemcpyAsync(p->ws.counts, p->h_counts, 2 * sizeof(int32_t), hipMemcpyHostToDevice, p->stream));
    p->ext_capture = false;
    const int rc = enqueue_search(p, p->ws, bt, true, seg, nullptr, true, p->stream, false, workspace_dest(p, true));
    if (rc != ACQ_OK) return rc;
    ACQ_HIP(hipStreamSynchronize(p->stream));
    return deliver(p, out, capacity, n_found);
}

int acq_correlate_power(acq_plan_t p, const void* block, int64_t n, float* power) {
    int rc = check_block(p, block, n);
    if (rc != ACQ_OK) return rc;
    if (n < p->g.L) {
        acq::clear_error();
        return ACQ_OK;
    }
    if (!power) return acq::fail(ACQ_ERR_INVALID_ARG, "null power output");
    reset_timers(p);
    BlockTable bt{};
    bt.one = single_desc(p, block, n);
    rc = note_capture(p);
    if (rc != ACQ_OK) return rc;
    rc = enqueue_search(p, p->ws, bt, false, bt.one.nseg, power, false, p->stream, false, workspace_dest(p, false));
    if (rc != ACQ_OK) return rc;
    ACQ_HIP(hipStreamSynchronize(p->stream));
    acq::clear_error();
    return ACQ_OK;
}

int acq_get_tuning(acq_plan_t p, acq_tuning* out) {
    if (!p || !out) return acq::fail(ACQ_ERR_INVALID_ARG, "null argument");
    out->engine = p->engine;
    out->tag_tile = p->tile;
    out->batch_launch = p->batch_launch;
    out->track_bins = p->track_bins;
    return ACQ_OK;
}

int acq_set_tuning(acq_plan_t p, const acq_tuning* t) {
    if (!p || !t) return acq::fail(ACQ_ERR_INVALID_ARG, "null argument");
    if (t->engine < 0 || t->engine > 1 || t->tag_tile < 1 || t->tag_tile > acq::kMaxTagTile ||
        (t->batch_launch != ACQ_BATCH_GRID && t->batch_launch != ACQ_BATCH_PERSISTENT) || t->track_bins < 0 ||
        t->track_bins > acq::kMaxTagTile)
        return acq::fail(ACQ_ERR_INVALID_ARG,
                         "engine must be 0 or 1, tag_tile in [1, 64], batch_launch 0 or 1, track_bins in [0, 64]");
    const int tile = t->tag_tile < p->cfg.num_tags ? t->tag_tile : p->cfg.num_tags;
    if (t->engine != p->engine || tile != p->tile || t->batch_launch != p->batch_launch ||
        t->track_bins != p->track_bins)
        drop_graph(p);   // the captured kernels change
    p->engine = t->engine;
    p->tile = tile;
    p->batch_launch = t->batch_launch;
    p->track_bins = t->track_bins;
    return ACQ_OK;
}

int acq_tune(acq_plan_t p, const void* block, int64_t n, int32_t reps, acq_tune_entry* out, int32_t capacity,
             int32_t* n_out) {
    int rc = check_block(p, block, n);
    if (rc != ACQ_OK) return rc;
    if (!n_out || reps < 1 || capacity < 0 || (capacity > 0 && !out))
        return acq::fail(ACQ_ERR_INVALID_ARG, "bad arguments");
    if (n < p->g.L) return acq::fail(ACQ_ERR_INVALID_ARG, "block shorter than a template");
    const int was_profiling = p->profile_mode;
    rc = acq_set_profiling(p, ACQ_PROFILE_CORRELATE);          // the tuner times the correlation kernel
    if (rc != ACQ_OK) return rc;
    std::vector<acq_tune_entry> cand;
    const int engines = p->g.log2_sub == 14 ? 2 : 1;
    for (int e = 0; e < engines; ++e)
        for (int tile : {4, 8, 16, 32, 64}) {
            if (tile > p->cfg.num_tags && tile != 4) continue;
            acq_tune_entry c{};
            c.tuning.engine = e;
            c.tuning.tag_tile = tile;
            c.fft_len = int32_t(p->g.M);
            cand.push_back(c);
        }
    const acq_tuning before{p->engine, p->tile, p->batch_launch, p->track_bins};
    BlockTable bt{};
    bt.one = single_desc(p, block, n);
    // the same block repeated as a batch (device descriptor table): as many
    // copies as the plan's batch capacity holds, at most 16
    BlockTable bbt{};
    bbt.descs = p->ws.descs;
    bbt.counts = p->ws.counts;
    const int64_t copies = std::min<int64_t>({int64_t(p->g.max_blocks), p->g.max_batch_samples / n, 16});
    const bool batch_ok = copies >= 1;
    int32_t batch_seg = 0;
    rc = wait_descriptors(p);
    if (rc != ACQ_OK) return rc;
    p->ext_capture = false;
    if (batch_ok) {
        for (int64_t b = 0; b < copies; ++b) {
            p->h_descs[b] = bt.one;
            p->h_descs[b].seg0 = batch_seg;
            batch_seg += bt.one.nseg;
        }
        p->h_counts[0] = int32_t(copies);
        p->h_counts[1] = batch_seg;
        ACQ_HIP(hipMemcpyAsync(p->ws.descs, p->h_descs, sizeof(BlockDesc) * size_t(copies), hipMemcpyHostToDevice,
                               p->stream));
        ACQ_HIP(hipMemcpyAsync(p->ws.counts, p->h_counts, 2 * sizeof(int32_t), hipMemcpyHostToDevice, p->stream));
    }
    auto time_one = [&](const acq_tuning& t, bool batch, double* mean_ms) -> int {
        acq_set_tuning(p, &t);
        double total = 0.0;
        for (int r = 0; r <= reps; ++r) {           // one warm-up run
            reset_timers(p);
            const int rc2 = enqueue_search(p, p->ws, batch ? bbt : bt, batch, batch ? batch_seg : bt.one.nseg, nullptr,
                                           false, p->stream, false, workspace_dest(p, false));
            if (rc2 != ACQ_OK) return rc2;
            ACQ_HIP(hipStreamSynchronize(p->stream));
            float ms = 0.f;
            ACQ_HIP(hipEventElapsedTime(&ms, p->ev[ACQ_KERNEL_CORRELATE][0], p->ev[ACQ_KERNEL_CORRELATE][1]));
            if (r > 0) total += ms;
        }
        *mean_ms = total / reps;
        return ACQ_OK;
    };
    size_t best = 0;
    for (size_t i = 0; i < cand.size() && rc == ACQ_OK; ++i) {
        cand[i].tuning.batch_launch = before.batch_launch;
        cand[i].tuning.track_bins = before.track_bins;
        rc = time_one(cand[i].tuning, false, &cand[i].ms);
        if (cand[i].ms < cand[best].ms) best = i;
    }
    // launch form of batches, with the best engine and tile
    acq_tuning chosen = cand[best].tuning;
    if (rc == ACQ_OK && batch_ok) {
        double best_ms = 0.0;
        for (int form : {ACQ_BATCH_GRID, ACQ_BATCH_PERSISTENT}) {
            acq_tune_entry c{};
            c.tuning = cand[best].tuning;
            c.tuning.batch_launch = form;
            c.fft_len = int32_t(p->g.M);
            rc = time_one(c.tuning, true, &c.ms);
            if (rc != ACQ_OK) break;
            if (form == ACQ_BATCH_GRID || c.ms < best_ms) {
                best_ms = c.ms;
                chosen = c.tuning;
            }
            cand.push_back(c);
        }
    }
    if (rc != ACQ_OK) {
        acq_set_tuning(p, &before);
        acq_set_profiling(p, was_profiling);
        return rc;
    }
    acq_set_tuning(p, &chosen);
    acq_set_profiling(p, was_profiling);
    *n_out = int32_t(cand.size());
    for (size_t i = 0; i < cand.size() && int32_t(i) < capacity; ++i) out[i] = cand[i];
    acq::clear_error();
    return ACQ_OK;
}

int acq_tune_fft_len(const acq_config* cfg, const void* block, int64_t n, int32_t reps, void* stream,
                     acq_tune_entry* out, int32_t capacity, int32_t* n_out, int32_t* best_fft_len) {
    if (!cfg || !n_out || !best_fft_len || reps < 1 || capacity < 0 || (capacity > 0 && !out))
        return acq::fail(ACQ_ERR_INVALID_ARG, "bad arguments");
    acq_config base = *cfg;
    base.fft_len = 0;
    Geometry g0;
    int rc = acq::derive_geometry(&base, &g0);
    if (rc != ACQ_OK) return rc;
    if (n < g0.L) return acq::fail(ACQ_ERR_INVALID_ARG, "block shorter than a template");
    const int64_t spc = cfg->samples_per_chip;
    std::vector<acq_tune_entry> table;
    for (int64_t M = g0.m_min; table.size() < 4 && M / spc <= (int64_t(1) << 14); M *= 2) {
        acq_config c = base;
        c.fft_len = int32_t(M);
        Geometry gm;
        if (acq::derive_geometry(&c, &gm) != ACQ_OK) continue;      // e.g. M / spc below 2^10
        acq_plan_t p = nullptr;
        rc = acq_plan(&c, nullptr, 0, stream, &p);
        if (rc != ACQ_OK) return rc;
        acq_tune_entry e{};
        std::vector<acq_tune_entry> inner(32);
        int32_t ni = 0;
        rc = acq_tune(p, block, n, reps, inner.data(), int32_t(inner.size()), &ni);
        hipEvent_t t0 = nullptr, t1 = nullptr;
        if (rc == ACQ_OK && (hipEventCreate(&t0) != hipSuccess || hipEventCreate(&t1) != hipSuccess))
            rc = acq::fail(ACQ_ERR_DEVICE, "hipEventCreate failed");
        double total = 0.0;
        BlockTable bt{};
        bt.one = single_desc(p, block, n);
        for (int r = 0; r <= reps && rc == ACQ_OK; ++r) {       // one warm-up run
            if (hipEventRecord(t0, p->stream) != hipSuccess) rc = acq::fail(ACQ_ERR_DEVICE, "hipEventRecord");
            if (rc == ACQ_OK)
                rc = enqueue_search(p, p->ws, bt, false, bt.one.nseg, nullptr, true, p->stream, false,
                                    workspace_dest(p, false));
            float ms = 0.f;
            if (rc == ACQ_OK && (hipEventRecord(t1, p->stream) != hipSuccess ||
                                 hipEventSynchronize(t1) != hipSuccess ||
                                 hipEventElapsedTime(&ms, t0, t1) != hipSuccess))
                rc = acq::fail(ACQ_ERR_DEVICE, "timing the search failed");
            if (r > 0) total += ms;
        }
        if (t0) (void)hipEventDestroy(t0);
        if (t1) (void)hipEventDestroy(t1);
        if (rc == ACQ_OK) {
            e.tuning = acq_tuning{p->engine, p->tile, p->batch_launch, p->track_bins};
            e.fft_len = int32_t(M);
            e.ms = total / reps;
            table.push_back(e);
        }
        acq_release(p);
        if (rc != ACQ_OK) return rc;
    }
    if (table.empty()) return acq::fail(ACQ_ERR_UNSUPPORTED, "no segment length available");
    size_t best = 0;
    for (size_t i = 1; i < table.size(); ++i)
        if (table[i].ms < table[best].ms) best = i;
    *best_fft_len = table[best].fft_len;
    *n_out = int32_t(table.size());
    for (size_t i = 0; i < table.size() && int32_t(i) < capacity; ++i) out[i] = table[i];
    acq::clear_error();
    return ACQ_OK;
}

int acq_set_profiling(acq_plan_t p, int on) {
    if (!p) return acq::fail(ACQ_ERR_INVALID_ARG, "null plan");
    if (on < ACQ_PROFILE_OFF || on > ACQ_PROFILE_CORRELATE)
        return acq::fail(ACQ_ERR_INVALID_ARG, "profiling mode must be ACQ_PROFILE_OFF, _ALL or _CORRELATE");
    if (on && !p->ev[0][0]) {
        for (auto& pair : p->ev)
            for (hipEvent_t& e : pair) ACQ_HIP(hipEventCreate(&e));
    }
    p->profiling = on != ACQ_PROFILE_OFF;
    p->profile_mode = on;
    p->profile_mask = on == ACQ_PROFILE_ALL ? (1u << ACQ_NUM_KERNELS) - 1u
                      : on == ACQ_PROFILE_CORRELATE ? 1u << ACQ_KERNEL_CORRELATE : 0u;
    reset_timers(p);
    acq::clear_error();
    return ACQ_OK;
}

int acq_last_kernel_times(acq_plan_t p, double* ms, int32_t n, int32_t* count) {
    if (!p || !count || (n > 0 && !ms)) return acq::fail(ACQ_ERR_INVALID_ARG, "bad arguments");
    *count = ACQ_NUM_KERNELS;
    ACQ_HIP(hipStreamSynchronize(p->stream));
    for (int i = 0; i < n && i < ACQ_NUM_KERNELS; ++i) {
        float t = 0.f;
        if (p->profiling && p->ev_used[i]) ACQ_HIP(hipEventElapsedTime(&t, p->ev[i][0], p->ev[i][1]));
        ms[i] = double(t);
    }
    return ACQ_OK;
}

int acq_release(acq_plan_t p) {
    if (!p) return ACQ_OK;
    (void)hipStreamSynchronize(p->stream);
    free_plan(p);
    return ACQ_OK;
}

const char* acq_strerror(int status) {
    switch (status) {
        case ACQ_OK: return "ok";
        case ACQ_ERR_INVALID_ARG: return "invalid argument";
        case ACQ_ERR_OOM: return "out of memory";
        case ACQ_ERR_DEVICE: return "device error";
        case ACQ_ERR_TRUNCATED: return "output truncated";
        case ACQ_ERR_BLOCK_TOO_LONG: return "block too long";
        case ACQ_ERR_WORKSPACE_TOO_SMALL: return "workspace too small";
        case ACQ_ERR_UNSUPPORTED: return "unsupported";
        case ACQ_ERR_NON_FINITE: return "non-finite samples";
        default: return "unknown status";
    }
}

const char* acq_last_error(void) { return acq::last_error(); }

}  // extern "C"
