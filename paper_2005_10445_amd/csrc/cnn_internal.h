// Interface between the proposal network (cnn.hip) and the search plan
// (plan.hip) for acq_detect_learned.
#pragma once

#include <hip/hip_runtime.h>
#include <cstdint>

#include "acq.h"

namespace acq {

struct ProposalResult {
    int32_t proposals;          // frames proposed
    int32_t segments;           // segments listed in d_segs
    float median;               // power-map median of the block
};

// Power map, network, window scores and proposals of one device block on
// stream st; the proposed segments (ascending) go to device d_segs.  Waits for
// the stream.  Returns an ACQ status.
int cnn_propose(acq_cnn_t cnn, const void* block, int64_t n, int64_t L, int64_t V, int32_t max_segments,
                float kappa, int32_t* d_segs, hipStream_t st, ProposalResult* out);

// Running noise floor of the network's blocks: false until the first update.
bool cnn_floor(acq_cnn_t cnn, double* floor);
void cnn_update_floor(acq_cnn_t cnn, double median);

}  // namespace acq
