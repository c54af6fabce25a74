// Tables of the multi-target fusion (internal): several target objects of one
// scene fused in one launch sequence (targets.hip).
#pragma once

#include "kernels.h"

namespace divas {

constexpr int kMaxTargets = 8;

// Cull of every target's view bits, the chunk rectangle shared: views[t] are
// target t's view records (same cameras, own hot tiles), cull[t] its words.
struct TargetCull {
    const ChunkBox* box;
    const int64_t* n_act;
    double eps;
    int32_t n, s_begin, ns;
    const DView* views[kMaxTargets];
    uint64_t* cull[kMaxTargets];
};

// One fusion per target over the shared active list: f[t] as a single-target
// fusion of target t (act, n_act, cap, grid and parameters equal for all t).
struct TargetArgs {
    int32_t n;
    FuseArgs f[kMaxTargets];
};

hipError_t launch_cull_targets(const TargetCull& tc, int64_t cap, hipStream_t st);
// fusion of every chunk for the n_targets targets of the device table ta_dev,
// then every target's count reduction
hipError_t launch_fuse_targets(const TargetArgs* ta_dev, int n_targets, int64_t cap, bool any_nsamp,
                               hipStream_t st);

}  // namespace divas
