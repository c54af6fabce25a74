// Device tables of the batched launch (internal).
#pragma once

#include "kernels.h"

namespace divas {

struct BatchHeader {
    int32_t n_items, n_vjobs, n_cjobs, chunks_per_wave;
    int64_t total_rows, total_cull, total_chunks;
    // persistent schedule: descriptors in the queue and its head (zero in
    // every run's copy of the header; one integer atomic per pop)
    uint32_t n_desc, head;
};

// A descriptor of the persistent schedule: chunks [c0, c1) of one item.
struct BDesc {
    int32_t item;
    uint32_t c0, c1;
    int32_t pad;
};

// One item: a session's fusion (all its views, or one new view folded in or
// re-fused), with its outputs.
struct BItem {
    FuseArgs f;
    const ChunkBox* box;   // chunk boxes of the session
    DView* views_rw;       // the session's device view records
    uint64_t* cull_rw;     // the session's cull bits
    double gate;           // mask gate of the hot tiles
    uint64_t fuse_range;   // views fused by this item
};

struct BViewJob {
    int32_t item, slot;
};

struct BCullJob {
    int32_t item, s_begin, ns, p2;  // views [s_begin, s_begin + ns) of the item, p2 lanes per chunk
};

struct BatchTables {
    const BatchHeader* header;
    const BItem* items;
    const int64_t* item_chunk_base;  // [n_items + 1] first chunk of each item in the flattened chunk space
    const BCullJob* cjobs;
    const int64_t* cjob_lane_base;   // [n_cjobs] first cull lane of each job (multiple of 64)
    const BViewJob* vjobs;
    const int64_t* vjob_row_base;    // [n_vjobs] first tile row of each new view
    const DView* vrecs;              // [n_vjobs] new view records
    const BDesc* desc;               // [n_desc] descriptors of the persistent schedule, costliest items first
    uint32_t* head;                  // the queue head (inside the device copy of the header)
};

struct BatchGrid {
    unsigned prep_blocks, cull_blocks;
    unsigned fuse_blocks, fuse_threads;  // one wavefront per flattened chunk (at least total_chunks waves),
                                         // or the persistent grid
    int mode;                            // FuseMode of the fusion kernel (kThick, kAnyMode or kAnyThin)
    bool persistent;                     // waves pull descriptors from the queue
};

hipError_t launch_batch(const BatchTables& t, const BatchGrid& g, hipStream_t st);
// one of the launches: 0 = prep (records, hot tiles, gate bitmask), 1 = cull, 2 = fusion, 3 = counts
hipError_t launch_batch_phase(const BatchTables& t, const BatchGrid& g, int phase, hipStream_t st);
constexpr int kBatchPhases = 4;

}  // namespace divas
