// Execution of a recorded batch: the launches of all members are merged into
// grouped launches, one per (pipeline place, kernel), in pipeline order.
//
// Each member's launches carry increasing keys (stage, iteration, position;
// launch.h).  Sorting all records by key and grouping equal (key, kernel)
// pairs gives a sequence of grouped launches in which every member's own
// launches keep their order, while members never depend on each other.  A
// grouped launch covers the work-groups of all its members (a few thousand
// for the big products), so the machine stays full even where a single
// member's step is small (QR panels, triangular blocks, solves).
//
// The group tables (first work-group, grid width and arguments per member)
// are built on the host and copied once into the caller's workspace; the
// launches are then enqueued back to back on the stream, as often as a plan
// is executed (kernel launches only: capturable into a hipGraph).
#include <algorithm>
#include <vector>

#include "common.h"
#include "kernels.h"
#include "launch.h"
#include "profile.h"
#include "tune.h"

namespace pne {

namespace {

// Profile phase that ends with a stage (see profile.h).
int stage_phase(uint32_t st)
{
    switch (st) {
    case ST_INIT: return PH_START;
    case ST_CONDEST_GRAM: case ST_CONDEST_FACTOR: case ST_CONDEST_INV: case ST_CONDEST_EST: return PH_CONDEST;
    case ST_SKETCH: return PH_SK_GEMM;
    case ST_SKETCH_REDUCE: return PH_SK_REDUCE;
    case ST_QR_ROUND: case ST_QR: case ST_QR_EXTRACT: return PH_QR;
    case ST_TRSM: return PH_TRSM;
    case ST_GRAM: return PH_GRAM_GEMM;
    case ST_GRAM_REDUCE: return PH_GRAM_REDUCE;
    case ST_FACTOR: case ST_FACTOR_INV: return PH_FACTOR;
    case ST_SOLVE: return PH_SOLVE;
    default: return PH_REFINE;
    }
}

}  // namespace

int build_groups(const Recorder& rec, GroupSeq* out)
{
    const std::vector<LaunchRec>& R = rec.recs;
    std::vector<uint32_t> idx(R.size());
    for (size_t i = 0; i < idx.size(); ++i) idx[i] = (uint32_t)i;
    std::stable_sort(idx.begin(), idx.end(), [&](uint32_t a, uint32_t b) {
        if (R[a].key != R[b].key) return R[a].key < R[b].key;
        if (R[a].fn != R[b].fn) return (uintptr_t)R[a].fn < (uintptr_t)R[b].fn;
        return R[a].member < R[b].member;
    });
    std::vector<char>& blob = out->blob;
    std::vector<LaunchGroup>& groups = out->groups;
    blob.clear();
    groups.clear();
    size_t i = 0;
    while (i < idx.size()) {
        size_t j = i + 1;
        const LaunchRec& r0 = R[idx[i]];
        while (j < idx.size() && R[idx[j]].key == r0.key && R[idx[j]].fn == r0.fn) ++j;
        const int count = (int)(j - i);
        const size_t off = (blob.size() + 255) & ~(size_t)255;
        const size_t aoff = (size_t)group_args_offset(count);
        // arguments, then the two work counters of a persistent launch (zero)
        blob.resize(off + (size_t)group_counter_offset(count, r0.args_size) + GROUP_COUNTER_BYTES, 0);
        int32_t* start = (int32_t*)(blob.data() + off);
        int32_t* gx = start + count + 1;
        int64_t total = 0;
        for (int k = 0; k < count; ++k) {
            const LaunchRec& r = R[idx[i + k]];
            if (r.args_size != r0.args_size) return PNE_EINVAL;
            start[k] = (int32_t)total;
            gx[k] = r.gx;
            total += (int64_t)r.gx * r.gy;
            memcpy(blob.data() + off + aoff + (size_t)k * r0.args_size, rec.pool.data() + r.args_off, r.args_size);
        }
        if (total >= ((int64_t)1 << 31)) return PNE_ENOTSUP;
        start[count] = (int32_t)total;
        groups.push_back(LaunchGroup{r0.fn, off, count, total, (uint32_t)(r0.key >> 56)});
        i = j;
    }
    return PNE_OK;
}

void enqueue_groups(const std::vector<LaunchGroup>& groups, const char* dtables, hipStream_t st, bool marks)
{
    const int persistent = tune_params().persistent;
    for (size_t g = 0; g < groups.size(); ++g) {
        const LaunchGroup& G = groups[g];
        G.fn(dtables + G.off, G.count, G.total, st, persistent);
        if (!marks) continue;
        const bool last = g + 1 == groups.size();
        if (last || stage_phase(groups[g + 1].stage) != stage_phase(G.stage)) prof_mark(stage_phase(G.stage), st);
    }
}

int run_recorded(const Recorder& rec, char* dtables, size_t cap, hipStream_t st)
{
    GroupSeq seq;
    int rc = build_groups(rec, &seq);
    if (rc) return rc;
    if (seq.blob.empty()) return PNE_OK;
    if (seq.blob.size() > cap || !dtables) return PNE_EWORKSPACE;
    // the host blob is released on return: wait for the copy
    HIP_OK(hipMemcpyAsync(dtables, seq.blob.data(), seq.blob.size(), hipMemcpyHostToDevice, st));
    HIP_OK(hipStreamSynchronize(st));
    enqueue_groups(seq.groups, dtables, st, true);
    return hipGetLastError() == hipSuccess ? PNE_OK : PNE_EHIP;
}

}  // namespace pne
