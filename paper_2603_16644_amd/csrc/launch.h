// Launch layer shared by the single-problem and the batched solvers.
//
// Every kernel of the path is a struct K with
//   typedef/struct Args;                    trivially copyable arguments
//   static constexpr int NTH, WPE;          threads per work-group, waves per
//                                           SIMD to budget registers for (0:
//                                           compiler default)
//   static __device__ void run(const Args&, int bx, int by);
// and runs in one of two ways:
//   direct:  one launch of a gx x gy grid for one problem;
//   grouped: one launch for many problems of a batch.  The work-groups of
//            all members are numbered consecutively; a table in device
//            memory holds the first work-group of every member, its grid
//            width and its arguments, and each work-group finds its member
//            by binary search.
// Host drivers issue kernels through launch<K>(ex, gx, gy, args).  With
// ex.rec == nullptr the kernel is launched at once on ex.st; otherwise the
// launch is recorded under a key (stage, iteration, position) so that
// the batched driver can merge the i-th launch of every member into one
// grouped launch (see batched.hip).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>
#include <string.h>

#include <vector>

#include "common.h"

namespace pne {

// byte offset of the argument array in a group table of `count` members
__host__ __device__ inline int64_t group_args_offset(int count)
{
    return ((int64_t)(2 * count + 1) * 4 + 15) & ~(int64_t)15;
}

// Locate this work-group's member in a group table and run its share.
template <class K>
__device__ __forceinline__ void grouped_body(const char* __restrict__ table, int count)
{
    const int32_t* start = (const int32_t*)table;
    const int32_t* gx = start + count + 1;
    const typename K::Args* args = (const typename K::Args*)(table + group_args_offset(count));
    const int32_t b = (int32_t)blockIdx.x;
    int lo = 0, hi = count - 1;
    while (lo < hi) {  // last member whose first work-group is <= b
        const int mid = (lo + hi + 1) >> 1;
        if (start[mid] <= b) lo = mid;
        else hi = mid - 1;
    }
    const int32_t local = b - start[lo];
    const int32_t w = gx[lo];
    const typename K::Args a = args[lo];
    K::run(a, local % w, local / w);
}

// Kernels with K::WPE > 0 carry an occupancy target of WPE waves per SIMD
// (register budget); the others use the compiler's default.
template <class K>
__global__ __launch_bounds__(K::NTH) void direct_kernel(const typename K::Args a)
{
    K::run(a, blockIdx.x, blockIdx.y);
}
template <class K>
__global__ __launch_bounds__(K::NTH) __attribute__((amdgpu_waves_per_eu(K::WPE, K::WPE)))
void direct_kernel_wpe(const typename K::Args a)
{
    K::run(a, blockIdx.x, blockIdx.y);
}
template <class K>
__global__ __launch_bounds__(K::NTH) void grouped_kernel(const char* __restrict__ table, int count)
{
    grouped_body<K>(table, count);
}
template <class K>
__global__ __launch_bounds__(K::NTH) __attribute__((amdgpu_waves_per_eu(K::WPE, K::WPE)))
void grouped_kernel_wpe(const char* __restrict__ table, int count)
{
    grouped_body<K>(table, count);
}

typedef void (*GroupLaunchFn)(const char* dtable, int count, int64_t total_wgs, hipStream_t st);

template <class K>
void group_launch(const char* dtable, int count, int64_t total_wgs, hipStream_t st)
{
    if constexpr (K::WPE > 0) grouped_kernel_wpe<K><<<dim3((uint32_t)total_wgs), K::NTH, 0, st>>>(dtable, count);
    else grouped_kernel<K><<<dim3((uint32_t)total_wgs), K::NTH, 0, st>>>(dtable, count);
}

struct LaunchRec {
    uint64_t key;        // stage, iteration, position (Exec::next_key)
    GroupLaunchFn fn;    // identifies the kernel
    int32_t member;
    int32_t gx, gy;
    uint32_t args_size;
    size_t args_off;     // into Recorder::pool
};

struct Recorder {
    std::vector<LaunchRec> recs;
    std::vector<char> pool;
};

// Stages of the pipeline, in execution order (the major part of a launch
// key).  Within a stage, loop drivers number their iterations (iter) and the
// launches of one iteration are counted (sub), so a key names the same place
// of the pipeline in every member of a batch.
enum Stage : uint32_t {
    ST_INIT = 1, ST_CONDEST_GRAM, ST_CONDEST_FACTOR, ST_CONDEST_INV, ST_CONDEST_EST,
    ST_SKETCH, ST_SKETCH_REDUCE, ST_QR_ROUND, ST_QR, ST_QR_EXTRACT, ST_TRSM, ST_GRAM, ST_GRAM_REDUCE,
    ST_FACTOR, ST_FACTOR_INV, ST_SOLVE, ST_REFINE, ST_FINISH
};

// Where launches go, plus the planning knobs that differ between one large
// problem (fill the machine with one product) and a batch (many products
// side by side).
struct Exec {
    hipStream_t st = nullptr;
    Recorder* rec = nullptr;
    int32_t member = 0;
    uint32_t stage_ = 0, iter_ = 0, sub = 0;
    // > 0: split long-K products into chunks of this many rows instead of
    // planning the split count to fill the machine with one product
    int64_t kchunk_fixed = 0;
    void stage(uint32_t s)
    {
        stage_ = s;
        iter_ = 0;
        sub = 0;
    }
    void iter(uint32_t i)
    {
        iter_ = i;
        sub = 0;
    }
    uint64_t next_key() { return ((uint64_t)stage_ << 56) | ((uint64_t)(iter_ & 0xffffff) << 32) | (sub++ & 0xffffffffu); }
    bool recording() const { return rec != nullptr; }
};

// Status of the launches issued so far: a recording touches no device.
inline int launch_status(const Exec& ex)
{
    if (ex.recording()) return PNE_OK;
    return hipGetLastError() == hipSuccess ? PNE_OK : PNE_EHIP;
}

template <class K>
inline void launch(Exec& ex, int64_t gx, int64_t gy, const typename K::Args& a)
{
    if (gx <= 0 || gy <= 0) return;
    if (!ex.rec) {
        const dim3 grid((uint32_t)gx, (uint32_t)gy);
        if constexpr (K::WPE > 0) direct_kernel_wpe<K><<<grid, K::NTH, 0, ex.st>>>(a);
        else direct_kernel<K><<<grid, K::NTH, 0, ex.st>>>(a);
        return;
    }
    LaunchRec r;
    r.key = ex.next_key();
    r.fn = &group_launch<K>;
    r.member = ex.member;
    r.gx = (int32_t)gx;
    r.gy = (int32_t)gy;
    r.args_size = (uint32_t)sizeof(a);
    r.args_off = ex.rec->pool.size();
    ex.rec->pool.resize(r.args_off + sizeof(a));
    memcpy(ex.rec->pool.data() + r.args_off, &a, sizeof(a));
    ex.rec->recs.push_back(r);
}

}  // namespace pne
