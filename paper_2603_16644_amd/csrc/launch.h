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

#include <type_traits>
#include <vector>

#include "common.h"

namespace pne {

// byte offset of the argument array in a group table of `count` members
__host__ __device__ inline int64_t group_args_offset(int count)
{
    return ((int64_t)(2 * count + 1) * 4 + 15) & ~(int64_t)15;
}

// byte offset of the two work counters after the arguments (next work
// item, work-groups finished; used by persistent launches, zero otherwise)
__host__ __device__ inline int64_t group_counter_offset(int count, int64_t args_size)
{
    return (group_args_offset(count) + (int64_t)count * args_size + 15) & ~(int64_t)15;
}
constexpr int64_t GROUP_COUNTER_BYTES = 16;

// Locate work-group b's member in a group table and run its share.
template <class K>
__device__ __forceinline__ void grouped_item(const char* __restrict__ table, int count, int32_t b)
{
    const int32_t* start = (const int32_t*)table;
    const int32_t* gx = start + count + 1;
    const typename K::Args* args = (const typename K::Args*)(table + group_args_offset(count));
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
template <class K>
__device__ __forceinline__ void grouped_body(const char* __restrict__ table, int count)
{
    grouped_item<K>(table, count, (int32_t)blockIdx.x);
}

// Persistent form of a grouped launch: as many work-groups as fit on the
// machine at once, each taking work items (the work-groups of the ordinary
// launch, in order) from the table's counter until they run out.  The last
// work-group to finish puts the counters back to zero, so the table serves
// the next launch, or the next replay of a captured graph, as it is.  Every
// item computes what the ordinary launch's work-group does, in the same
// order, so results are bitwise the same.  For kernels without an early
// return (every thread reaches every barrier of K::run).
template <class K>
__device__ __forceinline__ void persistent_body(const char* __restrict__ table, int count, int32_t total)
{
    int32_t* ctr = (int32_t*)(const_cast<char*>(table) + group_counter_offset(count, sizeof(typename K::Args)));
    __shared__ int32_t item;
    for (;;) {
        if (threadIdx.x == 0) item = __hip_atomic_fetch_add(&ctr[0], 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        __syncthreads();
        const int32_t it = item;
        __syncthreads();
        if (it >= total) break;
        grouped_item<K>(table, count, it);
    }
    if (threadIdx.x == 0) {
        const int32_t done = __hip_atomic_fetch_add(&ctr[1], 1, __ATOMIC_ACQ_REL, __HIP_MEMORY_SCOPE_AGENT);
        if (done == (int32_t)gridDim.x - 1) {
            __hip_atomic_store(&ctr[0], 0, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            __hip_atomic_store(&ctr[1], 0, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
        }
    }
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

template <class K>
__global__ __launch_bounds__(K::NTH) __attribute__((amdgpu_waves_per_eu(K::WPE, K::WPE)))
void persistent_kernel_wpe(const char* __restrict__ table, int count, int32_t total)
{
    persistent_body<K>(table, count, total);
}

// Kernels that may run persistent declare `static constexpr bool PERSIST`.
template <class K, class = void>
struct can_persist : std::false_type {};
template <class K>
struct can_persist<K, std::void_t<decltype(K::PERSIST)>> : std::integral_constant<bool, K::PERSIST> {};

// Work-groups of K that fit on the device at once (queried once per kernel).
template <class K>
int64_t persistent_grid()
{
    static int64_t g = [] {
        int dev = 0, cus = 0, per_cu = 0;
        (void)hipGetDevice(&dev);
        (void)hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
        (void)hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, persistent_kernel_wpe<K>, K::NTH, 0);
        return (int64_t)(cus > 0 ? cus : 1) * (per_cu > 0 ? per_cu : 1);
    }();
    return g;
}

typedef void (*GroupLaunchFn)(const char* dtable, int count, int64_t total_wgs, hipStream_t st, int persistent);

template <class K>
void group_launch(const char* dtable, int count, int64_t total_wgs, hipStream_t st, int persistent)
{
    if constexpr (K::WPE > 0 && can_persist<K>::value) {
        const int64_t g = persistent ? persistent_grid<K>() : 0;
        if (g > 0 && g < total_wgs) {
            persistent_kernel_wpe<K><<<dim3((uint32_t)g), K::NTH, 0, st>>>(dtable, count, (int32_t)total_wgs);
            return;
        }
    }
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
