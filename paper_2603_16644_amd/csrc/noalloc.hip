// pne_solve_noalloc: the PNE/HPNE solve for callers that cannot allocate
// device memory (code under stream capture, tight serving loops, harnesses
// that forbid hipMalloc).  The solve's scratch lives in one file-scope device
// array of PNE_NOALLOC_MAX_BYTES per GPU instead of a caller workspace; the
// kernels and the launch sequence are those of pne_solve / hpne_solve.
#include <mutex>

#include "common.h"
#include "kernels.h"


namespace {

// One copy per GPU, held until the process ends.  In host code the name
// `scratch` is only a host-side stand-in: the kernels receive the device
// address looked up per device below, never this symbol.
__device__ __align__(256) unsigned char scratch[PNE_NOALLOC_MAX_BYTES];

constexpr int kMaxDevices = 64;
std::mutex g_mu;
void* g_ptr[kMaxDevices];   // device address of `scratch` on device d (null until looked up)

// Address of the current device's scratch array (looked up once per device,
// with that device current).  Returns null on a HIP error.
void* scratch_address(int* dev_out)
{
    int dev = -1;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= kMaxDevices) return nullptr;
    *dev_out = dev;
    std::lock_guard<std::mutex> lk(g_mu);
    if (!g_ptr[dev]) {
        void* p = nullptr;
        if (hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) != hipSuccess || !p) return nullptr;
        g_ptr[dev] = p;
    }
    return g_ptr[dev];
}

}  // namespace

extern "C" {

size_t pne_noalloc_max_bytes(void) { return PNE_NOALLOC_MAX_BYTES; }

pne_status pne_solve_noalloc(int64_t m, int64_t n, const double* dA, int64_t lda, const double* db, double* dx,
                             const pne_opts* o, int hpne, int32_t* dinfo, pne_info* hinfo, pne_stream_t stream)
{
    if (hpne != 0 && hpne != 1) return PNE_EINVAL;
    // size check on the host before any HIP call: a problem whose workspace
    // exceeds the array is rejected with nothing enqueued
    size_t need = 0;
    pne_status chk = pne::solve_workspace(hpne, m, n, lda, o, &need);
    if (chk) return chk;
    if (need > (size_t)PNE_NOALLOC_MAX_BYTES) return PNE_EWORKSPACE;
    if (!dA || !db || !dx || !dinfo) return PNE_EINVAL;
    int dev = -1;
    void* ptr = scratch_address(&dev);
    if (!ptr) return PNE_EHIP;
    return pne::solve_entry(hpne, m, n, dA, lda, db, dx, o, ptr, (size_t)PNE_NOALLOC_MAX_BYTES, dinfo, hinfo,
                            (hipStream_t)stream);
}

}  // extern "C"
