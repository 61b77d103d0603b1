// Phase timing: when enabled, the solvers record a HIP event on their stream
// after each phase; pne_profile_read waits for the last recorded events and
// returns the time between consecutive marks.  Off by default; recording
// never synchronises the stream.
#include <string.h>

#include "common.h"
#include "profile.h"

namespace pne {

static bool g_prof_on = false;
static bool g_prof_ready = false;
static hipEvent_t g_ev[PH_COUNT];
static bool g_marked[PH_COUNT];

void prof_mark(int phase, hipStream_t st)
{
    if (!g_prof_on || phase < 0 || phase >= PH_COUNT) return;
    if (hipEventRecord(g_ev[phase], st) == hipSuccess) g_marked[phase] = true;
}

void prof_reset()
{
    for (int i = 0; i < PH_COUNT; ++i) g_marked[i] = false;
}

}  // namespace pne

using namespace pne;

extern "C" {

static const char* k_phase_names[PH_COUNT] = {
    "start", "cond_est", "sketch_omega", "sketch_quantize", "sketch_gemm", "sketch_reduce", "qr",
    "trsm", "gram_gemm", "gram_reduce", "factor", "solve", "refine"};

int pne_profile_enable(int enable)
{
    if (enable && !g_prof_ready) {
        for (int i = 0; i < PH_COUNT; ++i)
            if (hipEventCreate(&g_ev[i]) != hipSuccess) return PNE_EHIP;
        g_prof_ready = true;
    }
    g_prof_on = enable != 0 && g_prof_ready;
    prof_reset();
    return PNE_OK;
}

const char* pne_profile_phase_name(int i) { return (i >= 0 && i < PH_COUNT) ? k_phase_names[i] : ""; }

int pne_profile_read(double* ms, int max_phases)
{
    if (!g_prof_ready) return 0;
    int count = max_phases < PH_COUNT ? max_phases : PH_COUNT;
    for (int i = 0; i < count; ++i) ms[i] = -1.0;
    int prev = -1;
    for (int i = 0; i < PH_COUNT; ++i) {
        if (!g_marked[i]) continue;
        if (hipEventSynchronize(g_ev[i]) != hipSuccess) return PNE_EHIP;
        if (prev >= 0 && i < count) {
            float t = 0.0f;
            if (hipEventElapsedTime(&t, g_ev[prev], g_ev[i]) == hipSuccess) ms[i] = t;
        }
        prev = i;
    }
    return count;
}

}  // extern "C"
