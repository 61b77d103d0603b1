// Phase timing: when enabled, the solvers record a HIP event on their stream
// after each phase; pne_profile_read waits for the last recorded events and
// returns the time between consecutive marks.  Off by default; recording
// never synchronises the stream.
#include <string.h>

#include <vector>

#include "common.h"
#include "profile.h"

namespace pne {

// Every mark records one event of a pool in order; the time between a mark
// and the previous one is charged to the later mark's phase, so a phase that
// recurs (the chunks of a long sketch) accumulates its pieces.
static bool g_prof_on = false;
static std::vector<hipEvent_t> g_pool;
static std::vector<int> g_phase;   // phase of each recorded event, in order

void prof_mark(int phase, hipStream_t st)
{
    if (!g_prof_on || phase < 0 || phase >= PH_COUNT) return;
    const size_t k = g_phase.size();
    if (k == g_pool.size()) {
        hipEvent_t e;
        if (hipEventCreate(&e) != hipSuccess) return;
        g_pool.push_back(e);
    }
    if (hipEventRecord(g_pool[k], st) == hipSuccess) g_phase.push_back(phase);
}

void prof_reset() { g_phase.clear(); }

}  // namespace pne

using namespace pne;

extern "C" {

static const char* k_phase_names[PH_COUNT] = {
    "start", "cond_est", "sketch_omega", "sketch_quantize", "sketch_gemm", "sketch_reduce", "qr",
    "trsm", "gram_gemm", "gram_reduce", "factor", "solve", "refine"};

int pne_profile_enable(int enable)
{
    g_prof_on = enable != 0;
    prof_reset();
    return PNE_OK;
}

const char* pne_profile_phase_name(int i) { return (i >= 0 && i < PH_COUNT) ? k_phase_names[i] : ""; }

int pne_profile_read(double* ms, int max_phases)
{
    const int count = max_phases < PH_COUNT ? max_phases : PH_COUNT;
    for (int i = 0; i < count; ++i) ms[i] = -1.0;
    if (g_phase.empty()) return g_prof_on ? count : 0;
    if (hipEventSynchronize(g_pool[g_phase.size() - 1]) != hipSuccess) return PNE_EHIP;
    for (size_t k = 1; k < g_phase.size(); ++k) {
        const int ph = g_phase[k];
        if (ph >= count) continue;
        float t = 0.0f;
        if (hipEventElapsedTime(&t, g_pool[k - 1], g_pool[k]) != hipSuccess) return PNE_EHIP;
        ms[ph] = (ms[ph] < 0.0 ? 0.0 : ms[ph]) + t;
    }
    return count;
}

}  // extern "C"
