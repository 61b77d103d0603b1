// Phase marks of the solve pipeline (see profile.hip).
#pragma once
#include <hip/hip_runtime.h>

namespace pne {

enum {
    PH_START = 0, PH_CONDEST, PH_SK_OMEGA, PH_SK_QUANT, PH_SK_GEMM, PH_SK_REDUCE, PH_QR, PH_TRSM,
    PH_GRAM_GEMM, PH_GRAM_REDUCE, PH_FACTOR, PH_SOLVE, PH_REFINE, PH_COUNT
};
void prof_mark(int phase, hipStream_t st);
void prof_reset();

}  // namespace pne
