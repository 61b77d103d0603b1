// Tunable launch parameters and their cache (tune.hip).
//
// The planners read the parameters of the calling thread (TuneScope sets
// them for the duration of an entry point); the defaults are the fixed rules
// the library uses without a cache.  The autotuner (pne_autotune_batched)
// times candidate settings on the caller's batch and stores the fastest
// under a key of the workload in a JSON file named by $PNE_TUNE_CACHE;
// later calls with the same key read it back.
#pragma once
#include <stdint.h>

#include <string>

namespace pne {

struct TuneParams {
    int64_t batch_kchunk = 8192;   // rows per split-K chunk of the long products of a batch
    int shortk_tile = 64;          // output tile (64 or 128) of products with K < 4096
    int lower_small_n = 512;       // lower-triangle long-K products of order <= this use 64 x 64 tiles
    int persistent = 0;            // 1: grouped MFMA products as persistent launches (launch.h)
};

// Parameters in force on this thread.
const TuneParams& tune_params();

// Sets this thread's parameters until the scope ends.
struct TuneScope {
    explicit TuneScope(const TuneParams& p);
    ~TuneScope();
    TuneParams saved;
};

// Cache key of a batched workload: solver, precisions, and power-of-two
// buckets of the member count, the mean n and the mean m.
std::string tune_key_batched(int hpne, int sketch_prec, int qr_prec, int64_t batch, double mean_n, double mean_m);
// Parameters stored under `key` in $PNE_TUNE_CACHE (false: no file, no entry).
bool tune_lookup(const std::string& key, TuneParams* out);
// Store (or replace) the entry of `key`; returns false if the file cannot be written.
bool tune_store(const std::string& key, const TuneParams& p, double ms);

}  // namespace pne
