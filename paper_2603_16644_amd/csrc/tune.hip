// Tunable launch parameters: per-thread scope and the JSON cache file.
//
// Cache format ($PNE_TUNE_CACHE): one JSON object whose members are
//   "<key>": {"batch_kchunk": K, "shortk_tile": T, "lower_small_n": L, "persistent": P, "ms": t}
// written by this file only; the reader accepts exactly that shape (any
// whitespace).  Reads go through an in-memory copy refreshed when the file's
// modification time or size changes.
#include <math.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>
#include <sys/stat.h>

#include <map>
#include <mutex>
#include <string>

#include "tune.h"

namespace pne {

namespace {

thread_local TuneParams t_params;

struct Entry {
    TuneParams p;
    double ms;
};

std::mutex g_mu;
std::map<std::string, Entry> g_cache;
std::string g_path;
long long g_mtime = -1, g_size = -1;

const char* cache_path() { return getenv("PNE_TUNE_CACHE"); }

void skip_ws(const char*& s)
{
    while (*s == ' ' || *s == '\n' || *s == '\t' || *s == '\r') ++s;
}

bool parse_string(const char*& s, std::string* out)
{
    skip_ws(s);
    if (*s != '"') return false;
    ++s;
    const char* b = s;
    while (*s && *s != '"') ++s;
    if (*s != '"') return false;
    out->assign(b, s - b);
    ++s;
    return true;
}

bool parse_number(const char*& s, double* v)
{
    skip_ws(s);
    char* end = nullptr;
    *v = strtod(s, &end);
    if (end == s) return false;
    s = end;
    return true;
}

bool expect(const char*& s, char c)
{
    skip_ws(s);
    if (*s != c) return false;
    ++s;
    return true;
}

// Parses the whole file; returns false (and leaves `out` partial) on any
// deviation from the format above.
bool parse_cache(const char* s, std::map<std::string, Entry>* out)
{
    if (!expect(s, '{')) return false;
    skip_ws(s);
    if (*s == '}') return true;
    for (;;) {
        std::string key;
        if (!parse_string(s, &key) || !expect(s, ':') || !expect(s, '{')) return false;
        Entry e{TuneParams{}, 0.0};
        for (;;) {
            std::string f;
            double v;
            if (!parse_string(s, &f) || !expect(s, ':') || !parse_number(s, &v)) return false;
            if (f == "batch_kchunk") e.p.batch_kchunk = (int64_t)v;
            else if (f == "shortk_tile") e.p.shortk_tile = (int)v;
            else if (f == "lower_small_n") e.p.lower_small_n = (int)v;
            else if (f == "persistent") e.p.persistent = (int)v;
            else if (f == "ms") e.ms = v;
            skip_ws(s);
            if (*s == ',') { ++s; continue; }
            if (*s == '}') { ++s; break; }
            return false;
        }
        (*out)[key] = e;
        skip_ws(s);
        if (*s == ',') { ++s; continue; }
        return *s == '}';
    }
}

bool valid(const TuneParams& p)
{
    return p.batch_kchunk >= 256 && p.batch_kchunk <= (1 << 22) && (p.shortk_tile == 64 || p.shortk_tile == 128) &&
           p.lower_small_n >= 0 && p.lower_small_n <= 4096 && (p.persistent == 0 || p.persistent == 1);
}

// Reload the in-memory copy if the file changed (g_mu held).
void refresh(const char* path)
{
    struct stat st;
    if (stat(path, &st) != 0) {
        g_cache.clear();
        g_path = path;
        g_mtime = g_size = -1;
        return;
    }
    if (g_path == path && g_mtime == (long long)st.st_mtime && g_size == (long long)st.st_size) return;
    g_cache.clear();
    g_path = path;
    g_mtime = (long long)st.st_mtime;
    g_size = (long long)st.st_size;
    FILE* f = fopen(path, "rb");
    if (!f) return;
    std::string text((size_t)st.st_size, '\0');
    const size_t got = fread(&text[0], 1, text.size(), f);
    fclose(f);
    text.resize(got);
    std::map<std::string, Entry> parsed;
    if (parse_cache(text.c_str(), &parsed)) g_cache.swap(parsed);
}

int log2_bucket(double v)
{
    if (!(v > 1.0)) return 0;
    return (int)floor(log2(v) + 0.5);
}

}  // namespace

const TuneParams& tune_params() { return t_params; }

TuneScope::TuneScope(const TuneParams& p) : saved(t_params) { t_params = p; }
TuneScope::~TuneScope() { t_params = saved; }

std::string tune_key_batched(int hpne, int sketch_prec, int qr_prec, int64_t batch, double mean_n, double mean_m)
{
    char buf[160];
    snprintf(buf, sizeof buf, "batched/%s/sk%d/qr%d/b2^%d/n2^%d/m2^%d", hpne ? "hpne" : "pne", sketch_prec, qr_prec,
             log2_bucket((double)batch), log2_bucket(mean_n), log2_bucket(mean_m));
    return buf;
}

bool tune_lookup(const std::string& key, TuneParams* out)
{
    const char* path = cache_path();
    if (!path || !*path) return false;
    std::lock_guard<std::mutex> lk(g_mu);
    refresh(path);
    auto it = g_cache.find(key);
    if (it == g_cache.end() || !valid(it->second.p)) return false;
    *out = it->second.p;
    return true;
}

bool tune_store(const std::string& key, const TuneParams& p, double ms)
{
    const char* path = cache_path();
    if (!path || !*path) return false;
    std::lock_guard<std::mutex> lk(g_mu);
    refresh(path);
    g_cache[key] = Entry{p, ms};
    const std::string tmp = std::string(path) + ".tmp";
    FILE* f = fopen(tmp.c_str(), "wb");
    if (!f) return false;
    fprintf(f, "{\n");
    size_t i = 0;
    for (const auto& kv : g_cache) {
        fprintf(f, "  \"%s\": {\"batch_kchunk\": %lld, \"shortk_tile\": %d, \"lower_small_n\": %d, \"persistent\": %d, \"ms\": %.4f}%s\n",
                kv.first.c_str(), (long long)kv.second.p.batch_kchunk, kv.second.p.shortk_tile,
                kv.second.p.lower_small_n, kv.second.p.persistent, kv.second.ms, ++i < g_cache.size() ? "," : "");
    }
    fprintf(f, "}\n");
    const bool ok = fclose(f) == 0 && rename(tmp.c_str(), path) == 0;
    g_mtime = g_size = -1;   // re-read on the next lookup
    return ok;
}

}  // namespace pne
