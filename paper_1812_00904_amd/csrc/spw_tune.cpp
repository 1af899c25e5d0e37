// Tuning cache and matrix fingerprints (host code only).
//
// The autotuner (spw_create_opts.autotune) times candidate kernel shapes and
// multi-RHS plans on the device and records each choice under a key that
// names the decision, for a fingerprint of the matrix's shape and sparsity
// structure.  The records live in memory for the process and, when a cache
// file is set (spw_tune_cache_path or the SPW_TUNE_CACHE environment
// variable), in that file: a later process that creates a matrix with the
// same fingerprint takes the recorded choices instead of timing again.
//
// File format: text, one record per line, "<16 hex digits> <key> <value>",
// after a first line "# spw tuning cache v1".  Lines that do not parse are
// ignored; a later record for the same (fingerprint, key) replaces an
// earlier one.  The file is rewritten whole (to a temporary file, then
// renamed) after every new record.
#include <cinttypes>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <map>
#include <mutex>
#include <string>
#include <utility>

#include "spw_internal.h"

namespace spw {
namespace {

struct TuneCache {
    std::mutex mu;
    bool env_checked = false;
    std::string path;                                              // empty: memory only
    std::map<std::pair<uint64_t, std::string>, int32_t> entries;
};

TuneCache &cache()
{
    static TuneCache c;
    return c;
}

bool valid_key(const char *key)
{
    if (!key || !*key) return false;
    const size_t n = strlen(key);
    if (n > 63) return false;
    for (size_t i = 0; i < n; ++i) {
        const char ch = key[i];
        if (ch <= ' ' || ch > '~') return false;    // printable, no blanks
    }
    return true;
}

// Reads `path` into the map (records there win over none; the caller holds the lock).
void load_file(TuneCache &c, const std::string &path)
{
    FILE *f = fopen(path.c_str(), "r");
    if (!f) return;
    char line[256];
    while (fgets(line, sizeof line, f)) {
        if (line[0] == '#') continue;
        char key[64];
        unsigned long long fp = 0;
        long long value = 0;
        if (sscanf(line, "%16llx %63s %lld", &fp, key, &value) == 3 && valid_key(key) &&
            value >= INT32_MIN && value <= INT32_MAX)
            c.entries[{(uint64_t)fp, std::string(key)}] = (int32_t)value;
    }
    fclose(f);
}

// Writes every record to the cache file (the caller holds the lock).
bool save_file(TuneCache &c)
{
    if (c.path.empty()) return true;
    const std::string tmp = c.path + ".tmp" + std::to_string((long long)std::rand());
    FILE *f = fopen(tmp.c_str(), "w");
    if (!f) return false;
    bool ok = fprintf(f, "# spw tuning cache v1\n") > 0;
    for (const auto &e : c.entries)
        ok = ok && fprintf(f, "%016" PRIx64 " %s %d\n", e.first.first, e.first.second.c_str(), (int)e.second) > 0;
    ok = (fclose(f) == 0) && ok;
    if (!ok || std::rename(tmp.c_str(), c.path.c_str()) != 0) {
        std::remove(tmp.c_str());
        return false;
    }
    return true;
}

void check_env(TuneCache &c)
{
    if (c.env_checked) return;
    c.env_checked = true;
    const char *p = std::getenv("SPW_TUNE_CACHE");
    if (p && *p && c.path.empty()) {
        c.path = p;
        load_file(c, c.path);
    }
}

// FNV-1a, 64 bits.
struct Fnv {
    uint64_t h = 1469598103934665603ull;
    void add(const void *p, size_t n)
    {
        const unsigned char *b = static_cast<const unsigned char *>(p);
        for (size_t i = 0; i < n; ++i) {
            h ^= b[i];
            h *= 1099511628211ull;
        }
    }
    template <typename T> void add(T v) { add(&v, sizeof v); }
};

}  // namespace

uint64_t matrix_fingerprint(spw_format fmt, spw_dtype storage, int64_t m, int64_t n, int64_t nnz,
                            const int64_t *ptr, const int32_t *idx)
{
    // shape, storage and up to 4,097 evenly spaced entries of the pointer and
    // index arrays: equal for equal matrices, and in practice different for
    // matrices of different structure
    Fnv f;
    f.add((int32_t)fmt);
    f.add((int32_t)storage);
    f.add(m);
    f.add(n);
    f.add(nnz);
    // every entry of an array of at most `samples` entries, else `samples`
    // evenly spaced ones including the first and the last
    const int64_t outer = fmt == SPW_CSC ? n : m;
    const int64_t samples = 4097;
    auto sample = [&](int64_t len, auto &&at) {
        if (len <= samples) {
            for (int64_t i = 0; i < len; ++i) f.add(at(i));
        } else {
            for (int64_t s = 0; s < samples; ++s) f.add(at((len - 1) * s / (samples - 1)));
        }
    };
    if (ptr) sample(outer + 1, [&](int64_t i) { return ptr[i]; });
    if (idx && nnz > 0) sample(nnz, [&](int64_t i) { return idx[i]; });
    return f.h;
}

bool tune_get(uint64_t fp, const std::string &key, int32_t *value)
{
    TuneCache &c = cache();
    std::lock_guard<std::mutex> lk(c.mu);
    check_env(c);
    const auto it = c.entries.find({fp, key});
    if (it == c.entries.end()) return false;
    *value = it->second;
    return true;
}

bool tune_put(uint64_t fp, const std::string &key, int32_t value)
{
    TuneCache &c = cache();
    std::lock_guard<std::mutex> lk(c.mu);
    check_env(c);
    c.entries[{fp, key}] = value;
    return save_file(c);
}

}  // namespace spw

using namespace spw;

extern "C" {

spw_status spw_tune_cache_path(const char *path)
{
    return guarded("spw_tune_cache_path", [&] {
        TuneCache &c = cache();
        std::lock_guard<std::mutex> lk(c.mu);
        c.env_checked = true;
        c.path = path ? path : "";
        if (!c.path.empty()) load_file(c, c.path);
        return SPW_OK;
    });
}

spw_status spw_tune_cache_clear(void)
{
    return guarded("spw_tune_cache_clear", [&] {
        TuneCache &c = cache();
        std::lock_guard<std::mutex> lk(c.mu);
        c.entries.clear();
        return SPW_OK;
    });
}

spw_status spw_tune_cache_put(uint64_t fingerprint, const char *key, int32_t value)
{
    return guarded("spw_tune_cache_put", [&] {
        if (!valid_key(key)) {
            set_error("spw_tune_cache_put: key must be 1..63 printable characters without blanks");
            return SPW_ERR_INVALID_ARG;
        }
        if (!tune_put(fingerprint, key, value)) {
            set_error("spw_tune_cache_put: the cache file could not be written");
            return SPW_ERR_DEVICE;
        }
        return SPW_OK;
    });
}

spw_status spw_tune_cache_get(uint64_t fingerprint, const char *key, int32_t *value, int32_t *found)
{
    return guarded("spw_tune_cache_get", [&] {
        if (!valid_key(key) || !value || !found) {
            set_error("spw_tune_cache_get: bad key or NULL output");
            return SPW_ERR_INVALID_ARG;
        }
        int32_t v = 0;
        *found = tune_get(fingerprint, key, &v) ? 1 : 0;
        *value = *found ? v : 0;
        return SPW_OK;
    });
}

spw_status spw_matrix_fingerprint(spw_format fmt, spw_dtype storage, int64_t m, int64_t n, int64_t nnz,
                                  const int64_t *ptr, const int32_t *idx, uint64_t *out)
{
    return guarded("spw_matrix_fingerprint", [&] {
        if (!out || !ptr || (nnz > 0 && !idx) || m < 0 || n < 0 || nnz < 0 || (fmt != SPW_CSC && fmt != SPW_CSR)) {
            set_error("spw_matrix_fingerprint: bad argument");
            return SPW_ERR_INVALID_ARG;
        }
        *out = matrix_fingerprint(fmt, storage, m, n, nnz, ptr, idx);
        return SPW_OK;
    });
}

}  // extern "C"
