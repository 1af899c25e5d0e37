// Host-only checks of the chunk / zone plan and the tuning cache, built with
// g++ and AddressSanitizer / UndefinedBehaviorSanitizer by
// tests/test_host_native_cpu.py.  The plan is compared with a brute-force
// statement of its definition (which chunks each column's positions fall in)
// on random column-pointer arrays with empty columns and columns spanning
// many chunks; the cache is written to a file and read back.  Prints one line
// per failed check and exits non-zero if any failed.
#include <cstdint>
#include <cstdio>
#include <cstdlib>
#include <random>
#include <string>
#include <vector>

#include "spw_internal.h"

// The library's error text setter lives with the device code; a stand-in here.
namespace spw {
void set_error(const std::string &) {}
}  // namespace spw

static int failures = 0;

static void expect(bool ok, const char *what, long long a = 0, long long b = 0)
{
    if (!ok) {
        std::printf("FAILED: %s (%lld, %lld)\n", what, a, b);
        ++failures;
    }
}

// Brute force from the definitions: chunk c holds positions [c*C, (c+1)*C);
// a column is a zone when its positions fall in two or more chunks; it owns
// chunk ptr[j]/C; chunk c's first and last positions lie in columns jlo, jhi.
static void check_plan(const std::vector<int64_t> &ptr, int64_t chunk)
{
    const int64_t cols = (int64_t)ptr.size() - 1, nnz = ptr[(size_t)cols];
    spw::ZonePlan zp;
    spw::build_zone_plan(cols, ptr.data(), chunk, zp);
    const int64_t nch = nnz > 0 ? (nnz + chunk - 1) / chunk : 0;
    expect(zp.n_chunks == nch, "chunk count", zp.n_chunks, nch);
    std::vector<int64_t> col_of((size_t)nnz);
    for (int64_t j = 0; j < cols; ++j)
        for (int64_t p = ptr[(size_t)j]; p < ptr[(size_t)j + 1]; ++p) col_of[(size_t)p] = j;
    for (int64_t c = 0; c < nch; ++c) {
        const int64_t s = c * chunk, e = std::min(nnz, s + chunk);
        expect(zp.jlo[(size_t)c] == col_of[(size_t)s], "jlo", c, zp.jlo[(size_t)c]);
        expect(zp.jhi[(size_t)c] == col_of[(size_t)e - 1], "jhi", c, zp.jhi[(size_t)c]);
        // owned[c]: the first column whose start is at or after s
        int64_t o = 0;
        while (o < cols && ptr[(size_t)o] < s) ++o;
        expect(zp.owned[(size_t)c] == o, "owned", c, zp.owned[(size_t)c]);
    }
    expect(zp.owned[(size_t)nch] == cols, "owned end", zp.owned[(size_t)nch], cols);
    size_t z = 0;
    for (int64_t j = 0; j < cols; ++j) {
        const int64_t a = ptr[(size_t)j], b = ptr[(size_t)j + 1];
        if (b - a == 0) continue;
        const int64_t c0 = a / chunk, c1 = (b - 1) / chunk;
        if (c1 == c0) continue;
        const bool have = z < zp.zone_col.size();
        expect(have && zp.zone_col[z] == j, "zone column", j, have ? zp.zone_col[z] : -1);
        expect(have && zp.zone_first[z] == c0, "zone first", j, have ? zp.zone_first[z] : -1);
        expect(have && zp.zone_last[z] == c1, "zone last", j, have ? zp.zone_last[z] : -1);
        ++z;
    }
    expect(z == zp.zone_col.size(), "zone count", (long long)z, (long long)zp.zone_col.size());
}

int main(int argc, char **argv)
{
    std::mt19937_64 rng(20251203);
    for (int t = 0; t < 300; ++t) {
        const int64_t cols = 1 + (int64_t)(rng() % 400);
        std::vector<int64_t> ptr((size_t)cols + 1, 0);
        for (int64_t j = 0; j < cols; ++j) {
            const unsigned r = (unsigned)(rng() % 100);
            int64_t len = r < 30 ? 0 : r < 90 ? (int64_t)(rng() % 12) : (int64_t)(rng() % 5000);
            ptr[(size_t)j + 1] = ptr[(size_t)j] + len;
        }
        for (int64_t chunk : {512, 1024, 7, 1})
            if (ptr[(size_t)cols] / chunk < 200000) check_plan(ptr, chunk);
    }
    check_plan(std::vector<int64_t>{0}, 1024);            // no columns
    check_plan(std::vector<int64_t>{0, 0, 0}, 512);       // no nonzeros
    check_plan(std::vector<int64_t>{0, 5000}, 512);       // one column over ten chunks

    // fingerprints: equal arrays, equal keys; a changed index, another key
    std::vector<int64_t> p{0, 3, 3, 7};
    std::vector<int32_t> i{0, 1, 2, 0, 1, 2, 3};
    const uint64_t f1 = spw::matrix_fingerprint(SPW_CSC, SPW_F64, 4, 3, 7, p.data(), i.data());
    const uint64_t f2 = spw::matrix_fingerprint(SPW_CSC, SPW_F64, 4, 3, 7, p.data(), i.data());
    i[4] = 2;
    const uint64_t f3 = spw::matrix_fingerprint(SPW_CSC, SPW_F64, 4, 3, 7, p.data(), i.data());
    expect(f1 == f2, "fingerprint repeat");
    expect(f1 != f3, "fingerprint sees indices");

    // the cache: records survive a reload from the file
    const std::string path = argc > 1 ? argv[1] : "host_check_cache.txt";
    expect(spw_tune_cache_path(path.c_str()) == SPW_OK, "cache path");
    expect(spw_tune_cache_put(f1, "plan.sc.f64.k16", 3) == SPW_OK, "put");
    expect(spw_tune_cache_put(f1, "coldot.chunk", 512) == SPW_OK, "put");
    expect(spw_tune_cache_put(f1, "bad key", 1) == SPW_ERR_INVALID_ARG, "key with a blank");
    expect(spw_tune_cache_clear() == SPW_OK, "clear");
    int32_t v = 0, found = 0;
    expect(spw_tune_cache_get(f1, "coldot.chunk", &v, &found) == SPW_OK && found == 0, "cleared");
    expect(spw_tune_cache_path(path.c_str()) == SPW_OK, "reload");
    expect(spw_tune_cache_get(f1, "coldot.chunk", &v, &found) == SPW_OK && found == 1 && v == 512, "chunk back");
    expect(spw_tune_cache_get(f1, "plan.sc.f64.k16", &v, &found) == SPW_OK && found == 1 && v == 3, "plan back");
    std::remove(path.c_str());

    if (failures == 0) std::printf("host ok\n");
    return failures == 0 ? 0 : 1;
}
