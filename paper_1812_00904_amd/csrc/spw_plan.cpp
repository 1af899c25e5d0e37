// Host-side plan for the column-dot product: equal-nonzero chunks, the columns
// each chunk owns, and the overlap zones (columns cut by a chunk boundary).
//
// The paper determines the zones with neighbour exchanges and scans across
// processors (Section IV-B) because no processor sees the whole matrix.  Here
// the host holds the column pointer array, so the same objects follow from a
// binary search per chunk boundary: the boundary at position s cuts the column
// holding s unless s is the start of a column.  The zone's chunk set S_k is
// the run from the chunk holding the column's start to the last chunk the
// column reaches (Table I).
#include <algorithm>
#include <cstdint>
#include <vector>

#include "spw_internal.h"

namespace spw {

void build_zone_plan(int64_t cols, const int64_t *ptr, int64_t chunk, ZonePlan &zp)
{
    const int64_t nnz = ptr[cols];
    zp.chunk = chunk;
    zp.n_chunks = nnz > 0 ? (nnz + chunk - 1) / chunk : 0;
    zp.owned.assign((size_t)zp.n_chunks + 1, 0);
    zp.jlo.assign((size_t)zp.n_chunks, 0);
    zp.jhi.assign((size_t)zp.n_chunks, 0);
    zp.zone_col.clear();
    zp.zone_first.clear();
    zp.zone_last.clear();
    const int64_t *end = ptr + cols + 1;
    for (int64_t c = 0; c < zp.n_chunks; ++c) {
        const int64_t s = c * chunk;
        // first column whose start is at or after s
        const int64_t o = std::lower_bound(ptr, end, s) - ptr;
        zp.owned[(size_t)c] = (int32_t)o;
        // columns holding the first and the last position of the chunk
        const int64_t e = std::min(nnz, s + chunk);
        zp.jlo[(size_t)c] = (int32_t)(std::upper_bound(ptr, end, s) - ptr - 1);
        zp.jhi[(size_t)c] = (int32_t)(std::upper_bound(ptr, end, e - 1) - ptr - 1);
        if (c > 0 && ptr[o] > s) {
            // column o-1 starts before s and reaches into chunk c: a zone member
            const int32_t j = (int32_t)(o - 1);
            if (!zp.zone_col.empty() && zp.zone_col.back() == j) {
                zp.zone_last.back() = (int32_t)c;
            } else {
                zp.zone_col.push_back(j);
                zp.zone_first.push_back((int32_t)(ptr[j] / chunk));
                zp.zone_last.push_back((int32_t)c);
            }
        }
    }
    zp.owned[(size_t)zp.n_chunks] = (int32_t)cols;
}

}  // namespace spw
