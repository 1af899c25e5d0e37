// Request scheduling policy of the server (pure host code, no HIP).
//
// Requests wait in one arrival-ordered queue.  Each registered matrix owns the
// scratch (partial sums, carries) its products use, so all work on a matrix
// runs on one stream at a time: a matrix with work in flight is bound to that
// stream until the work completes.  Each stream holds at most `depth` issued
// groups; requests arriving meanwhile stay queued and are merged into the next
// group of their matrix (continuous batching).
#pragma once

#include <cstdint>
#include <deque>
#include <vector>

namespace spw {

struct SchedReq {
    uint64_t ticket;
    int32_t mat;     // registered matrix index
    int32_t op;      // 0 = A x, 1 = v^T A
    int32_t vdt;     // vector type
    int32_t k;       // columns
};

struct SchedState {
    int32_t depth = 2;                  // groups in flight per stream
    std::vector<int32_t> stream_busy;   // groups in flight per stream
    std::vector<int32_t> mat_stream;    // per matrix: stream it is bound to, -1 when idle
};

// Chooses the next group to issue.  The group starts with the oldest queued
// request that can run now: its matrix is idle and some stream has room (the
// least busy, lowest index on ties), or its matrix's stream has room.  Later
// requests with the same matrix, operation and vector type join in arrival
// order while the total column count stays <= max_cols.  Fills `picked` with
// queue positions (ascending) and returns the stream, or -1 if nothing can run.
inline int sched_pick(const std::deque<SchedReq> &q, const SchedState &st, int32_t max_cols,
                      std::vector<size_t> &picked)
{
    picked.clear();
    const int ns = (int)st.stream_busy.size();
    int free_stream = -1;
    for (int s = 0; s < ns; ++s)
        if (st.stream_busy[(size_t)s] < st.depth &&
            (free_stream < 0 || st.stream_busy[(size_t)s] < st.stream_busy[(size_t)free_stream]))
            free_stream = s;
    for (size_t i = 0; i < q.size(); ++i) {
        const SchedReq &h = q[i];
        const int bound = st.mat_stream[(size_t)h.mat];
        int s = -1;
        if (bound >= 0) {
            if (st.stream_busy[(size_t)bound] < st.depth) s = bound;
        } else {
            s = free_stream;
        }
        if (s < 0) continue;
        picked.push_back(i);
        int32_t cols = h.k;
        for (size_t j = i + 1; j < q.size(); ++j) {
            const SchedReq &r = q[j];
            if (r.mat == h.mat && r.op == h.op && r.vdt == h.vdt && cols + r.k <= max_cols) {
                picked.push_back(j);
                cols += r.k;
            }
        }
        return s;
    }
    return -1;
}

}  // namespace spw
