// Host-only checks of the server's request scheduling policy (sched_pick).
// Built and run by tests/test_sched_cpu.py; prints one line per failed check
// and exits non-zero if any failed.
#include <cstdio>
#include <deque>
#include <vector>

#include "spw_sched.h"

using spw::SchedReq;
using spw::SchedState;

static int failures = 0;

static void expect(bool ok, const char *what)
{
    if (!ok) {
        std::printf("FAILED: %s\n", what);
        ++failures;
    }
}

static SchedState state(std::vector<int> busy, std::vector<int> mat_stream, int depth = 2)
{
    SchedState s;
    s.depth = depth;
    s.stream_busy.assign(busy.begin(), busy.end());
    s.mat_stream.assign(mat_stream.begin(), mat_stream.end());
    return s;
}

int main()
{
    std::vector<size_t> picked;
    {
        // same matrix, op and vector type merge in arrival order; others stay
        std::deque<SchedReq> q = {{1, 0, 0, 0, 1}, {2, 1, 0, 0, 2}, {3, 0, 0, 0, 3},
                                  {4, 0, 1, 0, 1}, {5, 0, 0, 1, 1}, {6, 0, 0, 0, 2}};
        const int s = spw::sched_pick(q, state({0, 0}, {-1, -1}), 64, picked);
        expect(s == 0, "idle server picks stream 0");
        expect(picked == std::vector<size_t>({0, 2, 5}), "merge by (matrix, op, vtype) in arrival order");
    }
    {
        // the column cap stops the merge (a later, smaller request may still fit)
        std::deque<SchedReq> q = {{1, 0, 0, 0, 8}, {2, 0, 0, 0, 8}, {3, 0, 0, 0, 7}, {4, 0, 0, 0, 1}};
        spw::sched_pick(q, state({0}, {-1}), 16, picked);
        expect(picked == std::vector<size_t>({0, 1}), "column cap 16 takes 8 + 8");
        spw::sched_pick(q, state({0}, {-1}), 17, picked);
        expect(picked == std::vector<size_t>({0, 1, 3}), "column cap 17 skips the 7 and takes the 1");
    }
    {
        // a matrix bound to a full stream waits; the next runnable request goes
        // to the least busy stream
        std::deque<SchedReq> q = {{1, 0, 0, 0, 1}, {2, 1, 0, 0, 1}, {3, 0, 0, 0, 1}};
        const int s = spw::sched_pick(q, state({2, 1, 0, 1}, {0, -1}), 64, picked);
        expect(s == 2, "least busy stream");
        expect(picked == std::vector<size_t>({1}), "head-of-line request of a busy matrix is skipped");
    }
    {
        // a bound matrix with room stays on its stream even if others are idle
        std::deque<SchedReq> q = {{1, 0, 0, 0, 1}};
        const int s = spw::sched_pick(q, state({1, 0, 0}, {0}), 64, picked);
        expect(s == 0 && picked.size() == 1, "bound matrix keeps its stream");
    }
    {
        // every stream full: nothing runs
        std::deque<SchedReq> q = {{1, 0, 0, 0, 1}, {2, 1, 0, 0, 1}};
        const int s = spw::sched_pick(q, state({2, 2}, {-1, -1}), 64, picked);
        expect(s == -1 && picked.empty(), "all streams at depth");
    }
    {
        // ties go to the lowest stream index; depth 1
        std::deque<SchedReq> q = {{1, 3, 1, 1, 4}};
        const int s = spw::sched_pick(q, state({1, 0, 0}, {-1, -1, -1, -1}, 1), 64, picked);
        expect(s == 1, "tie -> lowest index among free streams");
    }
    {
        std::deque<SchedReq> q;
        const int s = spw::sched_pick(q, state({0}, {}), 64, picked);
        expect(s == -1 && picked.empty(), "empty queue");
    }
    if (failures == 0) std::printf("sched ok\n");
    return failures ? 1 : 0;
}
