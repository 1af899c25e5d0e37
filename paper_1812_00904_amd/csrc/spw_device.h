// Device helpers and launch glue shared by the HIP sources of libspw
// (spw_kernels.hip: single- and few-column products; spw_tile.hip: the tiled
// multi-RHS column dots).  Everything here has internal linkage: each source
// gets its own copy.
#pragma once

#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdint>

#include "spw_internal.h"

namespace spw {
namespace {

constexpr int WAVE = 64;

// Native vector types: non-temporal loads need them.
typedef unsigned int u32x4_t __attribute__((ext_vector_type(4)));
typedef double f64x2_t __attribute__((ext_vector_type(2)));
typedef float f32x4_t __attribute__((ext_vector_type(4)));

// A stored bfloat16 value: the high half of a binary32 number.
struct Bf16 {
    uint16_t bits;
};

__device__ __forceinline__ double bf16_bits_to_f64(uint32_t h) { return (double)__uint_as_float(h << 16); }

// Elements per 16 bytes of a stored value type.
template <typename ValT> struct ValGroup;
template <> struct ValGroup<double> {
    static constexpr int G = 2;
};
template <> struct ValGroup<float> {
    static constexpr int G = 4;
};
template <> struct ValGroup<Bf16> {
    static constexpr int G = 8;
};

// One stored value, promoted exactly to binary64.
__device__ __forceinline__ double val_at(const double *v, int64_t s) { return v[s]; }
__device__ __forceinline__ double val_at(const float *v, int64_t s) { return (double)v[s]; }
__device__ __forceinline__ double val_at(const Bf16 *v, int64_t s) { return bf16_bits_to_f64(v[s].bits); }

// A load of streamed matrix data: non-temporal (NT, the default: read once,
// so it should not push reused vectors out of the caches) or ordinary (data
// that other workgroups read again soon).
template <bool NT, typename T>
__device__ __forceinline__ T ld_stream(const T *p)
{
    if constexpr (NT) return __builtin_nontemporal_load(p);
    else return *p;
}

// N stored values of one lane from an interleaved run: 16-byte group g of
// lane l sits at byte (g*64 + l)*16.  get() promotes exactly to binary64; all
// accumulation is binary64.
template <typename ValT, int N> struct ValRaw;
template <int N> struct ValRaw<double, N> {
    double a[N];
    template <bool NT = true>
    __device__ __forceinline__ void load(const double *base, int lane)
    {
#pragma unroll
        for (int g = 0; g < N / 2; ++g) {
            const f64x2_t w = ld_stream<NT>(reinterpret_cast<const f64x2_t *>(base + (int64_t)(g * 64 + lane) * 2));
            a[2 * g] = w.x;
            a[2 * g + 1] = w.y;
        }
    }
    __device__ __forceinline__ double get(int i) const { return a[i]; }
};
template <int N> struct ValRaw<float, N> {
    float a[N];
    template <bool NT = true>
    __device__ __forceinline__ void load(const float *base, int lane)
    {
#pragma unroll
        for (int g = 0; g < N / 4; ++g) {
            const f32x4_t w = ld_stream<NT>(reinterpret_cast<const f32x4_t *>(base + (int64_t)(g * 64 + lane) * 4));
            a[4 * g] = w.x;
            a[4 * g + 1] = w.y;
            a[4 * g + 2] = w.z;
            a[4 * g + 3] = w.w;
        }
    }
    __device__ __forceinline__ double get(int i) const { return (double)a[i]; }
};
template <int N> struct ValRaw<Bf16, N> {
    uint32_t w[N / 2];
    template <bool NT = true>
    __device__ __forceinline__ void load(const Bf16 *base, int lane)
    {
        const uint16_t *b = reinterpret_cast<const uint16_t *>(base);
#pragma unroll
        for (int g = 0; g < N / 8; ++g) {
            const u32x4_t q = ld_stream<NT>(reinterpret_cast<const u32x4_t *>(b + (int64_t)(g * 64 + lane) * 8));
            w[4 * g] = q.x;
            w[4 * g + 1] = q.y;
            w[4 * g + 2] = q.z;
            w[4 * g + 3] = q.w;
        }
    }
    __device__ __forceinline__ double get(int i) const
    {
        return bf16_bits_to_f64((w[i >> 1] >> ((i & 1) * 16)) & 0xFFFFu);
    }
};

// All lanes of the wave see each other's LDS writes after this point.  Only
// the LDS counter is waited on, so loads of later data stay in flight (a wave's
// LDS operations complete in issue order; the empty asm statements keep the
// compiler from moving memory accesses across this point).
__device__ __forceinline__ void wave_sync()
{
    asm volatile("" ::: "memory");
    __builtin_amdgcn_s_waitcnt(0xC07F);          // lgkmcnt(0); vmcnt and expcnt left open
    __builtin_amdgcn_wave_barrier();
    asm volatile("" ::: "memory");
}

// Raw index words of one lane, loaded from an interleaved chunk (see the
// column-dot kernel): 16-byte group g of lane l sits at byte (g*64 + l)*16.
template <typename IdxT, int N> struct IdxRaw;
template <int N> struct IdxRaw<uint16_t, N> {    // N 2-byte indices in N/2 words
    uint32_t w[N / 2];
    __device__ __forceinline__ void load(const uint16_t *base, int lane)
    {
#pragma unroll
        for (int g = 0; g < N / 8; ++g) {
            const u32x4_t q =
                __builtin_nontemporal_load(reinterpret_cast<const u32x4_t *>(base + (int64_t)(g * 64 + lane) * 8));
            w[4 * g] = q.x;
            w[4 * g + 1] = q.y;
            w[4 * g + 2] = q.z;
            w[4 * g + 3] = q.w;
        }
    }
    __device__ __forceinline__ int get(int i) const { return (int)((w[i >> 1] >> ((i & 1) * 16)) & 0xFFFFu); }
};
template <int N> struct IdxRaw<int32_t, N> {     // N 4-byte indices
    uint32_t w[N];
    __device__ __forceinline__ void load(const int32_t *base, int lane)
    {
#pragma unroll
        for (int g = 0; g < N / 4; ++g) {
            const u32x4_t q =
                __builtin_nontemporal_load(reinterpret_cast<const u32x4_t *>(base + (int64_t)(g * 64 + lane) * 4));
            w[4 * g] = q.x;
            w[4 * g + 1] = q.y;
            w[4 * g + 2] = q.z;
            w[4 * g + 3] = q.w;
        }
    }
    __device__ __forceinline__ int get(int i) const { return (int)w[i]; }
};

// Output columns of a multi-vector pass, each with its own base and stride
// (the columns may belong to different requests).
constexpr int MULTI_MAX = 8;
template <typename VecT> struct ColOut {
    VecT *u[MULTI_MAX];
    int64_t ld[MULTI_MAX];
};
template <typename VecT> struct ColIn {
    const VecT *v[MULTI_MAX];
    int64_t ld[MULTI_MAX];
};

// ------------------------------------------------------------------------
// Segmented sums across a wave.
//
// The pair operator is the paper's segmented addition (Section IV-B):
//     (s, k) o (t, l) = (s + t, l) if k == l, else (t, l)
// It is associative, so an inclusive scan of (partial sum, key) pairs over the
// lanes leaves in each lane the running sum of its key's segment.  The scan
// tree is fixed, so the rounding of every sum is reproducible.
// ------------------------------------------------------------------------
struct SegPair {
    double s;
    int k;
};

__device__ __forceinline__ SegPair seg_op(SegPair a, SegPair b)
{
    return (a.k == b.k) ? SegPair{a.s + b.s, b.k} : b;
}

// Data-parallel-primitive (DPP) moves: row_shr:n shifts within rows of 16
// lanes, row_bcast:15 / row_bcast:31 pass lane 15 / 31 to the following rows
// (row masks 0xA / 0xC).  Lanes without a source keep `old`.
constexpr int DPP_ROW_SHR1 = 0x111, DPP_ROW_SHR2 = 0x112, DPP_ROW_SHR4 = 0x114, DPP_ROW_SHR8 = 0x118;
constexpr int DPP_ROW_BCAST15 = 0x142, DPP_ROW_BCAST31 = 0x143;

template <int CTRL, int ROWS>
__device__ __forceinline__ int dpp_int(int old, int src)
{
    return __builtin_amdgcn_update_dpp(old, src, CTRL, ROWS, 0xF, false);
}
template <int CTRL, int ROWS>
__device__ __forceinline__ double dpp_double(double old, double src)
{
    const long long o = __double_as_longlong(old), v = __double_as_longlong(src);
    const int lo = __builtin_amdgcn_update_dpp((int)o, (int)v, CTRL, ROWS, 0xF, false);
    const int hi = __builtin_amdgcn_update_dpp((int)(o >> 32), (int)(v >> 32), CTRL, ROWS, 0xF, false);
    return __longlong_as_double(((long long)hi << 32) | (long long)(unsigned)lo);
}

// Inclusive sum of an int over the lanes of a wave.
__device__ __forceinline__ int wave_prefix_sum(int x)
{
    x += dpp_int<DPP_ROW_SHR1, 0xF>(0, x);
    x += dpp_int<DPP_ROW_SHR2, 0xF>(0, x);
    x += dpp_int<DPP_ROW_SHR4, 0xF>(0, x);
    x += dpp_int<DPP_ROW_SHR8, 0xF>(0, x);
    x += dpp_int<DPP_ROW_BCAST15, 0xA>(0, x);
    x += dpp_int<DPP_ROW_BCAST31, 0xC>(0, x);
    return x;
}

// One step of the segmented scan: combine with the pair CTRL brings in.
template <int CTRL, int ROWS>
__device__ __forceinline__ void seg_step(SegPair &x)
{
    const int pk = dpp_int<CTRL, ROWS>(-1, x.k);   // -1: no source (keys of live runs are >= 0)
    const double ps = dpp_double<CTRL, ROWS>(0.0, x.s);
    x = seg_op(SegPair{ps, pk}, x);
}

// Segmented inclusive scan over the lanes of a wave.  The keys must not
// decrease from lane to lane except into keys no other lane holds (then a
// lane equal to the last lane of an earlier row shares its run from there).
__device__ __forceinline__ SegPair wave_seg_scan(SegPair x)
{
    seg_step<DPP_ROW_SHR1, 0xF>(x);
    seg_step<DPP_ROW_SHR2, 0xF>(x);
    seg_step<DPP_ROW_SHR4, 0xF>(x);
    seg_step<DPP_ROW_SHR8, 0xF>(x);
    seg_step<DPP_ROW_BCAST15, 0xA>(x);
    seg_step<DPP_ROW_BCAST31, 0xC>(x);
    return x;
}

// ------------------------------------------------------------------------
// Column dots, one wave per chunk of 64*ITEMS positions.
//   idx, val : row (renumbered when relabeled) and value of every position,
//              interleaved inside each chunk: item i of lane l sits at value
//              slot ((i/2)*64 + l)*2 + i%2 and at index slot ((i/G)*64 + l)*G
//              + i%G (G indices per 16 bytes); tails are zero-padded
//   heads    : per chunk and lane, the column-start bits of its positions
//   cinfo    : per chunk, (first column, first segment, segments, flags)
//   segcol   : per segment of a chunk with empty columns inside, its column
//   v        : short input vector (renumbered); rows < vhot are read from LDS
//   u        : long output; a column wholly inside the chunk is final here
//   carry    : [2c] = part of the column entering chunk c from the left,
//              [2c+1] = part of the column leaving chunk c to the right
//              (a column crossing the whole chunk leaves its part in [2c])
// Each wave handles the chunks c, c + stride, ... (or its run of a column
// partition); the values, indices and column-start bits of the next chunk,
// and the description of the one after, are loaded while the current chunk
// is reduced.
// Dynamic LDS: each wave's segment stage, then the vhot hot rows.  Columns
// without nonzeros are written by zero_cols, not here.
// ------------------------------------------------------------------------
// Per-chunk description used by the column dots (built on the host):
//   jlo   : column holding the chunk's first position
//   seg0  : index of the chunk's first entry in the segment-to-column table
//   nseg  : number of segments (runs of positions in one column) in the chunk
//   flags : CHUNK_START_HEAD  the first position starts its column
//           CHUNK_END_CONT    the last column continues into the next chunk
//           CHUNK_DENSE       no empty column inside: segment q is column jlo+q
constexpr int CHUNK_START_HEAD = 1, CHUNK_END_CONT = 2, CHUNK_DENSE = 4;

// Joins the lanes' runs of one chunk and writes what they complete.  Lane
// inputs: `run` is the sum of the lane's last run (segment k), `head_sum` the
// sum of its first run (segment hk) when the lane holds a column start after
// its first position (multi).  A segmented scan adds the runs of each segment
// across lanes; the lane where a segment ends writes it (the chunk's first
// segment to carry [2c] when it started in an earlier chunk, the last to
// [2c+1] when it continues into the next, every other to u).
template <typename VecT>
__device__ __forceinline__ void vtm_chunk_tail(double run, int k, int hk, double head_sum, bool multi, bool active,
                                               int4 ci, const int32_t *__restrict__ segcol, int64_t c, int lane,
                                               VecT *__restrict__ u, int64_t ldu, double *__restrict__ carry, int kk,
                                               int col)
{
    const int jlo = ci.x, seg0 = ci.y, last_seg = ci.z - 1, flags = ci.w;
    const bool dense = (flags & CHUNK_DENSE) != 0;
    auto column = [&](int q) -> int64_t { return dense ? (int64_t)jlo + q : (int64_t)segcol[seg0 + q]; };
    const SegPair o = wave_seg_scan(SegPair{run, k});
    const double prev_s = __shfl_up(o.s, 1, WAVE);
    const int prev_k = __shfl_up(o.k, 1, WAVE);
    const int next_hk = __shfl_down(hk, 1, WAVE);
    if (active) {
        auto emit = [&](int q, double value) {
            const bool before = q == 0 && !(flags & CHUNK_START_HEAD);
            const bool after = q == last_seg && (flags & CHUNK_END_CONT);
            if (before) carry[(2 * c) * kk + col] = value;
            else if (after) carry[(2 * c + 1) * kk + col] = value;
            else u[column(q) * ldu] = (VecT)value;
        };
        if (multi) {
            // the lane's first column ends inside it: add what earlier lanes hold
            double tot = head_sum;
            if (lane > 0 && prev_k == hk) tot = prev_s + head_sum;
            emit(hk, tot);
        }
        if (lane == WAVE - 1 || next_hk != k) emit(k, o.s);
    }
}

// Buffer stores of one value; an offset at or past the view's size writes
// nothing (the hardware range check drops it), which predicates a store per
// lane without changing the exec mask.
typedef unsigned int spw_u32x2 __attribute__((ext_vector_type(2)));
constexpr uint32_t BUF_DROP = 0x80000000u;
__device__ __forceinline__ __amdgpu_buffer_rsrc_t buf_view(void *base, uint32_t bytes)
{
    return __builtin_amdgcn_make_buffer_rsrc(base, (short)0, (int)bytes, 0x00020000);
}
__device__ __forceinline__ void buf_store(double x, __amdgpu_buffer_rsrc_t r, uint32_t off)
{
    __builtin_amdgcn_raw_buffer_store_b64(__builtin_bit_cast(spw_u32x2, x), r, (int)off, 0, 0);
}
__device__ __forceinline__ void buf_store(float x, __amdgpu_buffer_rsrc_t r, uint32_t off)
{
    __builtin_amdgcn_raw_buffer_store_b32(__builtin_bit_cast(uint32_t, x), r, (int)off, 0, 0);
}
// The same with the non-temporal hint (cache policy bit 1 on gfx950), for
// stores a wave makes to whole consecutive lines: they then do not push the
// gathered vector out of L2.  Scattered or strided stores must not use it
// (partial lines written past the cache cost far more).
__device__ __forceinline__ void buf_store_nt(double x, __amdgpu_buffer_rsrc_t r, uint32_t off)
{
    __builtin_amdgcn_raw_buffer_store_b64(__builtin_bit_cast(spw_u32x2, x), r, (int)off, 0, 2);
}

// Segments of one chunk a wave stages in LDS before writing them out; chunks
// with more segments take the general path.
constexpr int STAGE_CAP = 256;
constexpr int STAGE_STRIDE = STAGE_CAP + 64;     // plus one spare slot per lane

// Reduces one full chunk (all 64*ITEMS positions are nonzeros) whose columns
// have no empty column between them, so segment q is column jlo + q, with at
// most STAGE_CAP segments.  Same additions in the same order as
// vtm_reduce_chunk, with the per-position branches replaced by selects.  Every
// segment's sum goes to this wave's LDS stage at its segment index (writes
// that carry nothing go to the lane's spare slot), then the wave copies the
// chunk's segments out: a contiguous run of columns in one or two coalesced
// buffer stores, and the two chunk-cut segments to their carry slots.  LDS
// instructions of one wave execute in order, so the copy sees every write.
// The caller guarantees nseg * ldu * sizeof(VecT) < 2^31.
template <int ITEMS, typename VecT>
__device__ __forceinline__ void vtm_reduce_dense(const double *prod, uint32_t mask, int4 ci, int64_t c, int lane,
                                                 VecT *__restrict__ u, int64_t ldu, double *__restrict__ carry,
                                                 int kk, int col, __attribute__((address_space(3))) double *stage)
{
    const uint32_t after_s = lane == 0 ? (mask & ~1u) : mask;
    const int cnt = __popc(after_s);
    const int incl = wave_prefix_sum(cnt);
    const int k0 = incl - cnt + (lane > 0 ? (int)(mask & 1u) : 0);   // segment of the lane's first position
    const uint32_t hb = mask & ((1u << ITEMS) - 1u) & ~1u;             // column starts after the first position
    const int spare = STAGE_CAP + lane;
    double run = 0.0, head_sum = 0.0;
#pragma unroll
    for (int i = 0; i < ITEMS; ++i) {
        if (i > 0) {
            const uint32_t below = hb & ((1u << i) - 1u);
            const bool hd = (hb >> i) & 1u;
            // the run ending at position i-1 is segment k0 + popc(below)
            stage[(hd && below != 0u) ? k0 + __popc(below) : spare] = run;
            head_sum = (hd && below == 0u) ? run : head_sum;
            run = hd ? 0.0 : run;
        }
        run += prod[i];
    }
    // join the lanes' first and last runs (segmented scan, as in vtm_chunk_tail)
    const int k = k0 + __popc(hb);
    const SegPair o = wave_seg_scan(SegPair{run, k});
    const double prev_s = __shfl_up(o.s, 1, WAVE);
    const int prev_k = __shfl_up(o.k, 1, WAVE);
    const int next_hk = __shfl_down(k0, 1, WAVE);
    const double tot = (lane > 0 && prev_k == k0) ? prev_s + head_sum : head_sum;
    stage[hb != 0u ? k0 : spare] = tot;
    stage[(lane == WAVE - 1 || next_hk != k) ? k : spare] = o.s;
    // copy out: segment t is column jlo + t, except a first segment that began
    // in an earlier chunk and a last one that continues into the next
    const int nseg = ci.z, flags = ci.w;
    const bool first_carry = !(flags & CHUNK_START_HEAD), last_carry = (flags & CHUNK_END_CONT) != 0;
    const __amdgpu_buffer_rsrc_t ub =
        buf_view(u + (int64_t)ci.x * ldu, (uint32_t)((int64_t)nseg * ldu * (int64_t)sizeof(VecT)));
    const uint32_t step_bytes = (uint32_t)(ldu * (int64_t)sizeof(VecT));
    if (sizeof(VecT) == 8 && ldu == 1) {
        // contiguous binary64 outputs: 64 lanes write 512 consecutive bytes
        for (int t = lane; t < nseg; t += WAVE) {
            const double val = stage[t];
            const bool to_carry = (t == 0 && first_carry) || (t == nseg - 1 && last_carry);
            buf_store_nt(val, ub, to_carry ? BUF_DROP : (uint32_t)t * 8u);
        }
    } else {
        for (int t = lane; t < nseg; t += WAVE) {
            const double val = stage[t];
            const bool to_carry = (t == 0 && first_carry) || (t == nseg - 1 && last_carry);
            buf_store((VecT)val, ub, to_carry ? BUF_DROP : (uint32_t)t * step_bytes);
        }
    }
    if (lane == 0) {
        if (first_carry) carry[(2 * c) * kk + col] = stage[0];
        if (last_carry) carry[(2 * c + 1) * kk + col] = stage[nseg - 1];
    }
}

// As vtm_reduce_dense, without the LDS stage (binary32 outputs, whose LDS is
// worth more as hot rows of v): the same additions in the same order, with a
// column wholly inside a lane written by a buffer store of its own.  Same
// additions in the same order as vtm_reduce_chunk, with the per-position
// branches replaced by selects: a column wholly inside a lane is written by a
// buffer store whose offset is out of range for every other position.  The
// caller guarantees nseg * ldu * sizeof(VecT) < 2^31.
template <int ITEMS, typename VecT>
__device__ __forceinline__ void vtm_reduce_dense_direct(const double *prod, uint32_t mask, int4 ci,
                                                 const int32_t *__restrict__ segcol, int64_t c, int lane,
                                                 VecT *__restrict__ u, int64_t ldu, double *__restrict__ carry,
                                                 int kk, int col)
{
    const uint32_t after_s = lane == 0 ? (mask & ~1u) : mask;
    const int cnt = __popc(after_s);
    const int incl = wave_prefix_sum(cnt);
    const int k0 = incl - cnt + (lane > 0 ? (int)(mask & 1u) : 0);   // segment of the lane's first position
    const uint32_t hb = mask & ((1u << ITEMS) - 1u) & ~1u;             // column starts after the first position
    const __amdgpu_buffer_rsrc_t ub =
        buf_view(u + (int64_t)ci.x * ldu, (uint32_t)((int64_t)ci.z * ldu * (int64_t)sizeof(VecT)));
    const uint32_t step_bytes = (uint32_t)(ldu * (int64_t)sizeof(VecT));
    double run = 0.0, head_sum = 0.0;
#pragma unroll
    for (int i = 0; i < ITEMS; ++i) {
        if (i > 0) {
            const uint32_t below = hb & ((1u << i) - 1u);
            const bool hd = (hb >> i) & 1u;
            // the run ending at position i-1 is segment k0 + popc(below)
            const uint32_t off = (uint32_t)(k0 + __popc(below)) * step_bytes;
            buf_store((VecT)run, ub, (hd && below != 0u) ? off : BUF_DROP);
            head_sum = (hd && below == 0u) ? run : head_sum;
            run = hd ? 0.0 : run;
        }
        run += prod[i];
    }
    vtm_chunk_tail<VecT>(run, k0 + __popc(hb), k0, head_sum, hb != 0u, true, ci, segcol, c, lane, u, ldu, carry,
                         kk, col);
}

// Reduces one chunk whose products are in `prod` (lane-owned positions
// p0 .. p0+ITEMS-1).  `mask` bit i is set when position p0+i is the first
// nonzero of its column, so column boundaries are register bit tests.  Runs
// are numbered by segment inside the chunk; the lane's first segment number
// is the count of column starts after the chunk's first position in earlier
// lanes (a wave prefix sum).  u is the output column (entry j at u[j*ldu]);
// carry slot (2c+side) of this column is carry[(2c+side)*kk + col].
template <int ITEMS, typename VecT>
__device__ __forceinline__ void vtm_reduce_chunk(const double *prod, uint32_t mask, int s, int e, int4 ci,
                                                 const int32_t *__restrict__ segcol, int64_t c, int lane,
                                                 VecT *__restrict__ u, int64_t ldu, double *__restrict__ carry,
                                                 int kk, int col)
{
    const int p0 = s + lane * ITEMS;
    const int my_n = max(0, min(ITEMS, e - p0));
    const int jlo = ci.x, seg0 = ci.y, flags = ci.w;
    const bool dense = (flags & CHUNK_DENSE) != 0;
    auto column = [&](int q) -> int64_t { return dense ? (int64_t)jlo + q : (int64_t)segcol[seg0 + q]; };
    // column starts after position s in this lane, and in all earlier lanes
    const uint32_t after_s = lane == 0 ? (mask & ~1u) : mask;
    const int cnt = __popc(after_s);
    const int incl = wave_prefix_sum(cnt);
    double head_sum = 0.0, run = 0.0;
    int hk, k;
    bool multi = false;
    if (my_n > 0) {
        k = incl - cnt + (lane > 0 ? (int)(mask & 1u) : 0);   // segment of the lane's first position
#pragma unroll
        for (int i = 0; i < ITEMS; ++i) {
            if (i < my_n) {
                if (i > 0 && ((mask >> i) & 1u)) {
                    if (!multi) {
                        head_sum = run;
                        hk = k;
                        multi = true;
                    } else {
                        u[column(k) * ldu] = (VecT)run;   // column wholly inside this lane
                    }
                    ++k;
                    run = 0.0;
                }
                run += prod[i];
            }
        }
        if (!multi) hk = k;
    } else {
        k = -2 - lane;                            // inactive lane: a key no one shares
        hk = -2 - lane;
    }

    vtm_chunk_tail<VecT>(run, k, hk, head_sum, multi, my_n > 0, ci, segcol, c, lane, u, ldu, carry, kk, col);
}

// dst[i] = src(i) for i < n, by the BLOCK threads of a workgroup, with U loads
// in flight per thread (a load-then-store loop would wait for every load).
template <int BLOCK, int U, typename T, typename Src>
__device__ __forceinline__ void stage_rows(T *dst, int n, Src src)
{
    for (int base = 0; base < n; base += BLOCK * U) {
        T tmp[U];
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int i = base + u * BLOCK + (int)threadIdx.x;
            tmp[u] = i < n ? src(i) : T(0);
        }
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int i = base + u * BLOCK + (int)threadIdx.x;
            if (i < n) dst[i] = tmp[u];
        }
    }
}

#ifndef SPW_VTM_BLOCK
#define SPW_VTM_BLOCK 512
#endif
#ifndef SPW_VTM_WG_PER_CU
#define SPW_VTM_WG_PER_CU 1
#endif
#ifndef SPW_MV_BLOCK
#define SPW_MV_BLOCK 256
#endif
constexpr int VTM_BLOCK = SPW_VTM_BLOCK;
constexpr int VTM_BLOCK_F32 = 1024;                // single-vector column dots, 4-byte values and vectors or less
constexpr int VTM_WG_PER_CU = SPW_VTM_WG_PER_CU;   // resident workgroups per CU (they share the LDS)
constexpr int VTM_ITEMS = 16;
constexpr int MV_BLOCK = SPW_MV_BLOCK;
constexpr int LDS_BYTES = 160 * 1024;

inline unsigned blocks_for(int64_t n, int per) { return (unsigned)((n + per - 1) / per); }

struct ProfScope {
    void *stream;
    void *token = nullptr;
    ProfScope(void *s, const char *name) : stream(s)
    {
        if (profile_on()) profile_begin(stream, name, &token);
    }
    ~ProfScope()
    {
        if (token) profile_end(stream, token);
    }
};

template <typename K>
bool allow_full_lds(K kernel)
{
    (void)hipFuncSetAttribute((const void *)kernel, hipFuncAttributeMaxDynamicSharedMemorySize, LDS_BYTES);
    return true;
}

// Calls fn(ValT(), VecT()) for the stored value type and the vector type.
template <typename Fn>
int with_types(spw_dtype storage, spw_dtype vdt, Fn &&fn)
{
    const bool v64 = vdt == SPW_F64;
    switch (storage) {
    case SPW_F64: return v64 ? fn(double(), double()) : fn(double(), float());
    case SPW_F32: return v64 ? fn(float(), double()) : fn(float(), float());
    case SPW_BF16: return v64 ? fn(Bf16(), double()) : fn(Bf16(), float());
    }
    return (int)hipErrorNotSupported;
}

}  // namespace
}  // namespace spw
