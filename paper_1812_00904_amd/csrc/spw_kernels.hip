// HIP kernels for gfx950 (CDNA4, wave64) and their launch glue.
//
// Both products are bound by HBM bandwidth (about 0.17 flop per byte for
// binary64 values with 2-byte row indices): no MFMA.  What decides their speed
// on this chip is (a) keeping enough bytes in flight per CU and (b) keeping
// the gathers of the dense vectors off the texture path when their addresses
// diverge across a wave (each distinct cache line costs the L1 a cycle).  So
// both kernels run persistent workgroups whose waves work independently (no
// workgroup barrier inside the main loops), and the gathers go to LDS or are
// arranged so that the lanes of one instruction touch few cache lines.
//
// Column dots (u_j = sum_i v_i b_ij over a CSC matrix B; the paper's v^T A,
// Section IV-A): each wave takes equal-nonzero chunks of 64*ITEMS positions
// (the paper's nonzero split, Section II, with a wave as the processor).  The
// most used entries of v (rows renumbered by count) are staged in LDS.  A lane
// walks ITEMS consecutive positions, closing a run at every column end; runs
// inside a lane are final, the first/last run of each lane are joined across
// the wave by a segmented scan, and a column cut by a chunk boundary leaves a
// carry that the zone kernel adds in ascending chunk order.
//
// Scatter product (y = B x; the paper's A x, Section III): a row panel of y
// lives in LDS per workgroup.  The panel's rows are dealt to the 4 waves of
// the workgroup (balanced by count), and each wave streams, in column order,
// only the nonzeros of its own rows, adding them into LDS.  No two waves touch
// the same LDS entry, and a wave adds in program order, so every sum is formed
// in a fixed order; the per-workgroup partial vectors are then added in
// ascending workgroup order (the paper's y = sum_i y_(i)).  Consecutive lanes
// hold consecutive nonzeros of one column range, so an x gather instruction
// touches only a few cache lines.  No floating-point atomics touch global
// memory: results are bit-identical from run to run.
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

template <typename IdxT, typename ValT, int ITEMS> struct VtmChunk {
    ValRaw<ValT, ITEMS> a;
    IdxRaw<IdxT, ITEMS> r;
    uint32_t mask;              // column-start bits of the lane's positions
};

// MULTI = false: one vector (k = 1, v and out.u[0] unit-stride).
// MULTI = true: k <= MULTI_MAX columns; v is a row-major rows x k block and
// column col goes to out.u[col] with stride out.ld[col].  Each chunk is loaded
// once and reduced once per column with exactly the single-vector arithmetic,
// so every column equals the single-vector result bit for bit.  The hot rows
// are staged in LDS as vh[r*k + col].
// wchunks: NULL, or per worker (wave) the first chunk of its run, P+1 entries
// (column partitioning: worker w reduces chunks wchunks[w] .. wchunks[w+1]-1
// in order instead of every P-th chunk).
template <int BLOCK, int ITEMS, typename IdxT, typename ValT, typename VecT, bool MULTI>
__global__ __launch_bounds__(BLOCK) void vtm_wave(
    const IdxT *__restrict__ idx, const ValT *__restrict__ val, const uint16_t *__restrict__ heads,
    const int4 *__restrict__ cinfo, const int32_t *__restrict__ segcol, int64_t nnz, int64_t nchunks,
    const int32_t *__restrict__ wchunks, const VecT *__restrict__ v, int k, int vhot, ColOut<VecT> out,
    double *__restrict__ carry)
{
    if (!MULTI) k = 1;
    const int64_t ldv = k;
    constexpr int NW = BLOCK / WAVE;
    constexpr int WCH = WAVE * ITEMS;
    extern __shared__ double lds[];
    // LDS: each wave's segment stage (STAGE_STRIDE doubles; binary64 vectors
    // only), then the hot rows of v
    constexpr int STAGED = sizeof(VecT) == 8 ? STAGE_STRIDE : 0;
    VecT *vh = reinterpret_cast<VecT *>(lds + NW * STAGED);
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x / WAVE);
    __attribute__((address_space(3))) double *stage =
        (__attribute__((address_space(3))) double *)(lds + wave * STAGED);
    const int lane = threadIdx.x & (WAVE - 1);

    if (MULTI) {
        stage_rows<BLOCK, 8, VecT>(vh, vhot * k, [&](int i) {
            const int r = i / k;
            return v[(int64_t)r * ldv + (i - r * k)];
        });
    } else {
        stage_rows<BLOCK, 16, VecT>(vh, vhot, [&](int i) { return v[i]; });
    }
    __syncthreads();
    const __attribute__((address_space(3))) VecT *vh3 = (const __attribute__((address_space(3))) VecT *)vh;
    const __attribute__((address_space(1))) VecT *vg1 = (const __attribute__((address_space(1))) VecT *)v;

    int64_t stride = (int64_t)gridDim.x * NW;
    int64_t c = (int64_t)blockIdx.x * NW + wave;
    int64_t cend = nchunks;
    if (wchunks) {
        cend = wchunks[c + 1];
        c = wchunks[c];
        stride = 1;
    }
    if (c >= cend) return;

    // Two chunk buffers used alternately (no register copies, so no wait for
    // data still in flight): while one chunk is reduced, the next one's
    // values, indices and column-start bits are being fetched.
    typedef VtmChunk<IdxT, ValT, ITEMS> Chunk;
    Chunk A, B;
    auto load_chunk = [&](Chunk &C, int64_t cc) {
        const int64_t cb = cc * WCH;
        C.a.load(val + cb, lane);
        C.r.load(idx + cb, lane);
        C.mask = heads[cc * WAVE + lane];
    };
    // Reduces chunk cc held in C (description ci), after issuing the loads of
    // chunk cn into N (when cn < cend).
    auto step = [&](Chunk &C, Chunk &N, int64_t cc, int4 ci, int64_t cn) {
        const int s = (int)(cc * WCH);
        const int e = (int)min((int64_t)s + WCH, nnz);
        for (int col = 0; col < k; ++col) {
            double prod[ITEMS];
            // The LDS reads and the global reads are typed with their address
            // spaces, so they stay ds_reads and global loads (a select between
            // two generic pointers would become one flat load, which every
            // later wait on either counter has to cover), and all LDS reads are
            // issued before the first global read, so none waits for another.
            VecT lv[ITEMS], gv[ITEMS];
#pragma unroll
            for (int i = 0; i < ITEMS; ++i) lv[i] = vh3[min(C.r.get(i), vhot - 1) * k + col];
#pragma unroll
            for (int i = 0; i < ITEMS; ++i) {
                const int ri = C.r.get(i);
                gv[i] = 0;
                if (ri >= vhot) gv[i] = vg1[(int64_t)ri * ldv + col];
            }
            if (col == 0) {
                // The next chunk's loads go out after the gathers (the
                // scheduling barriers keep that order): the load counter
                // retires in order, so the wait for the gathers then leaves
                // the prefetch in flight.  The loads are issued on every path
                // (after the wave's last chunk they fetch the current one
                // again, unused) so that the wait can count them.
                __builtin_amdgcn_sched_barrier(0);
                load_chunk(N, cn < cend ? cn : cc);
                __builtin_amdgcn_sched_barrier(0);
            }
            // a select of the two loaded values, not of two addresses: the
            // gathers stay ahead of the prefetch
#pragma unroll
            for (int i = 0; i < ITEMS; ++i)
                prod[i] = C.a.get(i) * (double)(C.r.get(i) < vhot ? lv[i] : gv[i]);
            VecT *uc = MULTI ? out.u[col] : out.u[0];
            const int64_t ldu = MULTI ? out.ld[col] : 1;
            // full chunk, no empty column inside, segments fit the stage, output
            // view within 2^31 bytes
            const bool dense_full = e - s == WCH && (ci.w & CHUNK_DENSE) &&
                                    ldu <= (int64_t)(1 << 28) / (WCH * (int64_t)sizeof(VecT));
            if constexpr (sizeof(VecT) == 8) {
                if (dense_full && ci.z <= STAGE_CAP)
                    vtm_reduce_dense<ITEMS, VecT>(prod, C.mask, ci, cc, lane, uc, ldu, carry, k, col, stage);
                else
                    vtm_reduce_chunk<ITEMS, VecT>(prod, C.mask, s, e, ci, segcol, cc, lane, uc, ldu, carry, k, col);
            } else {
                if (dense_full)
                    vtm_reduce_dense_direct<ITEMS, VecT>(prod, C.mask, ci, segcol, cc, lane, uc, ldu, carry, k, col);
                else
                    vtm_reduce_chunk<ITEMS, VecT>(prod, C.mask, s, e, ci, segcol, cc, lane, uc, ldu, carry, k, col);
            }
        }
    };

    // chunk sequence c, c + stride, ...; chunk descriptions are loaded one step ahead
    auto ci_at = [&](int64_t cc) { return cc < cend ? cinfo[cc] : make_int4(0, 0, 0, 0); };
    int4 ci0 = cinfo[c];
    load_chunk(A, c);
    for (;;) {
        const int64_t c1 = c + stride;
        const int4 ci1 = ci_at(c1);
        step(A, B, c, ci0, c1);
        if (c1 >= cend) break;
        const int64_t c2 = c1 + stride;
        ci0 = ci_at(c2);
        step(B, A, c1, ci1, c2);
        if (c2 >= cend) break;
        c = c2;
    }
}

// Columns without nonzeros: u_j = 0.
template <typename VecT>
__global__ void zero_cols(const int32_t *__restrict__ cols, int64_t count, VecT *__restrict__ u)
{
    const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (i < count) u[cols[i]] = (VecT)0;
}

// Zone reduction: u[j_k] = right carry of the first chunk + left carries of the
// following chunks of S_k, in ascending chunk order.
template <typename VecT>
__global__ void zone_fixup(const int32_t *__restrict__ zcol, const int32_t *__restrict__ zfirst,
                           const int32_t *__restrict__ zlast, int64_t nz, const double *__restrict__ carry,
                           VecT *__restrict__ u)
{
    const int64_t k = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (k >= nz) return;
    const int a = zfirst[k], b = zlast[k];
    double s = carry[2 * a + 1];
    for (int c = a + 1; c <= b; ++c) s += carry[2 * c];
    u[zcol[k]] = (VecT)s;
}

// Renumber a short vector: out[r] = in[inv[r]].
template <typename VecT>
__global__ void gather_vec(const int32_t *__restrict__ inv, int64_t len, const VecT *__restrict__ in,
                           VecT *__restrict__ out)
{
    const int64_t r = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (r < len) out[r] = in[inv[r]];
}

// ------------------------------------------------------------------------
// Scatter product over one row panel.  Panel q holds the internal rows
// r = q (mod P) for P panels, so every panel sees about the same share of each
// column, and the workgroups of different panels that cover the same column
// range gather the same x entries at about the same time (the second and
// later reads hit in cache instead of HBM).
// Storage: blocks of 64*MV_ITEMS nonzeros.  A block holds nonzeros of one
// wave's rows, in column order, from one workgroup's column range.  Logical
// nonzero j*64 + lane sits at word slot ((j/4)*64 + lane)*4 + j%4 and at value
// slot ((j/2)*64 + lane)*2 + j%2, so every load instruction reads one
// contiguous span while each add instruction covers 64 consecutive nonzeros
// (whose x entries share a few cache lines).  A word is
// (panel-local row << 16 | column - block column base).  The streams are read
// with non-temporal loads so they do not push x out of the caches.
//   blocks : (column base, count) per block
//   wg_blk : per workgroup, NW+1 offsets into blocks: wave w owns [wg_blk[w], wg_blk[w+1])
//   x      : input, entry j at x[j*ldx]
//   partial: per-workgroup partial sums, panel_rows entries each
// The loop keeps two blocks of words/values and one block of x gathers in
// flight.  Dynamic LDS: panel_rows doubles.
// ------------------------------------------------------------------------
constexpr int MV_ITEMS = 16;
constexpr int MV_BLK = WAVE * MV_ITEMS;

template <typename ValT> struct MvBlk {
    uint32_t w[MV_ITEMS];
    ValRaw<ValT, MV_ITEMS> a;
    int2 bd;
};

template <bool NT, typename ValT>
__device__ __forceinline__ void mv_load(MvBlk<ValT> &B, const uint32_t *__restrict__ packed,
                                        const ValT *__restrict__ val, const int2 *__restrict__ blocks, int b, int lane)
{
    B.bd = blocks[b];
    const int64_t base = (int64_t)b * MV_BLK;
#pragma unroll
    for (int g = 0; g < MV_ITEMS / 4; ++g) {
        const u32x4_t q = ld_stream<NT>(reinterpret_cast<const u32x4_t *>(packed + base + (int64_t)(g * 64 + lane) * 4));
        B.w[4 * g] = q.x;
        B.w[4 * g + 1] = q.y;
        B.w[4 * g + 2] = q.z;
        B.w[4 * g + 3] = q.w;
    }
    B.a.template load<NT>(val + base, lane);
}

// One workgroup range of the scatter product into the LDS panel ypan, written
// to out (panel_rows doubles).  Ends with a workgroup barrier, so the panel
// can be reused at once.
template <int BLOCK, typename ValT, typename VecT, bool NT>
__device__ __forceinline__ void mv_range(const uint32_t *__restrict__ packed, const ValT *__restrict__ val,
                                         const int2 *__restrict__ blocks, const int32_t *__restrict__ wg_blk,
                                         int range, const VecT *__restrict__ x, int64_t ldx,
                                         double *__restrict__ out, int panel_rows, double *ypan)
{
    constexpr int NW = BLOCK / WAVE;
    const int tid = threadIdx.x, wave = tid / WAVE, lane = tid & (WAVE - 1);
    for (int i = tid; i < panel_rows; i += BLOCK) ypan[i] = 0.0;
    __syncthreads();

    const int32_t *wb = wg_blk + (int64_t)range * (NW + 1);
    const int b0 = wb[wave], b1 = wb[wave + 1];
    // Two block buffers used alternately (no register copies, so no wait for
    // data still in flight): while block b is added, the x entries of block
    // b+1 and the words/values of block b+2 are being fetched.
    MvBlk<ValT> B0, B1;
    VecT x0[MV_ITEMS], x1[MV_ITEMS];
    // padding slots hold word 0, so their gather reads x[column base]: no branch
    auto gather = [&](const MvBlk<ValT> &B, VecT *xv) {
#pragma unroll
        for (int j = 0; j < MV_ITEMS; ++j) xv[j] = x[(int64_t)(B.bd.x + (int)(B.w[j] & 0xFFFFu)) * ldx];
    };
    auto add_block = [&](const MvBlk<ValT> &B, const VecT *xv, double *p, uint32_t *row) {
#pragma unroll
        for (int j = 0; j < MV_ITEMS; ++j) {
            p[j] = B.a.get(j) * (double)xv[j];
            row[j] = B.w[j] >> 16;
        }
    };
    auto commit = [&](int count, const double *p, const uint32_t *row) {
        const int lim = count - lane;             // item j is a nonzero when j*64 < lim
#pragma unroll
        for (int j = 0; j < MV_ITEMS; ++j)
            if (j * WAVE < lim) __hip_atomic_fetch_add(&ypan[row[j]], p[j], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
    };
    if (b0 < b1) {
        mv_load<NT>(B0, packed, val, blocks, b0, lane);
        gather(B0, x0);
        if (b0 + 1 < b1) mv_load<NT>(B1, packed, val, blocks, b0 + 1, lane);
    }
    for (int b = b0; b < b1; b += 2) {
        double p[MV_ITEMS];
        uint32_t row[MV_ITEMS];
        add_block(B0, x0, p, row);
        int cnt = B0.bd.y;
        if (b + 1 < b1) {
            gather(B1, x1);
            if (b + 2 < b1) mv_load<NT>(B0, packed, val, blocks, b + 2, lane);
        }
        commit(cnt, p, row);
        if (b + 1 >= b1) break;
        add_block(B1, x1, p, row);
        cnt = B1.bd.y;
        if (b + 2 < b1) {
            gather(B0, x0);
            if (b + 3 < b1) mv_load<NT>(B1, packed, val, blocks, b + 3, lane);
        }
        commit(cnt, p, row);
    }
    __syncthreads();
    for (int i = tid; i < panel_rows; i += BLOCK) out[i] = ypan[i];
    __syncthreads();
}

template <int BLOCK, typename ValT, typename VecT>
__global__ __launch_bounds__(BLOCK) void mv_bucket(
    const uint32_t *__restrict__ packed, const ValT *__restrict__ val, const int2 *__restrict__ blocks,
    const int32_t *__restrict__ wg_blk, const VecT *__restrict__ x, int64_t ldx, double *__restrict__ partial,
    int panel_rows)
{
    extern __shared__ double ypan[];
    mv_range<BLOCK, ValT, VecT, true>(packed, val, blocks, wg_blk, blockIdx.x, x, ldx,
                                partial + (int64_t)blockIdx.x * panel_rows, panel_rows, ypan);
}

// k columns in one launch.  TAB = false: column c of a row-major X (x + c,
// stride ldx).  TAB = true: column c read from xin.v[c] with stride
// xin.ld[c] (the inputs of different served requests; the entry is picked by
// a chain of selects on c, so the table stays in kernel-argument registers).
// Workgroup (column c, group g) runs the ranges g*S .. g*S+S-1 of the
// single-column product for column c, each into its own partial slot
// (c * W + range), so every column is summed exactly as the single-column
// call sums it.  The k workgroups of a group are dispatched to the same XCD
// (workgroup ids are dealt to the 8 XCDs round-robin: id b goes to XCD b mod
// 8), so they read the same blocks, and the same lines of a row-major X,
// through one L2 at about the same time (ordinary loads, so the lines stay for
// the others): A streams from HBM about once for the k columns.
template <int BLOCK, typename ValT, typename VecT, bool TAB>
__global__ __launch_bounds__(BLOCK) void mv_bucket_cols(
    const uint32_t *__restrict__ packed, const ValT *__restrict__ val, const int2 *__restrict__ blocks,
    const int32_t *__restrict__ wg_blk, const VecT *__restrict__ x, int64_t ldx, ColIn<VecT> xin,
    double *__restrict__ partial, int panel_rows, int k, int W, int S)
{
    extern __shared__ double ypan[];
    const int b = blockIdx.x;
    const int c = (b % (8 * k)) / 8;
    const int g = (b / (8 * k)) * 8 + b % 8;
    const int w0 = g * S, w1 = min(W, w0 + S);
    const VecT *xc = x + c;
    int64_t ld = ldx;
    if constexpr (TAB) {
        xc = xin.v[0];
        ld = xin.ld[0];
#pragma unroll
        for (int t = 1; t < MULTI_MAX; ++t) {
            xc = c == t ? xin.v[t] : xc;
            ld = c == t ? xin.ld[t] : ld;
        }
    }
    for (int w = w0; w < w1; ++w)
        mv_range<BLOCK, ValT, VecT, false>(packed, val, blocks, wg_blk, w, xc, ld,
                                    partial + ((int64_t)c * W + w) * panel_rows, panel_rows, ypan);
}

// y[caller row] = sum over the panel's workgroups of their partials.  Internal
// row r belongs to panel r mod npanels, at panel-local row r / npanels; threads
// walk the panels one after another so each reads consecutive partials.  Eight
// lanes share a row: lane t adds workgroups t, t+8, t+16, ... in ascending
// order, then the eight sums are combined by a fixed butterfly, so the order
// of every addition is fixed.
template <typename VecT>
__global__ void mv_reduce(const double *__restrict__ partial, int panel_rows, const PanelDesc *__restrict__ panels,
                          int npanels, int64_t rows, const int32_t *__restrict__ inv, VecT *__restrict__ y, int64_t ldy,
                          int64_t col_stride)
{
    // column blockIdx.y: its partials start col_stride doubles further, its output one entry further
    partial += blockIdx.y * col_stride;
    y += blockIdx.y;
    const int64_t g = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    const int64_t slot = g >> 3;              // panel * panel_rows + panel-local row
    const int t = (int)(g & 7);
    const int p = (int)(slot / panel_rows);
    const int local = (int)(slot - (int64_t)p * panel_rows);
    const int64_t r = (int64_t)local * npanels + p;
    const bool live = p < npanels && r < rows;
    double s = 0.0;
    if (live) {
        const PanelDesc pd = panels[p];
        const double *src = partial + (int64_t)pd.wg0 * panel_rows + local;
        int w = t;
        for (; w + 24 < pd.nwg; w += 32) {
            // four loads in flight, added in the same order as one at a time
            const double a0 = src[(int64_t)w * panel_rows], a1 = src[(int64_t)(w + 8) * panel_rows];
            const double a2 = src[(int64_t)(w + 16) * panel_rows], a3 = src[(int64_t)(w + 24) * panel_rows];
            s += a0;
            s += a1;
            s += a2;
            s += a3;
        }
        for (; w < pd.nwg; w += 8) s += src[(int64_t)w * panel_rows];
    }
    s += __shfl_xor(s, 1, 8);
    s += __shfl_xor(s, 2, 8);
    s += __shfl_xor(s, 4, 8);
    if (live && t == 0) y[(int64_t)(inv ? inv[r] : r) * ldy] = (VecT)s;
}

// ------------------------------------------------------------------------
// Multi-RHS column dots, tiled: U = C^T V for 2 <= k <= 64 right-hand sides.
// One wave per 1,024-position chunk.  Lane g*L + c is column lane c (L = k
// rounded up to a power of two) of sub-group g (S = 64/L sub-groups), and
// sub-group g walks positions [g*16L, (g+1)*16L) of the chunk in batches of 8
// (layout lanes g*L .. g*L+L-1 of the interleaved storage; the L lanes of a
// sub-group read the same words).  Column boundaries come from the
// column-start bits as in the single-vector kernel, with sub-groups in place
// of lanes: a sub-group's interior columns are final, its first and last runs
// are joined across sub-groups by the segmented scan, and chunk-cut columns
// leave k-wide carries.  V is row-major (leading dimension ldv): the L lanes of
// a sub-group read one contiguous row segment per item, so every v gather
// touches one or two cache lines.  Products are fused multiply-adds.  Loads
// run ahead of the arithmetic: indices two batches ahead, values and v
// entries one batch ahead, across chunk boundaries.
// ------------------------------------------------------------------------
template <typename IdxT> struct Idx8;            // indices of items half*8 .. half*8+7 of one layout lane
template <> struct Idx8<uint16_t> {
    uint32_t w[4];
    __device__ __forceinline__ void load(const uint16_t *cb, int ll, int half)
    {
        const u32x4_t q = *reinterpret_cast<const u32x4_t *>(cb + (int64_t)(half * 64 + ll) * 8);
        w[0] = q.x;
        w[1] = q.y;
        w[2] = q.z;
        w[3] = q.w;
    }
    __device__ __forceinline__ int get(int j) const { return (int)((w[j >> 1] >> ((j & 1) * 16)) & 0xFFFFu); }
};
template <> struct Idx8<int32_t> {
    uint32_t w[8];
    __device__ __forceinline__ void load(const int32_t *cb, int ll, int half)
    {
#pragma unroll
        for (int p = 0; p < 2; ++p) {
            const u32x4_t q = *reinterpret_cast<const u32x4_t *>(cb + (int64_t)((half * 2 + p) * 64 + ll) * 4);
            w[4 * p] = q.x;
            w[4 * p + 1] = q.y;
            w[4 * p + 2] = q.z;
            w[4 * p + 3] = q.w;
        }
    }
    __device__ __forceinline__ int get(int j) const { return (int)w[j]; }
};
template <typename ValT> struct Val8;           // values of items half*8 .. half*8+7 of one layout lane
template <> struct Val8<double> {
    double a[8];
    __device__ __forceinline__ void load(const double *cb, int ll, int half)
    {
#pragma unroll
        for (int p = 0; p < 4; ++p) {
            const f64x2_t q = *reinterpret_cast<const f64x2_t *>(cb + (int64_t)((half * 4 + p) * 64 + ll) * 2);
            a[2 * p] = q.x;
            a[2 * p + 1] = q.y;
        }
    }
    __device__ __forceinline__ double get(int j) const { return a[j]; }
};
template <> struct Val8<float> {
    float a[8];
    __device__ __forceinline__ void load(const float *cb, int ll, int half)
    {
#pragma unroll
        for (int p = 0; p < 2; ++p) {
            const f32x4_t q = *reinterpret_cast<const f32x4_t *>(cb + (int64_t)((half * 2 + p) * 64 + ll) * 4);
            a[4 * p] = q.x;
            a[4 * p + 1] = q.y;
            a[4 * p + 2] = q.z;
            a[4 * p + 3] = q.w;
        }
    }
    __device__ __forceinline__ double get(int j) const { return (double)a[j]; }
};
template <> struct Val8<Bf16> {
    uint32_t w[4];
    __device__ __forceinline__ void load(const Bf16 *cb, int ll, int half)
    {
        const u32x4_t q =
            *reinterpret_cast<const u32x4_t *>(reinterpret_cast<const uint16_t *>(cb) + (int64_t)(half * 64 + ll) * 8);
        w[0] = q.x;
        w[1] = q.y;
        w[2] = q.z;
        w[3] = q.w;
    }
    __device__ __forceinline__ double get(int j) const
    {
        return bf16_bits_to_f64((w[j >> 1] >> ((j & 1) * 16)) & 0xFFFFu);
    }
};

// BS consecutive items of one layout lane: part p holds items p*BS .. p*BS+BS-1.
template <typename IdxT, int BS> struct IdxB;
template <typename IdxT> struct IdxB<IdxT, 8> {
    Idx8<IdxT> r;
    __device__ __forceinline__ void load(const IdxT *cb, int ll, int part) { r.load(cb, ll, part); }
    __device__ __forceinline__ int get(int j) const { return r.get(j); }
};
template <typename IdxT> struct IdxB<IdxT, 16> {
    IdxRaw<IdxT, 16> r;
    __device__ __forceinline__ void load(const IdxT *cb, int ll, int) { r.load(cb, ll); }
    __device__ __forceinline__ int get(int j) const { return r.get(j); }
};
template <typename ValT, int BS> struct ValB;
template <typename ValT> struct ValB<ValT, 8> {
    Val8<ValT> a;
    __device__ __forceinline__ void load(const ValT *cb, int ll, int part) { a.load(cb, ll, part); }
    __device__ __forceinline__ double get(int j) const { return a.get(j); }
};
template <typename ValT> struct ValB<ValT, 16> {
    ValRaw<ValT, 16> a;
    __device__ __forceinline__ void load(const ValT *cb, int ll, int) { a.load(cb, ll); }
    __device__ __forceinline__ double get(int j) const { return a.get(j); }
};

template <typename VecT, int BS> struct TileGather {
    VecT gv[BS];                // v at the rows of the batch's items
    uint32_t m;                 // column-start bits of the batch's items
};

#ifndef SPW_TILE_BS
#define SPW_TILE_BS 8
#endif
constexpr int TILE_BS = SPW_TILE_BS;            // positions per batch

constexpr int TILE_BLOCK = 256;

template <typename IdxT, typename ValT, typename VecT, int L, int BS = TILE_BS>
__global__ __launch_bounds__(TILE_BLOCK) void cdot_tile(
    const IdxT *__restrict__ idx, const ValT *__restrict__ val, const uint16_t *__restrict__ heads,
    const int4 *__restrict__ cinfo, const int32_t *__restrict__ segcol, int64_t nnz, int64_t nchunks, int k,
    const VecT *__restrict__ V, int64_t ldv, VecT *__restrict__ U, int64_t ldu, double *__restrict__ carry)
{
    constexpr int S = WAVE / L;                   // sub-groups per wave
    constexpr int PPL = 16 / BS;                  // batches per layout lane
    constexpr int NB = L * PPL;                   // batches per sub-group and chunk
    constexpr int SPAN = 16 * L;                  // positions per sub-group
    constexpr int WCH = 1024;
    constexpr int NW = TILE_BLOCK / WAVE;

    const int lane = threadIdx.x & (WAVE - 1);
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x / WAVE);
    const int g = lane / L, cl = lane % L;
    const bool colok = cl < k;
    const int vc = min(cl, k - 1);                // idle lanes read a valid column
    const int64_t nw = (int64_t)gridDim.x * NW;
    const int64_t chunk0 = (int64_t)blockIdx.x * NW + wave;
    if (chunk0 >= nchunks) return;
    const int64_t nchunk_w = (nchunks - 1 - chunk0) / nw + 1;     // chunks of this wave
    const int64_t nq = nchunk_w * NB;                              // batches of this wave
    const int64_t clast = chunk0 + (nchunk_w - 1) * nw;

    auto chunk_of = [&](int64_t q) __attribute__((always_inline)) { return chunk0 + (q / NB) * nw; };
    auto load_idx = [&](IdxB<IdxT, BS> &R, uint32_t &m, int64_t q) __attribute__((always_inline)) {
        q = min(q, nq - 1);
        const int64_t cc = chunk_of(q);
        const int b = (int)(q % NB), ll = g * L + b / PPL, part = b % PPL;
        R.load(idx + cc * WCH, ll, part);
        m = ((uint32_t)heads[cc * WAVE + ll] >> (part * BS)) & ((1u << BS) - 1u);
    };
    auto load_val = [&](ValB<ValT, BS> &A, int64_t q) __attribute__((always_inline)) {
        q = min(q, nq - 1);
        const int64_t cc = chunk_of(q);
        const int b = (int)(q % NB);
        A.load(val + cc * WCH, g * L + b / PPL, b % PPL);
    };
    auto gather = [&](TileGather<VecT, BS> &G, const IdxB<IdxT, BS> &R, uint32_t m) __attribute__((always_inline)) {
#pragma unroll
        for (int j = 0; j < BS; ++j) G.gv[j] = V[(int64_t)R.get(j) * ldv + vc];
        G.m = m;
    };

    // per-chunk walk state; the next chunk's description and column-start
    // bits are loaded one chunk ahead
    int4 ci = make_int4(0, 0, 0, 0), ci_n = cinfo[chunk0];
    uint32_t mask_n = heads[chunk0 * WAVE + lane];
    int base = 0, rel = 0, hk = 0, my_n = 0, s = 0, e = 0;
    double run = 0.0, head_sum = 0.0;
    bool multi = false;
    int64_t cc = chunk0;

    auto column = [&](int q) __attribute__((always_inline)) -> int64_t {
        return (ci.w & CHUNK_DENSE) ? (int64_t)ci.x + q : (int64_t)segcol[ci.y + q];
    };
    auto emit = [&](int q, double value) __attribute__((always_inline)) {
        if (!colok) return;
        const bool before = q == 0 && !(ci.w & CHUNK_START_HEAD);
        const bool after = q == ci.z - 1 && (ci.w & CHUNK_END_CONT);
        if (before) carry[(2 * cc) * k + cl] = value;
        else if (after) carry[(2 * cc + 1) * k + cl] = value;
        else U[column(q) * ldu + cl] = (VecT)value;
    };
    auto chunk_start = [&](int64_t c) __attribute__((always_inline)) {
        cc = c;
        ci = ci_n;
        const uint32_t mask = mask_n;
        {
            const int64_t cn = min(c + nw, clast);
            ci_n = cinfo[cn];
            mask_n = heads[cn * WAVE + lane];
        }
        s = (int)(c * WCH);
        e = (int)min((int64_t)s + WCH, nnz);
        // first segment of each sub-group: column starts after position s in
        // earlier layout lanes, plus its own first position
        const uint32_t after_s = lane == 0 ? (mask & ~1u) : mask;
        const int cnt = __popc(after_s);
        int incl = cnt;
#pragma unroll
        for (int off = 1; off < WAVE; off <<= 1) {
            const int t = __shfl_up(incl, off, WAVE);
            if (lane >= off) incl += t;
        }
        const int first_ll = g * L;
        const int excl = __shfl(incl - cnt, first_ll, WAVE);
        const uint32_t m0 = (uint32_t)__shfl((int)mask, first_ll, WAVE);
        base = excl + (g > 0 ? (int)(m0 & 1u) : 0);
        my_n = max(0, min(SPAN, e - (s + g * SPAN)));
        rel = 0;
        run = 0.0;
        head_sum = 0.0;
        multi = false;
    };
    auto chunk_end = [&]() __attribute__((always_inline)) {
        const int klast = my_n > 0 ? base + rel : -2 - g;
        const int hkey = my_n > 0 ? (multi ? base + hk : klast) : -2 - g;
        SegPair x{run, klast};
#pragma unroll
        for (int off = 1; off < S; off <<= 1) {
            const double ps = __shfl_up(x.s, off * L, WAVE);
            const int pk = __shfl_up(x.k, off * L, WAVE);
            if (g >= off) x = seg_op(SegPair{ps, pk}, x);
        }
        double prev_s = 0.0;
        int prev_k = -1, next_hk = -1;
        if (S > 1) {
            prev_s = __shfl_up(x.s, L, WAVE);
            prev_k = __shfl_up(x.k, L, WAVE);
            next_hk = __shfl_down(hkey, L, WAVE);
        }
        if (my_n > 0) {
            if (multi) {
                double tot = head_sum;
                if (g > 0 && prev_k == hkey) tot = prev_s + head_sum;
                emit(hkey, tot);
            }
            if (g == S - 1 || next_hk != klast) emit(klast, x.s);
        }
    };
    auto compute = [&](int64_t q, const ValB<ValT, BS> &A, const TileGather<VecT, BS> &G) __attribute__((always_inline)) {
        const int b = (int)(q % NB);
        if (b == 0) chunk_start(chunk_of(q));
#pragma unroll
        for (int j = 0; j < BS; ++j) {
            const int t = b * BS + j;
            if (t < my_n) {
                if (t > 0 && ((G.m >> j) & 1u)) {
                    if (!multi) {
                        head_sum = run;
                        hk = rel;
                        multi = true;
                    } else {
                        if (colok) U[column(base + rel) * ldu + cl] = (VecT)run;   // column wholly inside
                    }
                    ++rel;
                    run = 0.0;
                }
                run = __fma_rn(A.get(j), (double)G.gv[j], run);
            }
        }
        if (b == NB - 1) chunk_end();
    };

    ValB<ValT, BS> A0, A1;
    IdxB<IdxT, BS> R0, R1;
    uint32_t m0 = 0, m1 = 0;
    TileGather<VecT, BS> G0, G1;
    load_idx(R0, m0, 0);
    load_val(A0, 0);
    load_idx(R1, m1, 1);
    gather(G0, R0, m0);
    // step q: values of q+1, indices of q+2, gathers of q+1, then batch q
    for (int64_t q = 0;; q += 2) {
        load_val(A1, q + 1);
        load_idx(R0, m0, q + 2);
        gather(G1, R1, m1);
        compute(q, A0, G0);
        if (q + 1 >= nq) break;
        load_val(A0, q + 2);
        load_idx(R1, m1, q + 3);
        gather(G0, R0, m0);
        compute(q + 1, A1, G1);
        if (q + 2 >= nq) break;
    }
}

// Multi-RHS zone reduction: one lane per (zone, right-hand side).
template <typename VoutT>
__global__ void zone_fixup_batch(const int32_t *__restrict__ zcol, const int32_t *__restrict__ zfirst,
                                 const int32_t *__restrict__ zlast, int64_t nz, int k,
                                 const double *__restrict__ carry, VoutT *__restrict__ U, int64_t ldu)
{
    const int64_t g = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (g >= nz * k) return;
    const int64_t z = g / k;
    const int cc = (int)(g - z * k);
    const int a = zfirst[z], b = zlast[z];
    double s = carry[(2 * (int64_t)a + 1) * k + cc];
    for (int c = a + 1; c <= b; ++c) s += carry[(2 * (int64_t)c) * k + cc];
    U[(int64_t)zcol[z] * ldu + cc] = (VoutT)s;
}

template <typename VoutT>
__global__ void zero_cols_batch(const int32_t *__restrict__ cols, int64_t count, int k, VoutT *__restrict__ U,
                                int64_t ldu)
{
    const int64_t g = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (g >= count * k) return;
    const int64_t i = g / k;
    U[(int64_t)cols[i] * ldu + (g - i * k)] = (VoutT)0;
}

// Multi-vector helpers over column tables (k <= MULTI_MAX columns).
template <typename VecT>
__global__ void zero_cols_tab(const int32_t *__restrict__ cols, int64_t count, int k, ColOut<VecT> out)
{
    const int64_t g = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (g >= count * k) return;
    const int64_t i = g / k;
    const int c = (int)(g - i * k);
    out.u[c][(int64_t)cols[i] * out.ld[c]] = (VecT)0;
}

template <typename VecT>
__global__ void zone_fixup_tab(const int32_t *__restrict__ zcol, const int32_t *__restrict__ zfirst,
                               const int32_t *__restrict__ zlast, int64_t nz, int k,
                               const double *__restrict__ carry, ColOut<VecT> out)
{
    const int64_t g = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (g >= nz * k) return;
    const int64_t z = g / k;
    const int cc = (int)(g - z * k);
    const int a = zfirst[z], b = zlast[z];
    double s = carry[(2 * (int64_t)a + 1) * k + cc];
    for (int c = a + 1; c <= b; ++c) s += carry[(2 * (int64_t)c) * k + cc];
    out.u[cc][(int64_t)zcol[z] * out.ld[cc]] = (VecT)s;
}

// out[r*k + c] = column c of the table at caller row inv[r] (or r).
template <typename VecT>
__global__ void gather_tab(const int32_t *__restrict__ inv, int64_t rows, int k, ColIn<VecT> in,
                           VecT *__restrict__ out)
{
    const int64_t g = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (g >= rows * k) return;
    const int64_t r = g / k;
    const int c = (int)(g - r * k);
    const int64_t src = inv ? inv[r] : r;
    out[g] = in.v[c][src * in.ld[c]];
}

// Renumber the rows of a k-wide block: out[r*ldo + c] = in[inv[r]*ldv + c].
template <typename VinT>
__global__ void gather_rows(const int32_t *__restrict__ inv, int64_t rows, int k, const VinT *__restrict__ in,
                            int64_t ldv, VinT *__restrict__ out, int64_t ldo)
{
    const int64_t g = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (g >= rows * k) return;
    const int64_t r = g / k;
    const int cc = (int)(g - r * k);
    out[r * ldo + cc] = in[(int64_t)inv[r] * ldv + cc];
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

// LDS of one column-dot workgroup outside the hot rows: the waves' segment
// stages, for binary64 vectors.
int64_t vtm_stage_bytes(size_t elem_bytes)
{
    return elem_bytes == 8 ? (int64_t)(VTM_BLOCK / WAVE) * STAGE_STRIDE * (int64_t)sizeof(double) : 0;
}
// Hot rows of v that fit beside the stages, for k columns of elem_bytes each.
int64_t hot_rows_limit(size_t elem_bytes, int64_t k)
{
    return (LDS_BYTES / VTM_WG_PER_CU - 256 - vtm_stage_bytes(elem_bytes)) / ((int64_t)elem_bytes * k);
}

template <typename IdxT, typename ValT, typename VecT, bool MULTI>
int launch_vtm_wave(const spw_matrix_s &A, const VecT *vin, int k, const ColOut<VecT> &out, hipStream_t stream)
{
    const ColDot &C = A.cd;
    if (C.zp.chunk != vtm_chunk_default()) return (int)hipErrorNotSupported;
    const int vhot = (int)std::min<int64_t>(A.rows, hot_rows_limit(sizeof(VecT), k));
    const size_t lds = (size_t)vtm_stage_bytes(sizeof(VecT)) + (size_t)vhot * k * sizeof(VecT);
    const int cus = device_cu_count(A.device);
    // column partitioning: one wave per worker of the plan (single-vector calls)
    const int32_t *wch = (!MULTI && C.d_wchunks) ? C.d_wchunks : nullptr;
    auto run = [&](auto kernel, int block) -> int {
        const int nw = block / WAVE;
        const int64_t wgs_needed = (C.zp.n_chunks + nw - 1) / nw;
        const unsigned grid =
            wch ? (unsigned)(C.n_workers / nw)
                : (unsigned)std::max<int64_t>(1, std::min<int64_t>((int64_t)cus * VTM_WG_PER_CU, wgs_needed));
        hipLaunchKernelGGL(kernel, dim3(grid), dim3(block), lds, stream, (const IdxT *)C.d_idx, (const ValT *)C.d_val,
                           C.d_heads, (const int4 *)C.d_cinfo, C.d_segcol, C.nnz, C.zp.n_chunks, wch, vin, k, vhot,
                           out, A.scratch.carry);
        return (int)hipGetLastError();
    };
    if constexpr (!MULTI && sizeof(VecT) == 4 && sizeof(ValT) <= 4) {
        // binary32 or bfloat16 values with binary32 vectors, one column: few
        // enough registers for 16 waves per workgroup, which hide more latency
        // (the plan's worker table of a column partition assumes VTM_BLOCK)
        if (!wch) {
            static const bool attr_w = allow_full_lds(vtm_wave<VTM_BLOCK_F32, VTM_ITEMS, IdxT, ValT, VecT, MULTI>);
            (void)attr_w;
            return run(vtm_wave<VTM_BLOCK_F32, VTM_ITEMS, IdxT, ValT, VecT, MULTI>, VTM_BLOCK_F32);
        }
    }
    static const bool attr = allow_full_lds(vtm_wave<VTM_BLOCK, VTM_ITEMS, IdxT, ValT, VecT, MULTI>);
    (void)attr;
    return run(vtm_wave<VTM_BLOCK, VTM_ITEMS, IdxT, ValT, VecT, MULTI>, VTM_BLOCK);
}

template <typename ValT, typename VecT>
int vtm_typed(const spw_matrix_s &A, const VecT *v, VecT *u, hipStream_t stream)
{
    const ColDot &C = A.cd;
    int e;
    if (C.cols == 0) return 0;
    if (C.n_empty > 0) {
        ProfScope ps(stream, "zero_cols");
        hipLaunchKernelGGL(zero_cols<VecT>, dim3(blocks_for(C.n_empty, 256)), dim3(256), 0, stream, C.d_empty,
                           C.n_empty, u);
        if ((e = (int)hipGetLastError())) return e;
    }
    if (C.nnz == 0) return 0;
    const VecT *vin = v;
    if (A.relabeled) {
        ProfScope ps(stream, "gather_vec");
        VecT *vp = reinterpret_cast<VecT *>(A.scratch.vperm);
        hipLaunchKernelGGL(gather_vec<VecT>, dim3(blocks_for(A.rows, 256)), dim3(256), 0, stream, A.d_inv, A.rows, v,
                           vp);
        if ((e = (int)hipGetLastError())) return e;
        vin = vp;
    }
    {
        ProfScope ps(stream, "vtm_wave");
        ColOut<VecT> out{};
        out.u[0] = u;
        out.ld[0] = 1;
        e = C.idx_kind == IdxKind::U16 ? launch_vtm_wave<uint16_t, ValT, VecT, false>(A, vin, 1, out, stream)
                                       : launch_vtm_wave<int32_t, ValT, VecT, false>(A, vin, 1, out, stream);
        if (e) return e;
    }
    if (C.n_zones > 0) {
        ProfScope ps(stream, "zone_fixup");
        hipLaunchKernelGGL(zone_fixup<VecT>, dim3(blocks_for(C.n_zones, 256)), dim3(256), 0, stream, C.d_zone_col,
                           C.d_zone_first, C.d_zone_last, C.n_zones, A.scratch.carry, u);
        if ((e = (int)hipGetLastError())) return e;
    }
    return 0;
}

// Up to MULTI_MAX columns in one pass, each with its own input and output
// base and stride; every column is bit-identical to the single-vector product.
template <typename ValT, typename VecT>
int vtm_cols_typed(const spw_matrix_s &A, int k, const ColIn<VecT> &in, const ColOut<VecT> &out,
                   hipStream_t stream)
{
    const ColDot &C = A.cd;
    int e;
    if (C.cols == 0) return 0;
    if (C.n_empty > 0) {
        ProfScope ps(stream, "zero_cols");
        hipLaunchKernelGGL(zero_cols_tab<VecT>, dim3(blocks_for(C.n_empty * k, 256)), dim3(256), 0, stream,
                           C.d_empty, C.n_empty, k, out);
        if ((e = (int)hipGetLastError())) return e;
    }
    if (C.nnz == 0) return 0;
    VecT *vp = reinterpret_cast<VecT *>(A.scratch.vperm);
    {
        // the k inputs, renumbered when the rows are, as one rows x k block
        ProfScope ps(stream, "gather_vec");
        hipLaunchKernelGGL(gather_tab<VecT>, dim3(blocks_for(A.rows * k, 256)), dim3(256), 0, stream,
                           A.relabeled ? A.d_inv : nullptr, A.rows, k, in, vp);
        if ((e = (int)hipGetLastError())) return e;
    }
    {
        ProfScope ps(stream, "vtm_wave_multi");
        e = C.idx_kind == IdxKind::U16 ? launch_vtm_wave<uint16_t, ValT, VecT, true>(A, vp, k, out, stream)
                                       : launch_vtm_wave<int32_t, ValT, VecT, true>(A, vp, k, out, stream);
        if (e) return e;
    }
    if (C.n_zones > 0) {
        ProfScope ps(stream, "zone_fixup");
        hipLaunchKernelGGL(zone_fixup_tab<VecT>, dim3(blocks_for(C.n_zones * k, 256)), dim3(256), 0, stream,
                           C.d_zone_col, C.d_zone_first, C.d_zone_last, C.n_zones, k, A.scratch.carry, out);
        if ((e = (int)hipGetLastError())) return e;
    }
    return 0;
}

template <typename VecT>
void fill_tables(int k, const void *const *in, const int64_t *ldi, void *const *out, const int64_t *ldo,
                 ColIn<VecT> &ti, ColOut<VecT> &to)
{
    ti = ColIn<VecT>{};
    to = ColOut<VecT>{};
    for (int c = 0; c < k; ++c) {
        ti.v[c] = (const VecT *)in[c];
        ti.ld[c] = ldi[c];
        to.u[c] = (VecT *)out[c];
        to.ld[c] = ldo[c];
    }
}

// k right-hand sides run as k passes of the scatter kernel over strided
// columns of X and Y.
template <typename ValT, typename VecT>
int mv_typed(const spw_matrix_s &A, int32_t k, const VecT *x, int64_t ldx, VecT *y, int64_t ldy, hipStream_t stream)
{
    if (A.rows == 0) return 0;
    int e;
    const unsigned red_blocks = blocks_for(A.n_panels * A.panel_rows * 8, 256);
    if (k > 1 && A.mv_wgs > 0 && A.scratch.partial_cols && A.scratch.pcols > 0) {
        // columns in batches of up to pcols, one launch per batch
        static const bool attr_c = allow_full_lds(mv_bucket_cols<MV_BLOCK, ValT, VecT, false>);
        (void)attr_c;
        const int W = (int)A.mv_wgs, cus = device_cu_count(A.device);
        for (int32_t c0 = 0; c0 < k; c0 += A.scratch.pcols) {
            const int kb = (int)std::min<int64_t>(A.scratch.pcols, k - c0);
            // S ranges per workgroup, the fewest for which all kb * ceil(W / S)
            // workgroups run at once (one per CU): a few workgroups over the CU
            // count would run as a second round and double the time
            int S = (int)std::max<int64_t>(1, ((int64_t)W * kb + cus - 1) / cus);
            while (S < W && (int64_t)kb * ((W + S - 1) / S) > cus) ++S;
            const int G = (W + S - 1) / S;
            const unsigned grid = (unsigned)(kb * 8 * ((G + 7) / 8));
            {
                ProfScope ps(stream, "mv_bucket");
                hipLaunchKernelGGL((mv_bucket_cols<MV_BLOCK, ValT, VecT, false>), dim3(grid), dim3(MV_BLOCK),
                                   (size_t)A.panel_rows * 8, stream, (const uint32_t *)A.d_mpacked,
                                   (const ValT *)A.d_mval, (const int2 *)A.d_mblocks, A.d_wg_blk, x + c0, ldx,
                                   ColIn<VecT>{}, A.scratch.partial_cols, (int)A.panel_rows, kb, W, S);
                if ((e = (int)hipGetLastError())) return e;
            }
            {
                ProfScope ps(stream, "mv_reduce");
                hipLaunchKernelGGL(mv_reduce<VecT>, dim3(red_blocks, (unsigned)kb), dim3(256), 0, stream,
                                   A.scratch.partial_cols, (int)A.panel_rows, A.d_panels, (int)A.n_panels, A.rows,
                                   A.relabeled ? A.d_inv : nullptr, y + c0, ldy, (int64_t)W * A.panel_rows);
                if ((e = (int)hipGetLastError())) return e;
            }
        }
        return 0;
    }
    static const bool attr = allow_full_lds(mv_bucket<MV_BLOCK, ValT, VecT>);
    (void)attr;
    for (int32_t c = 0; c < k; ++c) {
        if (A.mv_wgs > 0) {
            ProfScope ps(stream, "mv_bucket");
            const size_t lds = (size_t)A.panel_rows * 8;
            hipLaunchKernelGGL((mv_bucket<MV_BLOCK, ValT, VecT>), dim3((unsigned)A.mv_wgs), dim3(MV_BLOCK), lds,
                               stream, (const uint32_t *)A.d_mpacked, (const ValT *)A.d_mval,
                               (const int2 *)A.d_mblocks, A.d_wg_blk, x + c, ldx, A.scratch.partial,
                               (int)A.panel_rows);
            if ((e = (int)hipGetLastError())) return e;
        }
        {
            ProfScope ps(stream, "mv_reduce");
            hipLaunchKernelGGL(mv_reduce<VecT>, dim3(red_blocks), dim3(256), 0, stream, A.scratch.partial,
                               (int)A.panel_rows, A.d_panels, (int)A.n_panels, A.rows, A.relabeled ? A.d_inv : nullptr,
                               y + c, ldy, (int64_t)0);
            if ((e = (int)hipGetLastError())) return e;
        }
    }
    return 0;
}

}  // namespace

int64_t mv_lds_rows_limit(spw_dtype vdt, int32_t k)
{
    (void)vdt;
    return std::min<int64_t>((LDS_BYTES - 256) / (8 * std::max<int32_t>(k, 1)), 65536);
}
int64_t mv_block_nnz() { return MV_BLK; }
int64_t mv_waves() { return MV_BLOCK / WAVE; }
int64_t vtm_chunk_default() { return (int64_t)WAVE * VTM_ITEMS; }
int64_t vtm_workers(int device, int64_t nchunks)
{
    const int64_t nw = VTM_BLOCK / WAVE;
    const int64_t wgs = std::max<int64_t>(1, std::min<int64_t>((int64_t)device_cu_count(device) * VTM_WG_PER_CU,
                                                               (nchunks + nw - 1) / nw));
    return wgs * nw;
}
int64_t vtm_hot_rows_limit(spw_dtype vdt) { return hot_rows_limit(vdt == SPW_F64 ? 8 : 4, 1); }

int device_cu_count(int device)
{
    int cus = 0;
    if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, device) != hipSuccess) return 256;
    return cus > 0 ? cus : 256;
}

int launch_vtm(const spw_matrix_s &A, spw_dtype vdt, const void *v, void *u, void *stream)
{
    return with_types(A.value_storage, vdt, [&](auto vt, auto xt) {
        using ValT = decltype(vt);
        using VecT = decltype(xt);
        return vtm_typed<ValT, VecT>(A, (const VecT *)v, (VecT *)u, (hipStream_t)stream);
    });
}

int launch_vtm_cols(const spw_matrix_s &A, spw_dtype vdt, int32_t k, const void *const *in, const int64_t *ldi,
                    void *const *out, const int64_t *ldo, void *stream)
{
    if (k < 1 || k > MULTI_MAX) return (int)hipErrorInvalidValue;
    return with_types(A.value_storage, vdt, [&](auto vt, auto xt) {
        using ValT = decltype(vt);
        using VecT = decltype(xt);
        ColIn<VecT> ti;
        ColOut<VecT> to;
        fill_tables<VecT>(k, in, ldi, out, ldo, ti, to);
        return vtm_cols_typed<ValT, VecT>(A, k, ti, to, (hipStream_t)stream);
    });
}

int launch_vtm_multi(const spw_matrix_s &A, spw_dtype vdt, int32_t k, const void *v, int64_t ldv, void *u,
                     int64_t ldu, void *stream)
{
    const size_t es = vdt == SPW_F64 ? 8 : 4;
    for (int c0 = 0; c0 < k; c0 += MULTI_MAX) {
        const int kk = std::min(MULTI_MAX, k - c0);
        const void *in[MULTI_MAX];
        void *out[MULTI_MAX];
        int64_t li[MULTI_MAX], lo[MULTI_MAX];
        for (int c = 0; c < kk; ++c) {
            in[c] = (const char *)v + (size_t)(c0 + c) * es;
            out[c] = (char *)u + (size_t)(c0 + c) * es;
            li[c] = ldv;
            lo[c] = ldu;
        }
        const int e = launch_vtm_cols(A, vdt, kk, in, li, out, lo, stream);
        if (e) return e;
    }
    return 0;
}

int launch_mv(const spw_matrix_s &A, spw_dtype vdt, int32_t k, const void *x, int64_t ldx, void *y, int64_t ldy,
              void *stream)
{
    return with_types(A.value_storage, vdt, [&](auto vt, auto xt) {
        using ValT = decltype(vt);
        using VecT = decltype(xt);
        return mv_typed<ValT, VecT>(A, k, (const VecT *)x, ldx, (VecT *)y, ldy, (hipStream_t)stream);
    });
}

namespace {
// One launch of the scatter kernel for k <= MULTI_MAX columns with their own
// input bases and strides, then the fixed-order reduction of each column into
// its own output: every column is summed exactly as a single-column call sums
// it, and the matrix is read once for the k columns.
template <typename ValT, typename VecT>
int mv_cols_tab(const spw_matrix_s &A, int k, const ColIn<VecT> &xin, VecT *const *out, const int64_t *ldo,
                hipStream_t stream)
{
    if (A.rows == 0) return 0;
    int e;
    const int W = (int)A.mv_wgs;
    if (W > 0) {
        static const bool attr_t = allow_full_lds(mv_bucket_cols<MV_BLOCK, ValT, VecT, true>);
        (void)attr_t;
        const int cus = device_cu_count(A.device);
        // as in the row-major form: the fewest ranges per workgroup S for which
        // all k * ceil(W / S) workgroups run at once
        int S = (int)std::max<int64_t>(1, ((int64_t)W * k + cus - 1) / cus);
        while (S < W && (int64_t)k * ((W + S - 1) / S) > cus) ++S;
        const int G = (W + S - 1) / S;
        const unsigned grid = (unsigned)(k * 8 * ((G + 7) / 8));
        ProfScope ps(stream, "mv_bucket");
        hipLaunchKernelGGL((mv_bucket_cols<MV_BLOCK, ValT, VecT, true>), dim3(grid), dim3(MV_BLOCK),
                           (size_t)A.panel_rows * 8, stream, (const uint32_t *)A.d_mpacked, (const ValT *)A.d_mval,
                           (const int2 *)A.d_mblocks, A.d_wg_blk, (const VecT *)nullptr, (int64_t)0, xin,
                           A.scratch.partial_cols, (int)A.panel_rows, k, W, S);
        if ((e = (int)hipGetLastError())) return e;
    }
    const unsigned red_blocks = blocks_for(A.n_panels * A.panel_rows * 8, 256);
    for (int c = 0; c < k; ++c) {
        ProfScope ps(stream, "mv_reduce");
        hipLaunchKernelGGL(mv_reduce<VecT>, dim3(red_blocks), dim3(256), 0, stream,
                           A.scratch.partial_cols + (int64_t)c * W * A.panel_rows, (int)A.panel_rows, A.d_panels,
                           (int)A.n_panels, A.rows, A.relabeled ? A.d_inv : nullptr, out[c], ldo[c], (int64_t)0);
        if ((e = (int)hipGetLastError())) return e;
    }
    return 0;
}
}  // namespace

int launch_mv_cols(const spw_matrix_s &A, spw_dtype vdt, int32_t k, const void *const *in, const int64_t *ldi,
                   void *const *out, const int64_t *ldo, void *stream)
{
    if (k < 1 || k > MULTI_MAX) return (int)hipErrorInvalidValue;
    if (k == 1 || A.scratch.pcols < k || !A.scratch.partial_cols) {
        // one column, or no multi-column partial sums: one pass per column
        for (int c = 0; c < k; ++c) {
            const int e = launch_mv(A, vdt, 1, in[c], ldi[c], out[c], ldo[c], stream);
            if (e) return e;
        }
        return 0;
    }
    return with_types(A.value_storage, vdt, [&](auto vt, auto xt) {
        using ValT = decltype(vt);
        using VecT = decltype(xt);
        ColIn<VecT> ti{};
        VecT *to[MULTI_MAX];
        for (int c = 0; c < k; ++c) {
            ti.v[c] = (const VecT *)in[c];
            ti.ld[c] = ldi[c];
            to[c] = (VecT *)out[c];
        }
        return mv_cols_tab<ValT, VecT>(A, k, ti, to, ldo, (hipStream_t)stream);
    });
}

namespace {
template <typename IdxT, typename ValT, typename VecT>
int launch_tile(const spw_matrix_s &A, const ColDot &C, int k, const VecT *V, int64_t ldv, VecT *U, int64_t ldu,
                hipStream_t stream)
{
    int L = 2;
    while (L < k) L <<= 1;
    const int cus = device_cu_count(A.device);
    const int64_t want = (C.zp.n_chunks + TILE_BLOCK / WAVE - 1) / (TILE_BLOCK / WAVE);
    // persistent: as many workgroups as the chip keeps resident
    auto per_cu = [](const void *kern) {
        int nb = 0;
        if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, kern, TILE_BLOCK, 0) != hipSuccess || nb < 1) {
            (void)hipGetLastError();
            nb = 1;
        }
        return nb;
    };
#define SPW_TILE_CASE(LL)                                                                                           \
    case LL: {                                                                                                      \
        static const int nb = per_cu((const void *)cdot_tile<IdxT, ValT, VecT, LL>);                               \
        const unsigned grid = (unsigned)std::max<int64_t>(1, std::min<int64_t>((int64_t)cus * nb, want));        \
        hipLaunchKernelGGL((cdot_tile<IdxT, ValT, VecT, LL>), dim3(grid), dim3(TILE_BLOCK), 0, stream,              \
                           (const IdxT *)C.d_idx, (const ValT *)C.d_val, C.d_heads, (const int4 *)C.d_cinfo,         \
                           C.d_segcol, C.nnz, C.zp.n_chunks, k, V, ldv, U, ldu, A.scratch.carry);                   \
        break;                                                                                                      \
    }
    switch (L) {
        SPW_TILE_CASE(2)
        SPW_TILE_CASE(4)
        SPW_TILE_CASE(8)
        SPW_TILE_CASE(16)
        SPW_TILE_CASE(32)
        SPW_TILE_CASE(64)
    default: return (int)hipErrorInvalidValue;
    }
#undef SPW_TILE_CASE
    return (int)hipGetLastError();
}

template <typename ValT, typename VecT>
int coldot_batch_typed(const spw_matrix_s &A, const ColDot &C, const int32_t *inv, int k, const VecT *V,
                       int64_t ldv, VecT *U, int64_t ldu, hipStream_t stream)
{
    int e;
    if (C.n_empty > 0) {
        ProfScope ps(stream, "zero_cols_batch");
        hipLaunchKernelGGL(zero_cols_batch<VecT>, dim3(blocks_for(C.n_empty * k, 256)), dim3(256), 0, stream,
                           C.d_empty, C.n_empty, k, U, ldu);
        if ((e = (int)hipGetLastError())) return e;
    }
    if (C.nnz == 0) return 0;
    {
        ProfScope ps(stream, "cdot_tile");
        const VecT *Vin = V;
        int64_t ldin = ldv;
        if (inv) {
            // rows padded to the tile width, so that every gathered row starts
            // on a multiple of its size (a 12-wide binary64 row would straddle
            // two 128-byte lines half of the time)
            const int32_t L = coldot_tile_width(k);
            if (A.scratch.kcap < L) return (int)hipErrorInvalidValue;
            VecT *vp = reinterpret_cast<VecT *>(A.scratch.vperm);
            hipLaunchKernelGGL(gather_rows<VecT>, dim3(blocks_for(C.rows * k, 256)), dim3(256), 0, stream, inv,
                               C.rows, k, V, ldv, vp, (int64_t)L);
            if ((e = (int)hipGetLastError())) return e;
            Vin = vp;
            ldin = L;
        }
        e = C.idx_kind == IdxKind::U16 ? launch_tile<uint16_t, ValT, VecT>(A, C, k, Vin, ldin, U, ldu, stream)
                                       : launch_tile<int32_t, ValT, VecT>(A, C, k, Vin, ldin, U, ldu, stream);
        if (e) return e;
    }
    if (C.n_zones > 0) {
        ProfScope ps(stream, "zone_fixup_batch");
        hipLaunchKernelGGL(zone_fixup_batch<VecT>, dim3(blocks_for(C.n_zones * k, 256)), dim3(256), 0, stream,
                           C.d_zone_col, C.d_zone_first, C.d_zone_last, C.n_zones, k, A.scratch.carry, U, ldu);
        if ((e = (int)hipGetLastError())) return e;
    }
    return 0;
}
}  // namespace

int launch_coldot_batch(const spw_matrix_s &A, const ColDot &C, const int32_t *inv, spw_dtype vdt, int32_t k,
                        const void *V, int64_t ldv, void *U, int64_t ldu, void *stream)
{
    if (k < 1 || k > 64) return (int)hipErrorNotSupported;
    if (C.cols == 0) return 0;
    return with_types(A.value_storage, vdt, [&](auto vt, auto xt) {
        using ValT = decltype(vt);
        using VecT = decltype(xt);
        return coldot_batch_typed<ValT, VecT>(A, C, inv, k, (const VecT *)V, ldv, (VecT *)U, ldu,
                                              (hipStream_t)stream);
    });
}

template <typename T>
__global__ void zero_fill_rows(T *__restrict__ out, int64_t rows, int k, int64_t ld)
{
    const int64_t g = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (g >= rows * k) return;
    const int64_t r = g / k;
    out[r * ld + (g - r * k)] = (T)0;
}

int launch_zero_fill(spw_dtype vdt, int32_t k, void *out, int64_t ld, int64_t rows, void *stream_)
{
    hipStream_t stream = (hipStream_t)stream_;
    if (rows <= 0) return 0;
    if (vdt == SPW_F64)
        hipLaunchKernelGGL(zero_fill_rows<double>, dim3(blocks_for(rows * k, 256)), dim3(256), 0, stream, (double *)out,
                           rows, (int)k, ld);
    else
        hipLaunchKernelGGL(zero_fill_rows<float>, dim3(blocks_for(rows * k, 256)), dim3(256), 0, stream, (float *)out,
                           rows, (int)k, ld);
    return (int)hipGetLastError();
}

}  // namespace spw
