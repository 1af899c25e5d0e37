// Multi-RHS column dots for gfx950: the tiled kernel (one chunk per wave,
// column lanes x position sub-groups), its zone reduction and the launch glue
// of the k-column products that run it (spw_mv_batch / spw_vtm_batch with
// the tiled plan).  Shared helpers: spw_device.h.
#include <type_traits>

#include "spw_device.h"

namespace spw {
namespace {

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

// CW consecutive entries of a row of V, read by one load (16 bytes for
// CW = 2 binary64 or CW = 4 binary32 entries).
template <typename VecT, int CW> struct VecRow;
template <typename VecT> struct VecRow<VecT, 1> {
    VecT v[1];
    __device__ __forceinline__ void load(const VecT *p) { v[0] = *p; }
};
template <> struct VecRow<double, 2> {
    double v[2];
    __device__ __forceinline__ void load(const double *p)
    {
        const f64x2_t w = *reinterpret_cast<const f64x2_t *>(p);
        v[0] = w.x;
        v[1] = w.y;
    }
};
template <> struct VecRow<float, 2> {
    float v[2];
    __device__ __forceinline__ void load(const float *p)
    {
        typedef float f32x2_t __attribute__((ext_vector_type(2)));
        const f32x2_t w = *reinterpret_cast<const f32x2_t *>(p);
        v[0] = w.x;
        v[1] = w.y;
    }
};
template <> struct VecRow<float, 4> {
    float v[4];
    __device__ __forceinline__ void load(const float *p)
    {
        const f32x4_t w = *reinterpret_cast<const f32x4_t *>(p);
        v[0] = w.x;
        v[1] = w.y;
        v[2] = w.z;
        v[3] = w.w;
    }
};

template <typename VecT, int BS, int CW> struct TileGather {
    VecRow<VecT, CW> gv[BS];    // v at the rows of the batch's items, CW columns each
    uint32_t m;                 // column-start bits of the batch's items
};

#ifndef SPW_TILE_BS
#define SPW_TILE_BS 8
#endif
constexpr int TILE_BS = SPW_TILE_BS;            // positions per batch

constexpr int TILE_BLOCK = 256;

// CW columns per lane: column lane cl holds columns cl*CW .. cl*CW+CW-1 and
// gathers them with one load; V's rows must then start on CW-entry
// boundaries (ldv a multiple of CW, V 16-byte aligned) and hold at least
// L*CW entries, or k must be a multiple of CW.  Every column is computed with
// the same operations in the same order whatever CW is.
// Stores the CW sums of one lane into a row of U with one store of the whole
// group (two for four binary64 values).  p is aligned to the group.
template <typename OutT, int CW>
__device__ __forceinline__ void put_group(OutT *p, const double *v)
{
    typedef float f32x2_t __attribute__((ext_vector_type(2)));
    if constexpr (sizeof(OutT) == 8 && CW >= 2) {
#pragma unroll
        for (int h = 0; h < CW / 2; ++h) reinterpret_cast<f64x2_t *>(p)[h] = f64x2_t{v[2 * h], v[2 * h + 1]};
    } else if constexpr (sizeof(OutT) == 4 && CW == 4) {
        *reinterpret_cast<f32x4_t *>(p) = f32x4_t{(float)v[0], (float)v[1], (float)v[2], (float)v[3]};
    } else if constexpr (sizeof(OutT) == 4 && CW == 2) {
        *reinterpret_cast<f32x2_t *>(p) = f32x2_t{(float)v[0], (float)v[1]};
    } else {
        *p = (OutT)v[0];
    }
}

// OutT: the type of U (binary64 partial sums for binary32 inputs, or VecT).
// ugroups: U's rows take whole groups of CW entries (ldu a multiple of CW, U
// aligned to a group), so a lane writes its CW sums with one store: a store
// instruction then covers whole 16-byte pieces of a row instead of every
// CW-th entry.
template <typename IdxT, typename ValT, typename VecT, int L, int ITEMS, int CW = 1, typename OutT = VecT,
          int BS = TILE_BS>
__global__ __launch_bounds__(TILE_BLOCK) void cdot_tile(
    const IdxT *__restrict__ idx, const ValT *__restrict__ val, const uint16_t *__restrict__ heads,
    const int4 *__restrict__ cinfo, const int32_t *__restrict__ segcol, int64_t nnz, int64_t nchunks, int k,
    const VecT *__restrict__ V, int64_t ldv, OutT *__restrict__ U, int64_t ldu, double *__restrict__ carry,
    int ugroups)
{
    constexpr int S = WAVE / L;                   // sub-groups per wave
    constexpr int PPL = ITEMS / BS;               // batches per layout lane
    constexpr int NB = L * PPL;                   // batches per sub-group and chunk
    constexpr int SPAN = ITEMS * L;               // positions per sub-group
    constexpr int WCH = WAVE * ITEMS;             // positions per chunk
    static_assert(ITEMS % BS == 0, "a layout lane holds whole batches");
    constexpr int NW = TILE_BLOCK / WAVE;

    const int lane = threadIdx.x & (WAVE - 1);
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x / WAVE);
    const int g = lane / L, cl = lane % L;
    const int c0 = cl * CW;                       // first column of this lane
    const bool colok = c0 < k;
    // idle lanes read a valid group of columns (the last one)
    const int vc = min(c0, ((k - 1) / CW) * CW);
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
    auto gather = [&](TileGather<VecT, BS, CW> &G, const IdxB<IdxT, BS> &R, uint32_t m) __attribute__((always_inline)) {
#pragma unroll
        for (int j = 0; j < BS; ++j) G.gv[j].load(V + (int64_t)R.get(j) * ldv + vc);
        G.m = m;
    };

    // per-chunk walk state; the next chunk's description and column-start
    // bits are loaded one chunk ahead
    int4 ci = make_int4(0, 0, 0, 0), ci_n = cinfo[chunk0];
    uint32_t mask_n = heads[chunk0 * WAVE + lane];
    int base = 0, rel = 0, hk = 0, my_n = 0, s = 0, e = 0;
    double run[CW], head_sum[CW];
#pragma unroll
    for (int w = 0; w < CW; ++w) run[w] = head_sum[w] = 0.0;
    bool multi = false;
    int64_t cc = chunk0;

    auto column = [&](int q) __attribute__((always_inline)) -> int64_t {
        return (ci.w & CHUNK_DENSE) ? (int64_t)ci.x + q : (int64_t)segcol[ci.y + q];
    };
    // the lane's CW sums of one column of U (row `row` of U)
    const bool grp = ugroups && c0 + CW <= k;
    auto put_row = [&](int64_t row, const double *v) __attribute__((always_inline)) {
        if (grp) {
            put_group<OutT, CW>(U + row * ldu + c0, v);
        } else {
#pragma unroll
            for (int w = 0; w < CW; ++w)
                if (c0 + w < k) U[row * ldu + c0 + w] = (OutT)v[w];
        }
    };
    // columns c0 .. c0+CW-1 of segment q: to carry slots when the chunk cuts it, else to U
    auto emit = [&](int q, const double *v) __attribute__((always_inline)) {
        const bool before = q == 0 && !(ci.w & CHUNK_START_HEAD);
        const bool after = q == ci.z - 1 && (ci.w & CHUNK_END_CONT);
        if (before || after) {
            // a segment cut on both sides (the chunk lies inside one column) is the left carry
            double *cr = carry + (2 * cc + (before ? 0 : 1)) * k;
#pragma unroll
            for (int w = 0; w < CW; ++w)
                if (c0 + w < k) cr[c0 + w] = v[w];
        } else {
            put_row(column(q), v);
        }
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
#pragma unroll
        for (int w = 0; w < CW; ++w) run[w] = head_sum[w] = 0.0;
        multi = false;
    };
    auto chunk_end = [&]() __attribute__((always_inline)) {
        const int klast = my_n > 0 ? base + rel : -2 - g;
        const int hkey = my_n > 0 ? (multi ? base + hk : klast) : -2 - g;
        // one segmented scan per column; every column has the same keys
        SegPair x[CW];
#pragma unroll
        for (int w = 0; w < CW; ++w) x[w] = SegPair{run[w], klast};
#pragma unroll
        for (int off = 1; off < S; off <<= 1) {
            const int pk = __shfl_up(x[0].k, off * L, WAVE);
#pragma unroll
            for (int w = 0; w < CW; ++w) {
                const double ps = __shfl_up(x[w].s, off * L, WAVE);
                if (g >= off) x[w] = seg_op(SegPair{ps, pk}, x[w]);
            }
        }
        double prev_s[CW];
        int prev_k = -1, next_hk = -1;
#pragma unroll
        for (int w = 0; w < CW; ++w) prev_s[w] = 0.0;
        if (S > 1) {
#pragma unroll
            for (int w = 0; w < CW; ++w) prev_s[w] = __shfl_up(x[w].s, L, WAVE);
            prev_k = __shfl_up(x[0].k, L, WAVE);
            next_hk = __shfl_down(hkey, L, WAVE);
        }
        if (my_n > 0 && colok) {
            if (multi) {
                double tot[CW];
#pragma unroll
                for (int w = 0; w < CW; ++w) {
                    tot[w] = head_sum[w];
                    if (g > 0 && prev_k == hkey) tot[w] = prev_s[w] + head_sum[w];
                }
                emit(hkey, tot);
            }
            if (g == S - 1 || next_hk != klast) {
                double last[CW];
#pragma unroll
                for (int w = 0; w < CW; ++w) last[w] = x[w].s;
                emit(klast, last);
            }
        }
    };
    auto compute = [&](int64_t q, const ValB<ValT, BS> &A, const TileGather<VecT, BS, CW> &G) __attribute__((always_inline)) {
        const int b = (int)(q % NB);
        if (b == 0) chunk_start(chunk_of(q));
#pragma unroll
        for (int j = 0; j < BS; ++j) {
            const int t = b * BS + j;
            if (t < my_n) {
                if (t > 0 && ((G.m >> j) & 1u)) {
                    if (!multi) {
#pragma unroll
                        for (int w = 0; w < CW; ++w) head_sum[w] = run[w];
                        hk = rel;
                        multi = true;
                    } else {
                        // a column wholly inside this sub-group's positions
                        put_row(column(base + rel), run);
                    }
                    ++rel;
#pragma unroll
                    for (int w = 0; w < CW; ++w) run[w] = 0.0;
                }
                const double a = A.get(j);
#pragma unroll
                for (int w = 0; w < CW; ++w) run[w] = __fma_rn(a, (double)G.gv[j].v[w], run[w]);
            }
        }
        if (b == NB - 1) chunk_end();
    };

    ValB<ValT, BS> A0, A1;
    IdxB<IdxT, BS> R0, R1;
    uint32_t m0 = 0, m1 = 0;
    TileGather<VecT, BS, CW> G0, G1;
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

}  // namespace

namespace {
// The tile shape for k columns: CW columns per lane (one 16-byte gather of
// 2 binary64 or 4 binary32 entries, when `wide`) and L column lanes, the
// power of two >= ceil(k / CW); narrow tiles keep L >= 2.
template <typename VecT>
void tile_shape(int k, bool wide, int *L, int *CW)
{
    int cw = 1;
    if (wide) cw = sizeof(VecT) == 8 ? (k >= 2 ? 2 : 1) : (k >= 4 ? 4 : (k >= 2 ? 2 : 1));
    int l = cw == 1 ? 2 : 1;
    while (l * cw < k) l <<= 1;
    *L = l;
    *CW = cw;
}

template <int ITEMS, typename IdxT, typename ValT, typename VecT, typename OutT>
int launch_tile_items(const spw_matrix_s &A, const ColDot &C, int k, const VecT *V, int64_t ldv, OutT *U,
                      int64_t ldu, bool wide, hipStream_t stream)
{
    int L = 2, CW = 1;
    tile_shape<VecT>(k, wide, &L, &CW);
    // whole groups of CW entries per store when U's rows and base allow them
    const int64_t gbytes = (int64_t)CW * (int64_t)sizeof(OutT);
    const bool ugroups = ldu % CW == 0 && (uintptr_t)U % (uintptr_t)gbytes == 0;
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
    auto go = [&](auto kern) -> int {
        static const int nb = per_cu((const void *)kern);
        const unsigned grid = (unsigned)std::max<int64_t>(1, std::min<int64_t>((int64_t)cus * nb, want));
        hipLaunchKernelGGL(kern, dim3(grid), dim3(TILE_BLOCK), 0, stream, (const IdxT *)C.d_idx,
                           (const ValT *)C.d_val, C.d_heads, (const int4 *)C.d_cinfo, C.d_segcol, C.nnz,
                           C.zp.n_chunks, k, V, ldv, U, ldu, A.scratch.carry, ugroups ? 1 : 0);
        return (int)hipGetLastError();
    };
#define SPW_TILE(LL, WW) \
    if (L == LL && CW == WW) return go(cdot_tile<IdxT, ValT, VecT, LL, ITEMS, WW, OutT>);
    SPW_TILE(2, 1) SPW_TILE(4, 1) SPW_TILE(8, 1) SPW_TILE(16, 1) SPW_TILE(32, 1) SPW_TILE(64, 1)
    SPW_TILE(1, 2) SPW_TILE(2, 2) SPW_TILE(4, 2) SPW_TILE(8, 2) SPW_TILE(16, 2) SPW_TILE(32, 2)
    if constexpr (sizeof(VecT) == 4) {
        SPW_TILE(1, 4) SPW_TILE(2, 4) SPW_TILE(4, 4) SPW_TILE(8, 4) SPW_TILE(16, 4)
    }
#undef SPW_TILE
    return (int)hipErrorInvalidValue;
}

// Chunks of 1,024 or 512 nonzeros (16 or 8 positions per layout lane).
// Chunks of 1,024 or 512 nonzeros.
template <typename IdxT, typename ValT, typename VecT, typename OutT>
int launch_tile(const spw_matrix_s &A, const ColDot &C, int k, const VecT *V, int64_t ldv, OutT *U, int64_t ldu,
                bool wide, hipStream_t stream)
{
    if (C.zp.chunk == 1024)
        return launch_tile_items<16, IdxT, ValT, VecT, OutT>(A, C, k, V, ldv, U, ldu, wide, stream);
    if (C.zp.chunk == 512) return launch_tile_items<8, IdxT, ValT, VecT, OutT>(A, C, k, V, ldv, U, ldu, wide, stream);
    return (int)hipErrorNotSupported;
}

template <typename ValT, typename VecT, typename OutT>
int coldot_batch_typed(const spw_matrix_s &A, const ColDot &C, const int32_t *inv, int k, const VecT *V,
                       int64_t ldv, OutT *U, int64_t ldu, hipStream_t stream)
{
    int e;
    if (C.n_empty > 0) {
        ProfScope ps(stream, "zero_cols_batch");
        hipLaunchKernelGGL(zero_cols_batch<OutT>, dim3(blocks_for(C.n_empty * k, 256)), dim3(256), 0, stream,
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
        // wide gathers (CW columns in one 16-byte load) need rows that start on
        // CW-entry boundaries; the renumbered copy's rows are padded to the
        // tile width, the caller's block must hold whole groups of CW columns
        int Lw = 1, CWw = 1;
        tile_shape<VecT>(k, true, &Lw, &CWw);
        const bool wide = inv != nullptr ||
                          (k % CWw == 0 && ldin % CWw == 0 && ((uintptr_t)Vin % 16) == 0);
        if constexpr (std::is_same<OutT, VecT>::value) {
            e = C.idx_kind == IdxKind::U16
                    ? launch_tile<uint16_t, ValT, VecT, OutT>(A, C, k, Vin, ldin, U, ldu, wide, stream)
                    : launch_tile<int32_t, ValT, VecT, OutT>(A, C, k, Vin, ldin, U, ldu, wide, stream);
        } else {
            // binary64 partial sums of binary32 inputs: the blocked transpose (4-byte indices) only
            if (C.idx_kind == IdxKind::U16 || inv) return (int)hipErrorNotSupported;
            e = launch_tile<int32_t, ValT, VecT, OutT>(A, C, k, Vin, ldin, U, ldu, wide, stream);
        }
        if (e) return e;
    }
    if (C.n_zones > 0) {
        ProfScope ps(stream, "zone_fixup_batch");
        hipLaunchKernelGGL(zone_fixup_batch<OutT>, dim3(blocks_for(C.n_zones * k, 256)), dim3(256), 0, stream,
                           C.d_zone_col, C.d_zone_first, C.d_zone_last, C.n_zones, k, A.scratch.carry, U, ldu);
        if ((e = (int)hipGetLastError())) return e;
    }
    return 0;
}
}  // namespace

int launch_coldot_batch(const spw_matrix_s &A, const ColDot &C, const int32_t *inv, spw_dtype vdt, int32_t k,
                        const void *V, int64_t ldv, void *U, int64_t ldu, void *stream, bool out_f64)
{
    if (k < 1 || k > 64) return (int)hipErrorNotSupported;
    if (C.cols == 0) return 0;
    return with_types(A.value_storage, vdt, [&](auto vt, auto xt) {
        using ValT = decltype(vt);
        using VecT = decltype(xt);
        if (out_f64 && !std::is_same<VecT, double>::value)
            return coldot_batch_typed<ValT, VecT, double>(A, C, inv, k, (const VecT *)V, ldv, (double *)U, ldu,
                                                          (hipStream_t)stream);
        return coldot_batch_typed<ValT, VecT, VecT>(A, C, inv, k, (const VecT *)V, ldv, (VecT *)U, ldu,
                                                    (hipStream_t)stream);
    });
}

// Y = the sum over blocks of the partial sums P (nb blocks of rows x k, row
// stride k), in ascending block order, each output rounded once.
template <typename VoutT>
__global__ void sum_blocks(const double *__restrict__ P, int64_t nb, int64_t rows, int k, VoutT *__restrict__ Y,
                           int64_t ldy)
{
    const int64_t g = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (g >= rows * k) return;
    const int64_t r = g / k;
    const int c = (int)(g - r * k);
    double s = P[g];
    for (int64_t b = 1; b < nb; ++b) s += P[(b * rows + r) * k + c];
    Y[r * ldy + c] = (VoutT)s;
}

int launch_sum_blocks(spw_dtype vdt, int64_t nb, int64_t rows, int32_t k, const double *P, void *out, int64_t ldo,
                      void *stream_)
{
    hipStream_t stream = (hipStream_t)stream_;
    if (rows <= 0) return 0;
    ProfScope ps(stream, "sum_blocks");
    if (vdt == SPW_F64)
        hipLaunchKernelGGL(sum_blocks<double>, dim3(blocks_for(rows * k, 256)), dim3(256), 0, stream, P, nb, rows,
                           (int)k, (double *)out, ldo);
    else
        hipLaunchKernelGGL(sum_blocks<float>, dim3(blocks_for(rows * k, 256)), dim3(256), 0, stream, P, nb, rows,
                           (int)k, (float *)out, ldo);
    return (int)hipGetLastError();
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
