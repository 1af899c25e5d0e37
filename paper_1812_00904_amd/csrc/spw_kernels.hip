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
#include "spw_device.h"

namespace spw {
namespace {

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
            // The wave issues its reads at raised priority and drops back for
            // the product and the reduction: a wave with reads to issue then
            // wins the issue slot over one that is reducing, which keeps more
            // reads in flight per CU.
            __builtin_amdgcn_s_setprio(3);
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
            __builtin_amdgcn_s_setprio(0);
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
    // Two block buffers used alternately: while block b is added, the x
    // entries of block b+1 and the words/values of block b+2 are being
    // fetched.  (The compiler issues block b+1's gathers ahead of block b's
    // products, so each step first waits for the words those gathers index;
    // a form of this loop without that wait, tried, was no faster.)
    MvBlk<ValT> B0, B1;
    VecT x0[MV_ITEMS], x1[MV_ITEMS];
    // padding slots hold word 0, so their gather reads x[column base]: no branch.
    // A unit-stride x (every single-vector call) takes 32-bit column offsets.
    auto gather = [&](const MvBlk<ValT> &B, VecT *xv) {
        if (ldx == 1) {
#pragma unroll
            for (int j = 0; j < MV_ITEMS; ++j) xv[j] = x[B.bd.x + (int)(B.w[j] & 0xFFFFu)];
        } else {
#pragma unroll
            for (int j = 0; j < MV_ITEMS; ++j) xv[j] = x[(int64_t)(B.bd.x + (int)(B.w[j] & 0xFFFFu)) * ldx];
        }
    };
    auto add_block = [&](const MvBlk<ValT> &B, const VecT *xv, double *p, uint32_t *row) {
#pragma unroll
        for (int j = 0; j < MV_ITEMS; ++j) {
            p[j] = B.a.get(j) * (double)xv[j];
            row[j] = B.w[j] >> 16;
        }
    };
    auto commit = [&](int count, const double *p, const uint32_t *row) {
        if (count == MV_BLK) {                    // a full block: every item is a nonzero
#pragma unroll
            for (int j = 0; j < MV_ITEMS; ++j)
                __hip_atomic_fetch_add(&ypan[row[j]], p[j], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
            return;
        }
        const int lim = count - lane;             // item j is a nonzero when j*64 < lim
#pragma unroll
        for (int j = 0; j < MV_ITEMS; ++j)
            if (j * WAVE < lim) __hip_atomic_fetch_add(&ypan[row[j]], p[j], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
    };
    // The loads and gathers are issued on every path, of the last block again
    // past the end of the range (so each buffer is written on every path and
    // the compiler keeps the two in place instead of copying between them).
    // Ranges of one or two blocks (small matrices) skip those repeats.
    if (b0 < b1 && b1 - b0 <= 2) {
        mv_load<NT>(B0, packed, val, blocks, b0, lane);
        gather(B0, x0);
        if (b1 - b0 == 2) mv_load<NT>(B1, packed, val, blocks, b0 + 1, lane);
        double p[MV_ITEMS];
        uint32_t row[MV_ITEMS];
        add_block(B0, x0, p, row);
        if (b1 - b0 == 2) gather(B1, x1);
        commit(B0.bd.y, p, row);
        if (b1 - b0 == 2) {
            add_block(B1, x1, p, row);
            commit(B1.bd.y, p, row);
        }
    } else if (b0 < b1) {
        const int last = b1 - 1;
        mv_load<NT>(B0, packed, val, blocks, b0, lane);
        gather(B0, x0);
        mv_load<NT>(B1, packed, val, blocks, min(b0 + 1, last), lane);
        for (int b = b0;; b += 2) {
            double p[MV_ITEMS];
            uint32_t row[MV_ITEMS];
            add_block(B0, x0, p, row);
            int cnt = B0.bd.y;
            gather(B1, x1);
            mv_load<NT>(B0, packed, val, blocks, min(b + 2, last), lane);
            commit(cnt, p, row);
            if (b + 1 >= b1) break;
            add_block(B1, x1, p, row);
            cnt = B1.bd.y;
            gather(B0, x0);
            mv_load<NT>(B1, packed, val, blocks, min(b + 3, last), lane);
            commit(cnt, p, row);
            if (b + 2 >= b1) break;
        }
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

// Resident column-dot workgroups per CU for a workgroup of `block` threads:
// smaller workgroups run two to a CU (8 waves, as one 512-thread workgroup),
// each with half the LDS.
int vtm_wgs_per_cu(int block) { return block >= VTM_BLOCK ? VTM_WG_PER_CU : VTM_BLOCK / block; }
// LDS of one column-dot workgroup outside the hot rows: the waves' segment
// stages, for binary64 vectors.
int64_t vtm_stage_bytes(size_t elem_bytes, int block = VTM_BLOCK)
{
    return elem_bytes == 8 ? (int64_t)(block / WAVE) * STAGE_STRIDE * (int64_t)sizeof(double) : 0;
}
// Hot rows of v that fit beside the stages, for k columns of elem_bytes each.
int64_t hot_rows_limit(size_t elem_bytes, int64_t k, int block = VTM_BLOCK)
{
    return (LDS_BYTES / vtm_wgs_per_cu(block) - 256 - vtm_stage_bytes(elem_bytes, block)) /
           ((int64_t)elem_bytes * k);
}

// Whether the single-vector column dots fit 16 waves per CU (128 registers
// per lane): binary32 vectors with 4- or 2-byte values, or chunks of 512
// (8 positions per lane) of any type.
template <int ITEMS, typename ValT, typename VecT>
constexpr bool vtm_fits_1024()
{
    return (sizeof(VecT) == 4 && sizeof(ValT) <= 4) || ITEMS <= 8;
}

// The column-dot workgroup size for a single-vector call: the matrix's choice
// for the vector type (spw_create_opts.wg_size or the tuner's), else 1,024
// threads for binary32 vectors with 4- or 2-byte values (16 waves hide more
// latency) and 512 otherwise.  1,024 needs few enough registers (above); a
// column partition keeps 512 (its worker table assumes it).
template <int ITEMS, typename ValT, typename VecT>
int vtm_block_for(const spw_matrix_s &A, bool colpart)
{
    if (colpart) return VTM_BLOCK;
    int b = A.vtm_block[sizeof(VecT) == 8 ? 0 : 1];
    if (b == 0) b = (sizeof(VecT) == 4 && sizeof(ValT) <= 4) ? VTM_BLOCK_F32 : VTM_BLOCK;
    if (b == 1024 && !vtm_fits_1024<ITEMS, ValT, VecT>()) b = VTM_BLOCK;
    return b;
}

template <int ITEMS, typename IdxT, typename ValT, typename VecT, bool MULTI>
int launch_vtm_wave_items(const spw_matrix_s &A, const VecT *vin, int k, const ColOut<VecT> &out,
                          hipStream_t stream)
{
    const ColDot &C = A.cd;
    const int cus = device_cu_count(A.device);
    // column partitioning: one wave per worker of the plan (single-vector calls)
    const int32_t *wch = (!MULTI && C.d_wchunks) ? C.d_wchunks : nullptr;
    const int block = MULTI ? VTM_BLOCK : vtm_block_for<ITEMS, ValT, VecT>(A, wch != nullptr);
    const int vhot = (int)std::min<int64_t>(A.rows, hot_rows_limit(sizeof(VecT), k, block));
    const size_t lds = (size_t)vtm_stage_bytes(sizeof(VecT), block) + (size_t)vhot * k * sizeof(VecT);
    auto run = [&](auto kernel) -> int {
        const int nw = block / WAVE;
        const int64_t wgs_needed = (C.zp.n_chunks + nw - 1) / nw;
        const unsigned grid =
            wch ? (unsigned)(C.n_workers / nw)
                : (unsigned)std::max<int64_t>(1, std::min<int64_t>((int64_t)cus * vtm_wgs_per_cu(block), wgs_needed));
        hipLaunchKernelGGL(kernel, dim3(grid), dim3(block), lds, stream, (const IdxT *)C.d_idx, (const ValT *)C.d_val,
                           C.d_heads, (const int4 *)C.d_cinfo, C.d_segcol, C.nnz, C.zp.n_chunks, wch, vin, k, vhot,
                           out, A.scratch.carry);
        return (int)hipGetLastError();
    };
    if constexpr (!MULTI && vtm_fits_1024<ITEMS, ValT, VecT>()) {
        if (block == 1024) {
            static const bool attr_w = allow_full_lds(vtm_wave<1024, ITEMS, IdxT, ValT, VecT, MULTI>);
            (void)attr_w;
            return run(vtm_wave<1024, ITEMS, IdxT, ValT, VecT, MULTI>);
        }
    }
    if constexpr (!MULTI) {
        if (block == 256) {
            static const bool attr_q = allow_full_lds(vtm_wave<256, ITEMS, IdxT, ValT, VecT, MULTI>);
            (void)attr_q;
            return run(vtm_wave<256, ITEMS, IdxT, ValT, VecT, MULTI>);
        }
    }
    static const bool attr = allow_full_lds(vtm_wave<VTM_BLOCK, ITEMS, IdxT, ValT, VecT, MULTI>);
    (void)attr;
    return run(vtm_wave<VTM_BLOCK, ITEMS, IdxT, ValT, VecT, MULTI>);
}

// Chunks of 1,024 (16 positions per lane) or 512 (8 per lane) nonzeros.
template <typename IdxT, typename ValT, typename VecT, bool MULTI>
int launch_vtm_wave(const spw_matrix_s &A, const VecT *vin, int k, const ColOut<VecT> &out, hipStream_t stream)
{
    if (A.cd.zp.chunk == 1024) return launch_vtm_wave_items<16, IdxT, ValT, VecT, MULTI>(A, vin, k, out, stream);
    if (A.cd.zp.chunk == 512) return launch_vtm_wave_items<8, IdxT, ValT, VecT, MULTI>(A, vin, k, out, stream);
    return (int)hipErrorNotSupported;
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
bool vtm_chunk_supported(int64_t chunk) { return chunk == 512 || chunk == 1024; }
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

}  // namespace spw
