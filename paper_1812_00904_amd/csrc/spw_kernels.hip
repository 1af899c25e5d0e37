// HIP kernels for gfx950 (CDNA4, wave64) and their launch glue.
//
// Both products are bound by HBM bandwidth (about 0.17 flop per byte for
// binary64 values with 2-byte row indices), so the kernels are written for
// streaming: coalesced 16-byte loads of the index and value arrays, the short
// vector read through L1/L2 (or held in LDS), no MFMA.
//
// Column dots (u_j = sum_i v_i b_ij over a CSC matrix B; the paper's v^T A,
// Section IV-A): one workgroup per equal-nonzero chunk.  The chunk's products
// are staged in LDS, each column that starts in the chunk is summed by one
// lane (or one wave when long), and the partial sums of columns cut by a chunk
// boundary ("overlap zones") go to a carry array; a second kernel adds the
// carries of each zone in ascending chunk order (the zone reduction).
//
// Scatter product (y = B x; the paper's A x, Section III): a row panel of y
// lives in LDS per workgroup; each workgroup streams a contiguous run of the
// panel's nonzeros and adds a_ij x_j into LDS.  The waves of a workgroup take
// turns (one wave at a time between barriers), so every LDS sum is formed in a
// fixed order; the per-workgroup partial vectors are then added in ascending
// workgroup order (the paper's y = sum_i y_(i)).  No floating-point atomics
// touch global memory, so results are bit-identical from run to run.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdint>

#include "spw_internal.h"

namespace spw {
namespace {

constexpr int WAVE = 64;

__device__ __forceinline__ double wave_sum(double v)
{
    // Butterfly over the 64 lanes; the pattern is fixed, so the result is too.
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) v += __shfl_xor(v, off, WAVE);
    return v;
}

// Fixed-order sum over a workgroup; every lane receives the result.
template <int BLOCK>
__device__ __forceinline__ double block_sum(double v, double *red)
{
    constexpr int NW = BLOCK / WAVE;
    v = wave_sum(v);
    const int wave = threadIdx.x / WAVE, lane = threadIdx.x % WAVE;
    __syncthreads();
    if (lane == 0) red[wave] = v;
    __syncthreads();
    double s = 0.0;
#pragma unroll
    for (int w = 0; w < NW; ++w) s += red[w];
    return s;
}

template <typename IdxT> struct IdxPair;
template <> struct IdxPair<uint16_t> {
    __device__ __forceinline__ static void load(const uint16_t *p, int &a, int &b)
    {
        uint32_t w = *reinterpret_cast<const uint32_t *>(p);
        a = (int)(w & 0xFFFFu);
        b = (int)(w >> 16);
    }
};
template <> struct IdxPair<int32_t> {
    __device__ __forceinline__ static void load(const int32_t *p, int &a, int &b)
    {
        int2 w = *reinterpret_cast<const int2 *>(p);
        a = w.x;
        b = w.y;
    }
};

// ------------------------------------------------------------------------
// Column dots over one chunk.
//   ptr    : cols+1 column starts (absolute positions)
//   idx    : row of every position (renumbered rows when relabeled)
//   val    : value of every position
//   owned  : first column starting in each chunk (n_chunks+1 entries)
//   v      : short input vector (already renumbered)
//   u      : long output; columns wholly inside one chunk are final here
//   carry  : [2c] = part of the column that entered chunk c from the left,
//            [2c+1] = part of the last owned column when it leaves chunk c
// ------------------------------------------------------------------------
template <int BLOCK, int CHUNK, typename IdxT>
__global__ __launch_bounds__(BLOCK) void vtm_chunk_f64(
    const int32_t *__restrict__ ptr, const IdxT *__restrict__ idx, const double *__restrict__ val,
    const int32_t *__restrict__ owned, int64_t nnz, const double *__restrict__ v,
    double *__restrict__ u, double *__restrict__ carry)
{
    constexpr int LONG_SEG = 96;                 // segments longer than this use a whole wave
    constexpr int NW = BLOCK / WAVE;
    __shared__ double prod[CHUNK];
    __shared__ int long_cols[CHUNK / LONG_SEG + 2];
    __shared__ int n_long;
    __shared__ double red[NW];

    const int tid = threadIdx.x;
    const int64_t c = blockIdx.x;
    const int64_t s = c * (int64_t)CHUNK;
    const int len = (int)min((int64_t)CHUNK, nnz - s);

    // Phase 1: products of the chunk into LDS (coalesced 16-byte value loads).
    if (len == CHUNK) {
#pragma unroll
        for (int r = 0; r < CHUNK / (2 * BLOCK); ++r) {
            const int e = 2 * (tid + r * BLOCK);
            const double2 a = *reinterpret_cast<const double2 *>(val + s + e);
            int i0, i1;
            IdxPair<IdxT>::load(idx + s + e, i0, i1);
            double2 pr;
            pr.x = a.x * v[i0];
            pr.y = a.y * v[i1];
            *reinterpret_cast<double2 *>(prod + e) = pr;
        }
    } else {
        for (int e = tid; e < len; e += BLOCK) prod[e] = val[s + e] * v[(int)idx[s + e]];
    }
    if (tid == 0) n_long = 0;
    __syncthreads();

    const int o0 = owned[c], o1 = owned[c + 1];
    const int64_t e_abs = s + len;

    // Phase 2a: the column entering from the left (a zone member), if any.
    const int lend = (int)min((int64_t)ptr[o0] - s, (int64_t)len);
    if (lend > 0) {
        double part = 0.0;
        for (int e = tid; e < lend; e += BLOCK) part += prod[e];
        part = block_sum<BLOCK>(part, red);
        if (tid == 0) carry[2 * c] = part;
    }

    // Phase 2b: columns starting in this chunk, one lane each.
    for (int j = o0 + tid; j < o1; j += BLOCK) {
        const int64_t a = ptr[j], b = ptr[j + 1];
        const int aa = (int)(a - s), bb = (int)(min(b, e_abs) - s);
        if (bb - aa > LONG_SEG) {
            long_cols[atomicAdd(&n_long, 1)] = j;
            continue;
        }
        double sum = 0.0;
        for (int e = aa; e < bb; ++e) sum += prod[e];
        if (b <= e_abs) u[j] = sum;
        else carry[2 * c + 1] = sum;
    }
    __syncthreads();

    // Phase 2c: long columns, one wave each (lane-strided, then a fixed butterfly).
    const int wave = tid / WAVE, lane = tid % WAVE;
    const int nl = n_long;
    for (int q = wave; q < nl; q += NW) {
        const int j = long_cols[q];
        const int64_t a = ptr[j], b = ptr[j + 1];
        const int aa = (int)(a - s), bb = (int)(min(b, e_abs) - s);
        double part = 0.0;
        for (int e = aa + lane; e < bb; e += WAVE) part += prod[e];
        part = wave_sum(part);
        if (lane == 0) {
            if (b <= e_abs) u[j] = part;
            else carry[2 * c + 1] = part;
        }
    }
}

// Zone reduction: u[j_k] = right carry of the first chunk + left carries of the
// following chunks of S_k, in ascending chunk order.
__global__ void zone_fixup_f64(const int32_t *__restrict__ zcol, const int32_t *__restrict__ zfirst,
                               const int32_t *__restrict__ zlast, int64_t nz,
                               const double *__restrict__ carry, double *__restrict__ u)
{
    const int64_t k = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (k >= nz) return;
    const int a = zfirst[k], b = zlast[k];
    double s = carry[2 * a + 1];
    for (int c = a + 1; c <= b; ++c) s += carry[2 * c];
    u[zcol[k]] = s;
}

// Renumber a short vector: out[r] = in[inv[r]].
__global__ void gather_f64(const int32_t *__restrict__ inv, int64_t len, const double *__restrict__ in,
                           double *__restrict__ out)
{
    const int64_t r = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (r < len) out[r] = in[inv[r]];
}

__global__ void fill_f64(double *__restrict__ out, int64_t len, double value)
{
    const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (i < len) out[i] = value;
}

// ------------------------------------------------------------------------
// Scatter product over one panel.
//   pptr    : n_panels blocks of cols+1 column starts (absolute positions)
//   idx/val : panel-local rows and values, panels padded to whole tiles
//   tiles   : [start, end) positions and column range [jlo, jhi] of each tile
//   wgs     : panel and tile range of each workgroup
//   partial : per-workgroup partial sums, panel_rows entries each
// Dynamic LDS: panel_rows doubles (the y panel) + SLICE ints (column starts).
// ------------------------------------------------------------------------
template <int BLOCK, int ITEMS, int SLICE, typename IdxT>
__global__ __launch_bounds__(BLOCK) void mv_panel_f64(
    const int32_t *__restrict__ pptr, int64_t ptr_len, const IdxT *__restrict__ idx,
    const double *__restrict__ val, const Tile *__restrict__ tiles, const WgDesc *__restrict__ wgs,
    const double *__restrict__ x, double *__restrict__ partial, int panel_rows)
{
    extern __shared__ double smem[];
    double *ypan = smem;
    int32_t *slice = reinterpret_cast<int32_t *>(smem + panel_rows);
    constexpr int NW = BLOCK / WAVE;
    const int tid = threadIdx.x, wave = tid / WAVE;

    const WgDesc wd = wgs[blockIdx.x];
    const int32_t *ptr = pptr + (int64_t)wd.panel * ptr_len;
    for (int i = tid; i < panel_rows; i += BLOCK) ypan[i] = 0.0;

    for (int t = wd.t0; t < wd.t1; ++t) {
        const Tile td = tiles[t];
        const int ncol = td.jhi - td.jlo + 2;        // column starts jlo .. jhi+1
        const bool in_lds = ncol <= SLICE;
        __syncthreads();                             // previous tile is done with `slice`
        if (in_lds)
            for (int i = tid; i < ncol; i += BLOCK) slice[i] = ptr[td.jlo + i];
        __syncthreads();
        const int32_t *cs = in_lds ? slice : ptr + td.jlo;   // cs[k] = start of column jlo+k

        double prod[ITEMS];
        int row[ITEMS];
        const int p0 = td.start + tid * ITEMS;
        if (p0 < td.end) {
            // largest k with cs[k] <= p0 (the column holding p0)
            int lo = 0, hi = ncol - 2;
            while (lo < hi) {
                const int mid = (lo + hi + 1) >> 1;
                if (cs[mid] <= p0) lo = mid;
                else hi = mid - 1;
            }
            int k = lo;
            int nxt = cs[k + 1];
            if (p0 + ITEMS <= td.end) {
                double vv[ITEMS];
                int rr[ITEMS];
#pragma unroll
                for (int i = 0; i < ITEMS; i += 2) {
                    const double2 a = *reinterpret_cast<const double2 *>(val + p0 + i);
                    vv[i] = a.x;
                    vv[i + 1] = a.y;
                    IdxPair<IdxT>::load(idx + p0 + i, rr[i], rr[i + 1]);
                }
#pragma unroll
                for (int i = 0; i < ITEMS; ++i) {
                    while (nxt <= p0 + i) { ++k; nxt = cs[k + 1]; }
                    prod[i] = vv[i] * x[td.jlo + k];
                    row[i] = rr[i];
                }
            } else {
#pragma unroll
                for (int i = 0; i < ITEMS; ++i) {
                    const int p = p0 + i;
                    if (p < td.end) {
                        while (nxt <= p) { ++k; nxt = cs[k + 1]; }
                        prod[i] = val[p] * x[td.jlo + k];
                        row[i] = (int)idx[p];
                    } else {
                        prod[i] = 0.0;
                        row[i] = -1;
                    }
                }
            }
        } else {
#pragma unroll
            for (int i = 0; i < ITEMS; ++i) { prod[i] = 0.0; row[i] = -1; }
        }
        // Waves add into the LDS panel one at a time: a fixed order per entry.
        for (int w = 0; w < NW; ++w) {
            if (wave == w) {
#pragma unroll
                for (int i = 0; i < ITEMS; ++i)
                    if (row[i] >= 0)
                        __hip_atomic_fetch_add(&ypan[row[i]], prod[i], __ATOMIC_RELAXED,
                                               __HIP_MEMORY_SCOPE_WORKGROUP);
            }
            __syncthreads();
        }
    }
    __syncthreads();
    double *out = partial + (int64_t)blockIdx.x * panel_rows;
    for (int i = tid; i < panel_rows; i += BLOCK) out[i] = ypan[i];
}

// y[caller row] = sum over the panel's workgroups of their partials, ascending.
__global__ void mv_reduce_f64(const double *__restrict__ partial, int panel_rows,
                              const PanelDesc *__restrict__ panels, int64_t rows,
                              const int32_t *__restrict__ inv, double *__restrict__ y)
{
    const int64_t r = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (r >= rows) return;
    const int p = (int)(r / panel_rows);
    const int local = (int)(r - (int64_t)p * panel_rows);
    const PanelDesc pd = panels[p];
    double s = 0.0;
    const double *src = partial + (int64_t)pd.wg0 * panel_rows + local;
    for (int w = 0; w < pd.nwg; ++w) s += src[(int64_t)w * panel_rows];
    y[inv ? inv[r] : r] = s;
}

constexpr int VTM_BLOCK = 256;
constexpr int VTM_CHUNK = 4096;
constexpr int MV_BLOCK = 512;
constexpr int MV_ITEMS = 8;
constexpr int MV_SLICE = 4160;

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

}  // namespace

int64_t mv_lds_rows_limit(spw_dtype vdt, int32_t k)
{
    (void)vdt;
    const int64_t lds = 160 * 1024 - MV_SLICE * 4 - 256;
    return lds / (8 * std::max<int32_t>(k, 1));
}
int64_t mv_tile_nnz() { return (int64_t)MV_BLOCK * MV_ITEMS; }
int64_t vtm_chunk_default() { return VTM_CHUNK; }

int device_cu_count(int device)
{
    int cus = 0;
    if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, device) != hipSuccess) return 256;
    return cus > 0 ? cus : 256;
}

int launch_vtm(const spw_matrix_s &A, spw_dtype vdt, int32_t k, const void *v, int64_t ldv, void *u,
               int64_t ldu, void *stream_)
{
    hipStream_t stream = (hipStream_t)stream_;
    if (vdt != SPW_F64 || k != 1 || ldv != 1 || ldu != 1 || A.value_storage != SPW_F64)
        return (int)hipErrorNotSupported;
    double *uo = (double *)u;
    if (A.cols == 0) return 0;
    if (A.nnz == 0) {
        ProfScope ps(stream, "fill_f64");
        hipLaunchKernelGGL(fill_f64, dim3(blocks_for(A.cols, 256)), dim3(256), 0, stream, uo, A.cols, 0.0);
        return (int)hipGetLastError();
    }
    const double *vin = (const double *)v;
    if (A.relabeled) {
        ProfScope ps(stream, "gather_f64");
        hipLaunchKernelGGL(gather_f64, dim3(blocks_for(A.rows, 256)), dim3(256), 0, stream, A.d_inv, A.rows,
                           vin, (double *)A.scratch.vperm);
        vin = (const double *)A.scratch.vperm;
    }
    {
        ProfScope ps(stream, "vtm_chunk_f64");
        if (A.zp.chunk != VTM_CHUNK) return (int)hipErrorNotSupported;
        if (A.idx_kind == IdxKind::U16)
            hipLaunchKernelGGL((vtm_chunk_f64<VTM_BLOCK, VTM_CHUNK, uint16_t>), dim3((unsigned)A.zp.n_chunks),
                               dim3(VTM_BLOCK), 0, stream, A.d_ptr, (const uint16_t *)A.d_idx,
                               (const double *)A.d_val, A.d_owned, A.nnz, vin, uo, A.scratch.carry);
        else
            hipLaunchKernelGGL((vtm_chunk_f64<VTM_BLOCK, VTM_CHUNK, int32_t>), dim3((unsigned)A.zp.n_chunks),
                               dim3(VTM_BLOCK), 0, stream, A.d_ptr, (const int32_t *)A.d_idx,
                               (const double *)A.d_val, A.d_owned, A.nnz, vin, uo, A.scratch.carry);
        int e = (int)hipGetLastError();
        if (e) return e;
    }
    if (A.n_zones > 0) {
        ProfScope ps(stream, "zone_fixup_f64");
        hipLaunchKernelGGL(zone_fixup_f64, dim3(blocks_for(A.n_zones, 256)), dim3(256), 0, stream, A.d_zone_col,
                           A.d_zone_first, A.d_zone_last, A.n_zones, A.scratch.carry, uo);
        int e = (int)hipGetLastError();
        if (e) return e;
    }
    return 0;
}

int launch_mv(const spw_matrix_s &A, spw_dtype vdt, int32_t k, const void *x, int64_t ldx, void *y,
              int64_t ldy, void *stream_)
{
    hipStream_t stream = (hipStream_t)stream_;
    if (vdt != SPW_F64 || k != 1 || ldx != 1 || ldy != 1 || A.value_storage != SPW_F64)
        return (int)hipErrorNotSupported;
    double *yo = (double *)y;
    if (A.rows == 0) return 0;
    if (A.mv_wgs > 0) {
        ProfScope ps(stream, "mv_panel_f64");
        const size_t lds = (size_t)A.panel_rows * 8 + (size_t)MV_SLICE * 4;
        static bool attr_set = false;
        if (!attr_set) {
            const int cap = 160 * 1024;
            (void)hipFuncSetAttribute((const void *)mv_panel_f64<MV_BLOCK, MV_ITEMS, MV_SLICE, uint16_t>,
                                      hipFuncAttributeMaxDynamicSharedMemorySize, cap);
            (void)hipFuncSetAttribute((const void *)mv_panel_f64<MV_BLOCK, MV_ITEMS, MV_SLICE, int32_t>,
                                      hipFuncAttributeMaxDynamicSharedMemorySize, cap);
            attr_set = true;
        }
        if (A.idx_kind == IdxKind::U16)
            hipLaunchKernelGGL((mv_panel_f64<MV_BLOCK, MV_ITEMS, MV_SLICE, uint16_t>), dim3((unsigned)A.mv_wgs),
                               dim3(MV_BLOCK), lds, stream, A.d_pptr, A.cols + 1, (const uint16_t *)A.d_pidx,
                               (const double *)A.d_pval, A.d_tiles, A.d_wgs, (const double *)x,
                               A.scratch.partial, (int)A.panel_rows);
        else
            hipLaunchKernelGGL((mv_panel_f64<MV_BLOCK, MV_ITEMS, MV_SLICE, int32_t>), dim3((unsigned)A.mv_wgs),
                               dim3(MV_BLOCK), lds, stream, A.d_pptr, A.cols + 1, (const int32_t *)A.d_pidx,
                               (const double *)A.d_pval, A.d_tiles, A.d_wgs, (const double *)x,
                               A.scratch.partial, (int)A.panel_rows);
        int e = (int)hipGetLastError();
        if (e) return e;
    }
    {
        ProfScope ps(stream, "mv_reduce_f64");
        hipLaunchKernelGGL(mv_reduce_f64, dim3(blocks_for(A.rows, 256)), dim3(256), 0, stream, A.scratch.partial,
                           (int)A.panel_rows, A.d_panels, A.rows, A.relabeled ? A.d_inv : nullptr, yo);
        int e = (int)hipGetLastError();
        if (e) return e;
    }
    return 0;
}

}  // namespace spw
