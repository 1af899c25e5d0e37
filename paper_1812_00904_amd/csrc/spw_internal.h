// Internal declarations shared by the host and device halves of libspw.
//
// Storage model.  Every matrix is held as the column-major (CSC) arrays of a
// short-by-long matrix B with `rows` (the short dimension) and `cols` (the
// long one): a wide CSC input is B = A, a tall CSR input is B = A^T (the
// role swap of Section II).  Then
//     wide  A x   = scatter product  (B x)          -- "mv" kernels
//     wide  v^T A = column dots      (v^T B)        -- "vtm" kernels
//     tall  A x   = column dots of B with x
//     tall  v^T A = scatter product of B with v
#pragma once

#include <cstdint>
#include <exception>
#include <map>
#include <mutex>
#include <new>
#include <string>
#include <utility>
#include <vector>

#include "spw.h"

namespace spw {

// ---------------------------------------------------------------- plan (host)

// Column-dot plan over equal-nonzero chunks (Section II's split with a fixed
// chunk size instead of a fixed count).  Chunk c covers positions
// [c*C, min((c+1)*C, nnz)); it owns the columns whose start lies inside it
// (owned[c] .. owned[c+1]-1; owned[n_chunks] = cols).  A zone is a column cut
// by a chunk boundary; its chunk set is first..last (inclusive).
struct ZonePlan {
    int64_t chunk = 0;
    int64_t n_chunks = 0;
    std::vector<int32_t> owned;       // n_chunks + 1
    std::vector<int32_t> jlo, jhi;    // per chunk: columns holding its first / last position
    std::vector<int32_t> zone_col;    // per zone
    std::vector<int32_t> zone_first;  // first chunk (holds the column start)
    std::vector<int32_t> zone_last;   // last chunk touching the column
};

// Builds the zone plan; ptr has cols+1 entries.  Pure host code.
void build_zone_plan(int64_t cols, const int64_t *ptr, int64_t chunk, ZonePlan &out);

// Panel of the scatter product: the internal rows row0, row0 + P, row0 + 2P, ...
// (rows of them; P panels, row0 = panel index), at panel-local rows 0, 1, 2, ...;
// workgroups [wg0, wg0+nwg) hold its partial vectors.
struct PanelDesc {
    int32_t row0, rows, wg0, nwg;
};

// ------------------------------------------------------------ device handle

enum class IdxKind : int32_t { U16 = 0, I32 = 1 };

// Column-dot storage of a short-by-long CSC matrix: int32 column starts (plus
// a padding window), 2- or 4-byte rows and values in the storage type (8, 4
// or 2 bytes), both interleaved inside each chunk (see the column-dot kernel),
// column-start bits and segment tables per chunk, the chunk/zone plan and the
// columns without nonzeros.
struct ColDot {
    int64_t rows = 0, cols = 0, nnz = 0;
    IdxKind idx_kind = IdxKind::U16;
    void *d_idx = nullptr;
    void *d_val = nullptr;
    ZonePlan zp;
    int32_t *d_empty = nullptr;
    int64_t n_empty = 0;
    int32_t *d_zone_col = nullptr, *d_zone_first = nullptr, *d_zone_last = nullptr;
    int64_t n_zones = 0;
    int32_t *d_wchunks = nullptr;       // column partitioning: first chunk of each worker (n_workers+1)
    int64_t n_workers = 0;              // workers (waves) of the single-vector column dots
    int64_t worker_max_nnz = 0, worker_min_nnz = 0;
    uint16_t *d_heads = nullptr;        // per chunk and lane: column-start bits of the lane's positions
    int32_t *d_cinfo = nullptr;         // per chunk: first column, first segment, segments, flags
    int32_t *d_segcol = nullptr;        // per chunk segment: its column
    bool built = false;
};

// Workspace of the CGLS loop (allocated on its first call, kept until destroy).
struct CglsScratch {
    double *r = nullptr, *q = nullptr, *t = nullptr;   // m entries each
    double *s = nullptr, *p = nullptr;        // n entries each
    double *partial = nullptr;                // partial sums of one inner product
    double *scal = nullptr;                   // gamma, alpha, beta
    double *hist = nullptr;                   // hist_cap entries: gamma history, then rho history
    int64_t hist_cap = 0;
};

struct Scratch {
    double *partial = nullptr;    // mv_wgs * panel_rows  (binary64 partial sums of one column)
    double *partial_cols = nullptr;   // pcols * mv_wgs * panel_rows (multi-column scatter launches)
    int32_t pcols = 0;
    double *carry = nullptr;      // 2 * max chunks * kcap
    int64_t carry_chunks = 0;     // the chunk count the carries were sized for
    double *vperm = nullptr;      // rows * kcap elements of 8 bytes (renumbered input of the column dots)
    int32_t kcap = 0;
};

}  // namespace spw

struct spw_matrix_s {
    spw_format format = SPW_CSC;
    spw_dtype value_storage = SPW_F64;
    spw_partition partition = SPW_PART_NONZERO;
    int64_t m = 0, n = 0, nnz = 0;      // caller's shape
    int64_t rows = 0, cols = 0;         // B = short x long
    int device = 0;
    int32_t relabeled = 0;
    int32_t *d_rank = nullptr;          // rows: caller row -> internal row
    int32_t *d_inv = nullptr;           // rows: internal row -> caller row

    spw::ColDot cd;                     // B itself (renumbered rows)
    // Column-dot workgroup size per vector type ([0] binary64, [1] binary32):
    // 0 = the default rule, else 256 / 512 / 1024 (wg_size or the tuner's).
    int32_t vtm_block[2] = {0, 0};
    int32_t autotune = 0;
    int32_t tuned = 0;                  // chunk / workgroup sizes from the tuner (timed or cached)
    uint64_t fingerprint = 0;           // tuning-cache key (spw_tune.cpp)
    // Multi-RHS plans chosen per (direction, vector type, k): set by the
    // caller or the tuner (spw_plan values); absent = the fixed rule.
    std::mutex plan_mu;
    std::map<int64_t, int32_t> plans;
    // B^T (caller's numbering), for multi-RHS scatter products, in blocks of
    // TRANSPOSE_BLOCK_ROWS of its rows: column b*rows + i of cdt holds the
    // entries of B's row i in B's columns b*R .. (b+1)*R-1
    spw::ColDot cdt;
    int64_t cdt_blocks = 1;
    double *cdt_partial = nullptr;      // cdt.cols x k binary64 partial sums (cdt_blocks > 1)
    int64_t cdt_partial_elems = 0;

    // scatter-product storage: row panels; inside a panel, per workgroup column
    // range and per wave (a set of the panel's rows), blocks of 512 nonzeros
    int64_t panel_rows = 0, n_panels = 0;
    uint32_t *d_mpacked = nullptr;      // (panel-local row << 16) | (column - block column base)
    void *d_mval = nullptr;             // values in the storage type, interleaved like d_mpacked
    int32_t *d_mblocks = nullptr;       // per block: column base, count
    int32_t *d_wg_blk = nullptr;        // per workgroup: waves+1 offsets into the blocks
    int64_t n_mblocks = 0;
    std::vector<spw::PanelDesc> panels;
    spw::PanelDesc *d_panels = nullptr;
    int64_t mv_wgs = 0;

    spw::Scratch scratch;
    spw::CglsScratch cgls;
    int64_t device_bytes = 0;
    std::vector<std::pair<void *, int64_t>> allocations;   // device buffers and their sizes

    // The stream of the last product call and an event recorded after it: a
    // call on another stream while that event is pending would race on the
    // scratch, and is refused (SPW_ERR_BUSY).
    std::mutex use_mu;
    void *last_stream = nullptr;
    void *last_done = nullptr;          // hipEvent_t, created on first use
    bool used = false;
};

namespace spw {

// ------------------------------------------------------------ launch glue
// All return hipError_t as int (0 = success).  Implemented in spw_kernels.hip.

// Single-vector column dots (u = B^T v) over A.cd.
int launch_vtm(const spw_matrix_s &A, spw_dtype vdt, const void *v, void *u, void *stream);
// Column dots for k <= 8 columns in one pass: column c reads in[c] (stride
// ldi[c]) and writes out[c] (stride ldo[c]); in/out/ldi/ldo are host arrays.
// Every column is bit-identical to launch_vtm on it.
int launch_vtm_cols(const spw_matrix_s &A, spw_dtype vdt, int32_t k, const void *const *in, const int64_t *ldi,
                    void *const *out, const int64_t *ldo, void *stream);
// Column dots for k columns of row-major V (ldv) into U (ldu), at most 8
// columns per pass; every column is bit-identical to launch_vtm on it.
int launch_vtm_multi(const spw_matrix_s &A, spw_dtype vdt, int32_t k, const void *v, int64_t ldv, void *u,
                     int64_t ldu, void *stream);
// Scatter products for k <= 8 columns with their own bases and strides (host
// arrays): one pass over the matrix for all k when the multi-column partial
// sums hold k columns (grow_partial_cols), else one pass per column.  Every
// column is bit-identical to the single-column product on it.
int launch_mv_cols(const spw_matrix_s &A, spw_dtype vdt, int32_t k, const void *const *in, const int64_t *ldi,
                   void *const *out, const int64_t *ldo, void *stream);
// Scatter product y = B x, k times over strided columns of X (ldx) and Y (ldy);
// every column is bit-identical to the k = 1 product on it.
int launch_mv(const spw_matrix_s &A, spw_dtype vdt, int32_t k, const void *x, int64_t ldx,
              void *y, int64_t ldy, void *stream);
// The chunk-per-wave column dots address a chunk's outputs through a buffer
// view of up to 1,024 columns x ld entries x 8 bytes, which must stay below
// 2^31 bytes: their output leading dimension must be below this.
constexpr int64_t CHUNK_OUT_LD_LIMIT = (int64_t)1 << 18;
// Lanes per nonzero of the multi-RHS column dots: the power of two >= k.
// A renumbered copy of V is stored with this row stride, so the scratch
// (Scratch::kcap) must be grown to it before the call.
inline int32_t coldot_tile_width(int32_t k)
{
    int32_t L = 1;
    while (L < k) L <<= 1;
    return L;
}
// Multi-RHS column dots over C (U = C^T V): V is C.rows x k, U is C.cols x k.
// inv renumbers the rows of V (NULL when C uses the caller's numbering).
// out_f64: U holds binary64 whatever vdt is (the blocked transpose's partial sums).
int launch_coldot_batch(const spw_matrix_s &A, const ColDot &C, const int32_t *inv, spw_dtype vdt, int32_t k,
                        const void *V, int64_t ldv, void *U, int64_t ldu, void *stream, bool out_f64 = false);
// out (rows x k, leading dimension ldo, type vdt) = the sum of nb binary64 blocks
// of rows x k partial sums (block b at P + b*rows*k, row stride k), in block order.
int launch_sum_blocks(spw_dtype vdt, int64_t nb, int64_t rows, int32_t k, const double *P, void *out, int64_t ldo,
                      void *stream);
// Rows of the long side per block of the kept transpose: a block's slice of a
// 64-column binary64 input is 128 MiB, which the Infinity Cache holds.
constexpr int64_t TRANSPOSE_BLOCK_ROWS = (int64_t)1 << 18;
// Fills rows x k of a row-major block (leading dimension ld) with zeros.
int launch_zero_fill(spw_dtype vdt, int32_t k, void *out, int64_t ld, int64_t rows, void *stream);
// Device-side limits the host plan must respect.
int64_t mv_lds_rows_limit(spw_dtype vdt, int32_t k);
int64_t mv_block_nnz();
int64_t mv_waves();
int64_t vtm_chunk_default();
// Column-dot chunk sizes the kernels take (512 or 1,024 nonzeros).
bool vtm_chunk_supported(int64_t chunk);
// Waves the single-vector column-dot kernel runs for nchunks chunks on device.
int64_t vtm_workers(int device, int64_t nchunks);
int64_t vtm_hot_rows_limit(spw_dtype vdt);
int device_cu_count(int device);

// CGLS vector steps (spw_solve.hip).  x and p have n entries, b, r and q
// have m; hist_gamma / hist_rho receive the inner products of iteration k.
struct CglsWork {
    int64_t m = 0, n = 0;
    const double *b = nullptr;
    double *x = nullptr, *r = nullptr, *q = nullptr, *t = nullptr, *s = nullptr, *p = nullptr;
    double *partial = nullptr, *scal = nullptr, *hist_gamma = nullptr, *hist_rho = nullptr;
};
// The steps around the two products of a CGLS iteration.  An iteration takes
// t = A s (s = A^T r of the previous step) and forms q = A p by linearity,
// q = t + beta q, so that the long vector update (p, then x) runs just before
// the A^T r product rather than just before the A p product.
enum class CglsVecOp : int {
    R_INIT,      // r = b - q (q = A x_0); rho_0 = ||r||^2
    GAMMA0,      // gamma_0 = ||s||^2 (s = A^T r_0)
    ALPHA_R0,    // first iteration: q = t; alpha = gamma / ||q||^2; r = r - alpha q; rho_k = ||r||^2
    ALPHA_R,     // q = t + beta q; alpha = gamma / ||q||^2; r = r - alpha q; rho_k = ||r||^2
    PX0,         // first iteration: p = s; x = x + alpha p
    PX,          // p = s + beta p; x = x + alpha p
    P,           // p = s + beta p          (an iteration that forms q = A p directly)
    X,           // x = x + alpha p
    GAMMA        // gamma_k = ||s||^2 (s = A^T r); beta = gamma_k / gamma_{k-1}
};
// The history index advances on the device (see spw_solve.hip), so the
// launches of one iteration are the same every time.
int launch_cgls_vec(CglsVecOp op, const CglsWork &w, void *stream);
int64_t cgls_dot_parts();

// Profiling hooks (spw_profile.cpp).
bool profile_on();
void profile_begin(void *stream, const char *name, void **token);
void profile_end(void *stream, void *token);

// Tuning cache (spw_tune.cpp): fingerprint of a matrix's shape and structure,
// and the recorded choices.  tune_put returns false if the cache file could
// not be written (the record stays in memory).
uint64_t matrix_fingerprint(spw_format fmt, spw_dtype storage, int64_t m, int64_t n, int64_t nnz,
                            const int64_t *ptr, const int32_t *idx);
bool tune_get(uint64_t fp, const std::string &key, int32_t *value);
bool tune_put(uint64_t fp, const std::string &key, int32_t value);

// Error text for the calling thread (spw_api.cpp).
void set_error(const std::string &msg);

// Runs the body of an exported function and turns a C++ exception into a
// status (host memory exhausted, a thread that cannot start, ...), so that
// nothing is thrown across the C ABI.
template <typename F>
spw_status guarded(const char *fname, F &&body) noexcept
{
    try {
        return body();
    } catch (const std::bad_alloc &) {
        try { set_error(std::string(fname) + ": out of host memory"); } catch (...) {}
        return SPW_ERR_OUT_OF_MEMORY;
    } catch (const std::exception &e) {
        try { set_error(std::string(fname) + ": " + e.what()); } catch (...) {}
        return SPW_ERR_DEVICE;
    } catch (...) {
        try { set_error(std::string(fname) + ": unexpected C++ exception"); } catch (...) {}
        return SPW_ERR_DEVICE;
    }
}

// Makes the handle's scratch hold k-wide carries and renumbered inputs (and
// the one-column partial sums); growing waits for the device (spw_api.cpp).
spw_status grow_scratch(spw_matrix_s &A, int32_t k);
// Partial sums for scatter launches of up to cols columns (spw_api.cpp).
spw_status grow_partial_cols(spw_matrix_s &A, int32_t cols);

}  // namespace spw
