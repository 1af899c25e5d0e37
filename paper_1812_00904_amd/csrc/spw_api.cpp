// C ABI of libspw: matrix creation (validation, row renumbering, chunk/zone
// plan, row panels), products, and error reporting.  See include/spw.h.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <exception>
#include <memory>
#include <numeric>
#include <string>
#include <system_error>
#include <thread>
#include <vector>

#include "spw_internal.h"

namespace spw {

static thread_local std::string t_err;
void set_error(const std::string &msg) { t_err = msg; }

namespace {

// Runs part(t) for t = 0 .. nparts-1 on host threads.  A part whose thread
// cannot be started runs on the calling thread; every thread is joined before
// the first exception any part threw is rethrown here, so no exception escapes
// a worker thread.
template <typename F>
void run_parts(int64_t nparts, F &&part)
{
    std::vector<std::exception_ptr> errs((size_t)std::max<int64_t>(nparts, 0));
    std::vector<std::thread> th;
    th.reserve(errs.size());
    auto body = [&part, &errs](int64_t t) {
        try {
            part(t);
        } catch (...) {
            errs[(size_t)t] = std::current_exception();
        }
    };
    for (int64_t t = 0; t < nparts; ++t) {
        try {
            th.emplace_back(body, t);
        } catch (const std::system_error &) {
            body(t);
        }
    }
    for (auto &t : th) t.join();
    for (auto &e : errs)
        if (e) std::rethrow_exception(e);
}

template <typename F>
void parallel_for(int64_t n, F &&f)
{
    int nt = (int)std::min<unsigned>(16u, std::max(1u, std::thread::hardware_concurrency()));
    if (n < (int64_t)1 << 16 || nt == 1) {
        f((int64_t)0, n);
        return;
    }
    const int64_t per = (n + nt - 1) / nt;
    run_parts(nt, [&](int64_t t) {
        const int64_t a = t * per, b = std::min(n, a + per);
        if (a < b) f(a, b);
    });
}

spw_status fail(spw_status s, const std::string &msg)
{
    set_error(msg);
    return s;
}

int64_t round_up(int64_t a, int64_t b) { return (a + b - 1) / b * b; }

// Device allocation owned by the matrix (freed in spw_destroy).
template <typename T>
spw_status dev_alloc(spw_matrix_s &A, T **out, int64_t count, const char *what)
{
    *out = nullptr;
    const size_t bytes = (size_t)std::max<int64_t>(count, 1) * sizeof(T);
    void *p = nullptr;
    if (hipMalloc(&p, bytes) != hipSuccess) {
        (void)hipGetLastError();
        return fail(SPW_ERR_OUT_OF_MEMORY, std::string("hipMalloc failed for ") + what + " (" +
                                               std::to_string(bytes) + " bytes)");
    }
    A.allocations.emplace_back(p, (int64_t)bytes);
    A.device_bytes += (int64_t)bytes;
    *out = (T *)p;
    return SPW_OK;
}

// Copies host arrays to the device in pieces through a ring of pinned
// staging slots on a stream of its own: put() returns once the last piece is
// staged (the caller may then free its array), so the copy of one array runs
// while the host builds the next.  Arrays below one slot, and every array
// when no pinned memory can be had, are copied synchronously.  finish()
// waits for every copy; the destructor does too, before the slots go.
class Uploader {
public:
    static constexpr size_t SLOT = (size_t)32 << 20;
    static constexpr int NSLOT = 4;
    ~Uploader()
    {
        (void)finish();
        for (int i = 0; i < NSLOT; ++i) {
            if (ev_[i]) (void)hipEventDestroy(ev_[i]);
            if (slot_[i]) (void)hipHostFree(slot_[i]);
        }
        if (s_) (void)hipStreamDestroy(s_);
    }
    spw_status put(void *dst, const void *src, size_t bytes, const char *what)
    {
        if (bytes == 0) return SPW_OK;
        if (bytes < SLOT || !ready()) {
            if (hipMemcpy(dst, src, bytes, hipMemcpyHostToDevice) != hipSuccess) {
                (void)hipGetLastError();
                return fail(SPW_ERR_DEVICE, std::string("hipMemcpy to device failed for ") + what);
            }
            return SPW_OK;
        }
        for (size_t off = 0; off < bytes; off += SLOT) {
            const size_t n = std::min(SLOT, bytes - off);
            const int i = next_;
            next_ = (next_ + 1) % NSLOT;
            if (used_[i] && hipEventSynchronize(ev_[i]) != hipSuccess) return device_error(what);
            // stage the piece with several host threads, then hand it to the DMA engine
            char *slot = static_cast<char *>(slot_[i]);
            const char *from = static_cast<const char *>(src) + off;
            parallel_for((int64_t)n, [&](int64_t a, int64_t b) { std::memcpy(slot + a, from + a, (size_t)(b - a)); });
            if (hipMemcpyAsync(static_cast<char *>(dst) + off, slot, n, hipMemcpyHostToDevice, s_) != hipSuccess ||
                hipEventRecord(ev_[i], s_) != hipSuccess)
                return device_error(what);
            used_[i] = true;
        }
        return SPW_OK;
    }
    spw_status finish()
    {
        if (s_ && hipStreamSynchronize(s_) != hipSuccess) return device_error("the staged copies");
        return SPW_OK;
    }

private:
    bool ready()
    {
        if (tried_) return s_ != nullptr;
        tried_ = true;
        hipStream_t s = nullptr;
        if (hipStreamCreateWithFlags(&s, hipStreamNonBlocking) != hipSuccess) {
            (void)hipGetLastError();
            return false;
        }
        for (int i = 0; i < NSLOT; ++i)
            if (hipHostMalloc(&slot_[i], SLOT, hipHostMallocDefault) != hipSuccess ||
                hipEventCreateWithFlags(&ev_[i], hipEventDisableTiming) != hipSuccess) {
                (void)hipGetLastError();
                s_ = s;   // the destructor releases what was made
                (void)finish();
                for (int k = 0; k < NSLOT; ++k) {
                    if (ev_[k]) (void)hipEventDestroy(ev_[k]);
                    if (slot_[k]) (void)hipHostFree(slot_[k]);
                    ev_[k] = nullptr;
                    slot_[k] = nullptr;
                }
                (void)hipStreamDestroy(s);
                s_ = nullptr;
                return false;
            }
        s_ = s;
        return true;
    }
    spw_status device_error(const char *what)
    {
        (void)hipGetLastError();
        return fail(SPW_ERR_DEVICE, std::string("staged copy to device failed for ") + what);
    }
    hipStream_t s_ = nullptr;
    void *slot_[NSLOT] = {};
    hipEvent_t ev_[NSLOT] = {};
    bool used_[NSLOT] = {};
    int next_ = 0;
    bool tried_ = false;
};

// The uploader of the spw_create running on this thread (NULL outside one).
thread_local Uploader *t_uploader = nullptr;

spw_status h2d(void *dst, const void *src, size_t bytes, const char *what)
{
    if (bytes == 0) return SPW_OK;
    if (t_uploader) return t_uploader->put(dst, src, bytes, what);
    if (hipMemcpy(dst, src, bytes, hipMemcpyHostToDevice) != hipSuccess) {
        (void)hipGetLastError();
        return fail(SPW_ERR_DEVICE, std::string("hipMemcpy to device failed for ") + what);
    }
    return SPW_OK;
}

void free_all(spw_matrix_s *A)
{
    for (auto &a : A->allocations) (void)hipFree(a.first);
    A->allocations.clear();
}

// Frees one device buffer of the matrix and forgets it.
void free_one(spw_matrix_s &A, void *p)
{
    if (!p) return;
    for (size_t i = 0; i < A.allocations.size(); ++i)
        if (A.allocations[i].first == p) {
            A.device_bytes -= A.allocations[i].second;
            A.allocations.erase(A.allocations.begin() + (long)i);
            break;
        }
    (void)hipFree(p);
}

// Frees the device arrays of a column-dot storage and resets it.
void free_coldot(spw_matrix_s &A, ColDot &C)
{
    for (void *p : {C.d_idx, C.d_val, (void *)C.d_empty, (void *)C.d_zone_col, (void *)C.d_zone_first,
                    (void *)C.d_zone_last, (void *)C.d_wchunks, (void *)C.d_heads, (void *)C.d_cinfo,
                    (void *)C.d_segcol})
        free_one(A, p);
    C = ColDot();
}

spw_status validate(int64_t outer, int64_t inner, int64_t nnz, const int64_t *ptr, const int32_t *idx,
                    const char *outer_name)
{
    if (ptr[0] != 0) return fail(SPW_ERR_BAD_MATRIX, "ptr[0] must be 0, got " + std::to_string(ptr[0]));
    if (ptr[outer] != nnz)
        return fail(SPW_ERR_BAD_MATRIX, "ptr[" + std::to_string(outer) + "] must equal nnz = " +
                                            std::to_string(nnz) + ", got " + std::to_string(ptr[outer]));
    for (int64_t j = 0; j < outer; ++j)
        if (ptr[j + 1] < ptr[j])
            return fail(SPW_ERR_BAD_MATRIX, std::string("ptr decreases at ") + outer_name + " " + std::to_string(j));
    // indices: in range and strictly increasing inside each column (row)
    std::vector<int64_t> bad((size_t)std::min<int64_t>(16, std::max<int64_t>(outer, 1)), -1);
    const int64_t nparts = (int64_t)bad.size();
    const int64_t per = (outer + nparts - 1) / std::max<int64_t>(nparts, 1);
    run_parts(nparts, [&](int64_t t) {
        const int64_t a = t * per, b = std::min(outer, a + per);
        for (int64_t j = a; j < b; ++j) {
            for (int64_t p = ptr[j]; p < ptr[j + 1]; ++p) {
                const int32_t r = idx[p];
                if (r < 0 || r >= inner || (p > ptr[j] && idx[p - 1] >= r)) {
                    bad[(size_t)t] = p;
                    return;
                }
            }
        }
    });
    for (int64_t b : bad) {
        if (b >= 0) {
            const int32_t r = idx[b];
            std::string why = (r < 0 || r >= inner) ? "index " + std::to_string(r) + " out of range [0, " +
                                                          std::to_string(inner) + ")"
                                                    : "indices not strictly increasing inside a " +
                                                          std::string(outer_name);
            return fail(SPW_ERR_BAD_MATRIX, "position " + std::to_string(b) + ": " + why);
        }
    }
    return SPW_OK;
}

// ------------------------------------------------------------ value storage
// Stored values are rounded once from the given binary64 value to nearest,
// ties to even.  binary32: the C conversion (round-to-nearest-even is the
// default mode).  bfloat16 (8 significant bits, binary32's exponent range,
// gradual underflow down to 2^-133): rounded directly from the binary64 bits,
// so there is no double rounding through binary32.
int64_t storage_bytes(spw_dtype t) { return t == SPW_F64 ? 8 : t == SPW_F32 ? 4 : 2; }

// Returns false when the rounded value is not finite.
bool round_f32(double x, double *out)
{
    const float f = (float)x;
    *out = (double)f;
    return std::isfinite(f) || !std::isfinite(x);
}

bool round_bf16(double x, double *out)
{
    uint64_t b;
    std::memcpy(&b, &x, 8);
    const uint64_t mag = b & 0x7FFFFFFFFFFFFFFFull;
    const int bexp = (int)(mag >> 52);
    if (bexp == 0x7FF) {                      // inf / nan stay as they are
        *out = x;
        return true;
    }
    if (mag == 0 || bexp == 0) {              // zero or a binary64 subnormal (far below 2^-134)
        *out = std::copysign(0.0, x);
        return true;
    }
    const int e = bexp - 1023;                // x = sig * 2^(e-52), sig in [2^52, 2^53)
    const uint64_t sig = (mag & ((1ull << 52) - 1)) | (1ull << 52);
    const int qe = std::max(e, -126) - 7;     // exponent of the last kept bit
    const int drop = qe - (e - 52);           // low bits of sig below that bit (>= 45)
    uint64_t q = 0;
    if (drop < 64) {
        q = sig >> drop;
        const uint64_t rem = sig & ((1ull << drop) - 1), half = 1ull << (drop - 1);
        if (rem > half || (rem == half && (q & 1))) ++q;
    }
    const double r = std::ldexp((double)q, qe);
    *out = std::copysign(r, x);
    return r <= 3.3895313892515355e38;        // largest finite bfloat16, (2 - 2^-7) * 2^127
}

// Rounds n values to `storage`; on overflow returns the first bad position.
int64_t round_values(spw_dtype storage, int64_t n, const double *in, double *out)
{
    std::vector<int64_t> bad(16, -1);
    const int64_t per = (n + 15) / 16;
    run_parts(16, [&](int64_t t) {
        const int64_t a = t * per, b = std::min(n, a + per);
        for (int64_t p = a; p < b; ++p) {
            double r = in[p];
            const bool ok = storage == SPW_F32 ? round_f32(in[p], &r)
                                               : storage == SPW_BF16 ? round_bf16(in[p], &r) : true;
            out[p] = r;
            if (!ok && bad[(size_t)t] < 0) bad[(size_t)t] = p;
        }
    });
    for (int64_t v : bad)
        if (v >= 0) return v;
    return -1;
}

// Writes rounded value r (exactly representable in `storage`) at element slot.
void put_value(spw_dtype storage, void *base, int64_t slot, double r)
{
    if (storage == SPW_F64) {
        static_cast<double *>(base)[slot] = r;
    } else if (storage == SPW_F32) {
        static_cast<float *>(base)[slot] = (float)r;
    } else {
        const float f = (float)r;
        uint32_t u;
        std::memcpy(&u, &f, 4);
        static_cast<uint16_t *>(base)[slot] = (uint16_t)(u >> 16);
    }
}

struct DeviceGuard {
    int prev = -1;
    bool changed = false;
    spw_status st = SPW_OK;
    explicit DeviceGuard(int dev)
    {
        if (hipGetDevice(&prev) != hipSuccess) {
            (void)hipGetLastError();
            st = fail(SPW_ERR_DEVICE, "hipGetDevice failed (no usable GPU?)");
            return;
        }
        if (dev >= 0 && dev != prev) {
            if (hipSetDevice(dev) != hipSuccess) {
                (void)hipGetLastError();
                st = fail(SPW_ERR_DEVICE, "hipSetDevice(" + std::to_string(dev) + ") failed");
                return;
            }
            changed = true;
        }
    }
    ~DeviceGuard()
    {
        if (changed) (void)hipSetDevice(prev);
    }
};

// One stream at a time per matrix: a call on another stream than the last
// call's, while the last call's work is still pending, returns SPW_ERR_BUSY.
// Work being captured into a graph is ordered by the caller and is not tracked.
bool capturing(void *stream)
{
    hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
    const bool yes = hipStreamIsCapturing((hipStream_t)stream, &cs) == hipSuccess && cs != hipStreamCaptureStatusNone;
    (void)hipGetLastError();
    return yes;
}

spw_status claim_stream(spw_matrix_s &A, void *stream, const char *fname)
{
    if (capturing(stream)) return SPW_OK;
    std::lock_guard<std::mutex> lk(A.use_mu);
    if (A.used && stream != A.last_stream && A.last_done) {
        const hipError_t q = hipEventQuery((hipEvent_t)A.last_done);
        if (q == hipErrorNotReady)
            return fail(SPW_ERR_BUSY, std::string(fname) + ": the matrix still has work in flight on another stream");
        if (q != hipSuccess) {
            (void)hipGetLastError();
            return fail(SPW_ERR_DEVICE, std::string(fname) + ": hipEventQuery failed");
        }
    }
    return SPW_OK;
}

// Marks the end of a call's work on stream.
spw_status release_stream(spw_matrix_s &A, void *stream, const char *fname)
{
    if (capturing(stream)) return SPW_OK;
    std::lock_guard<std::mutex> lk(A.use_mu);
    if (!A.last_done) {
        hipEvent_t e;
        if (hipEventCreateWithFlags(&e, hipEventDisableTiming) != hipSuccess) {
            (void)hipGetLastError();
            return fail(SPW_ERR_DEVICE, std::string(fname) + ": hipEventCreate failed");
        }
        A.last_done = e;
    }
    if (hipEventRecord((hipEvent_t)A.last_done, (hipStream_t)stream) != hipSuccess) {
        (void)hipGetLastError();
        return fail(SPW_ERR_DEVICE, std::string(fname) + ": hipEventRecord failed");
    }
    A.last_stream = stream;
    A.used = true;
    return SPW_OK;
}

// Column-dot storage of a rows x cols CSC matrix (ptr over columns, rows[]
// already in the numbering the kernel will use).
spw_status build_coldot(spw_matrix_s &A, ColDot &C, int64_t rows, int64_t cols, const int64_t *ptr,
                        const int32_t *rowi, const double *val, spw_dtype storage, int64_t chunk)
{
    const int64_t nnz = ptr[cols];
    C.rows = rows;
    C.cols = cols;
    C.nnz = nnz;
    C.idx_kind = rows <= 65536 ? IdxKind::U16 : IdxKind::I32;
    spw_status st;
    const int64_t WCH = chunk, ITEMS = WCH / 64;
    const int64_t zpad = round_up(std::max<int64_t>(nnz, 1), 4096);
    // Chunk-interleaved copies: inside each chunk of W = 64*I positions, item i
    // of lane l (position l*I + i) is stored at ((i/G)*64 + l)*G + i%G, G being
    // the number of elements in 16 bytes.
    auto ilv = [&](int64_t p, int64_t G) -> int64_t {
        const int64_t o = p % WCH, cb = p - o, ln = o / ITEMS, i = o % ITEMS;
        return cb + ((i / G) * 64 + ln) * G + i % G;
    };
    if (C.idx_kind == IdxKind::U16) {
        std::vector<uint16_t> ii((size_t)zpad, 0);
        parallel_for(nnz, [&](int64_t a, int64_t b) {
            for (int64_t p = a; p < b; ++p) ii[(size_t)ilv(p, 8)] = (uint16_t)rowi[p];
        });
        uint16_t *d = nullptr;
        if ((st = dev_alloc(A, &d, zpad, "row indices"))) return st;
        if ((st = h2d(d, ii.data(), (size_t)zpad * 2, "row indices"))) return st;
        C.d_idx = d;
    } else {
        std::vector<int32_t> ii((size_t)zpad, 0);
        parallel_for(nnz, [&](int64_t a, int64_t b) {
            for (int64_t p = a; p < b; ++p) ii[(size_t)ilv(p, 4)] = rowi[p];
        });
        int32_t *d = nullptr;
        if ((st = dev_alloc(A, &d, zpad, "row indices"))) return st;
        if ((st = h2d(d, ii.data(), (size_t)zpad * 4, "row indices"))) return st;
        C.d_idx = d;
    }
    {
        const int64_t es = storage_bytes(storage), G = 16 / es;
        std::vector<uint8_t> vi((size_t)(zpad * es), 0);
        parallel_for(nnz, [&](int64_t a, int64_t b) {
            for (int64_t p = a; p < b; ++p) put_value(storage, vi.data(), ilv(p, G), val[p]);
        });
        uint8_t *d = nullptr;
        if ((st = dev_alloc(A, &d, zpad * es, "values"))) return st;
        if ((st = h2d(d, vi.data(), vi.size(), "values"))) return st;
        C.d_val = d;
    }
    build_zone_plan(cols, ptr, WCH, C.zp);
    C.n_zones = (int64_t)C.zp.zone_col.size();
    {
        // Column-start bits (bit i of lane l of chunk c: position c*W + l*I + i
        // is the first nonzero of its column) and per-chunk descriptions: the
        // column of the first position, the chunk's runs ("segments") of
        // positions in one column with the table of their columns, and flags.
        const int64_t nch = C.zp.n_chunks;
        std::vector<uint16_t> heads((size_t)std::max<int64_t>(nch * 64, 1), 0);
        for (int64_t j = 0; j < cols; ++j)
            if (ptr[j] < ptr[j + 1]) {
                const int64_t p = ptr[j], o = p % WCH;
                heads[(size_t)((p / WCH) * 64 + o / ITEMS)] |= (uint16_t)(1u << (o % ITEMS));
            }
        std::vector<int32_t> cinfo((size_t)(4 * std::max<int64_t>(nch, 1)), 0);
        std::vector<int32_t> segcol;
        segcol.reserve((size_t)(cols + nch + 1));
        for (int64_t c = 0; c < nch; ++c) {
            const int64_t cs = c * WCH, ce = std::min(cs + WCH, nnz);
            const int64_t jlo = C.zp.jlo[(size_t)c], jhi = C.zp.jhi[(size_t)c];
            const int64_t seg0 = (int64_t)segcol.size();
            segcol.push_back((int32_t)jlo);
            for (int64_t j = jlo + 1; j <= jhi; ++j)
                if (ptr[j] < ptr[j + 1]) segcol.push_back((int32_t)j);
            const int64_t nseg = (int64_t)segcol.size() - seg0;
            int32_t flags = 0;
            if (ptr[jlo] == cs) flags |= 1;                      // the first position starts its column
            if (ce < nnz && ptr[jhi + 1] > ce) flags |= 2;       // the last column continues
            if (nseg == jhi - jlo + 1) flags |= 4;               // no empty column inside
            int32_t *ci = &cinfo[(size_t)(4 * c)];
            ci[0] = (int32_t)jlo;
            ci[1] = (int32_t)seg0;
            ci[2] = (int32_t)nseg;
            ci[3] = flags;
        }
        if (segcol.size() >= ((size_t)1 << 31)) return fail(SPW_ERR_UNSUPPORTED, "segment table exceeds 2^31 entries");
        if ((st = dev_alloc(A, &C.d_heads, (int64_t)heads.size(), "column-start bits"))) return st;
        if ((st = h2d(C.d_heads, heads.data(), heads.size() * 2, "column-start bits"))) return st;
        if ((st = dev_alloc(A, &C.d_cinfo, (int64_t)cinfo.size(), "chunk descriptions"))) return st;
        if ((st = h2d(C.d_cinfo, cinfo.data(), cinfo.size() * 4, "chunk descriptions"))) return st;
        if ((st = dev_alloc(A, &C.d_segcol, std::max<int64_t>((int64_t)segcol.size(), 1), "segment columns")))
            return st;
        if ((st = h2d(C.d_segcol, segcol.data(), segcol.size() * 4, "segment columns"))) return st;
    }
    {
        std::vector<int32_t> empty;
        for (int64_t j = 0; j < cols; ++j)
            if (ptr[j + 1] == ptr[j]) empty.push_back((int32_t)j);
        C.n_empty = (int64_t)empty.size();
        if ((st = dev_alloc(A, &C.d_empty, std::max<int64_t>(C.n_empty, 1), "empty columns"))) return st;
        if ((st = h2d(C.d_empty, empty.data(), empty.size() * 4, "empty columns"))) return st;
    }
    if ((st = dev_alloc(A, &C.d_zone_col, std::max<int64_t>(C.n_zones, 1), "zone table"))) return st;
    if ((st = dev_alloc(A, &C.d_zone_first, std::max<int64_t>(C.n_zones, 1), "zone table"))) return st;
    if ((st = dev_alloc(A, &C.d_zone_last, std::max<int64_t>(C.n_zones, 1), "zone table"))) return st;
    if ((st = h2d(C.d_zone_col, C.zp.zone_col.data(), (size_t)C.n_zones * 4, "zone table"))) return st;
    if ((st = h2d(C.d_zone_first, C.zp.zone_first.data(), (size_t)C.n_zones * 4, "zone table"))) return st;
    if ((st = h2d(C.d_zone_last, C.zp.zone_last.data(), (size_t)C.n_zones * 4, "zone table"))) return st;
    C.built = true;
    return SPW_OK;
}

// Workers of the single-vector column dots and how much each owns.  Nonzero
// partitioning: worker w reduces chunks w, w+P, ... (the kernel's grid
// stride).  Column partitioning (Section VI's comparison): worker w owns
// columns [j0_w, j1_w), equal counts with the first cols mod P workers one
// more, and reduces the chunks whose first position lies in its columns.
// Merge-path partitioning: the chunks are cut into P contiguous runs of about
// equal cost, a chunk costing its nonzeros plus the columns whose start lies
// in it (empty columns included), so a worker whose chunks hold many short
// or empty columns (many outputs) gets fewer nonzeros.
spw_status plan_workers(spw_matrix_s &A, ColDot &C, const int64_t *ptr, spw_partition part)
{
    const int64_t nch = C.zp.n_chunks, P = vtm_workers(A.device, nch), W = C.zp.chunk;
    C.n_workers = P;
    C.worker_max_nnz = C.worker_min_nnz = 0;
    if (nch == 0) return SPW_OK;
    if (part == SPW_PART_NONZERO) {
        // worker w holds chunks w, w+P, ...; only the last chunk is short
        const int64_t last_len = C.nnz - (nch - 1) * W;
        int64_t mx = -1, mn = -1;
        for (int64_t w = 0; w < std::min<int64_t>(P, nch + 1); ++w) {
            const int64_t cnt = w < nch ? (nch - 1 - w) / P + 1 : 0;
            int64_t z = cnt * W;
            if (cnt > 0 && (nch - 1 - w) % P == 0) z -= W - last_len;    // holds the last chunk
            mx = mx < 0 ? z : std::max(mx, z);
            mn = mn < 0 ? z : std::min(mn, z);
        }
        if (P > nch) mn = 0;
        C.worker_max_nnz = mx;
        C.worker_min_nnz = mn;
        return SPW_OK;
    }
    const int64_t cols = C.cols, q = cols / P, big = cols % P;
    std::vector<int32_t> first((size_t)P + 1, (int32_t)nch);
    int64_t mx = -1, mn = -1, j0 = 0, c = 0;
    if (part == SPW_PART_MERGE) {
        // prefix cost up to chunk c: its positions plus the columns owned by chunks before it
        auto cost_before = [&](int64_t cc) -> int64_t { return std::min(cc * W, C.nnz) + C.zp.owned[(size_t)cc]; };
        const int64_t total = C.nnz + cols;
        int64_t cc = 0;
        for (int64_t w = 0; w < P; ++w) {
            const int64_t target = total * w / P;
            while (cc < nch && cost_before(cc) < target) ++cc;
            first[(size_t)w] = (int32_t)cc;
        }
        for (int64_t w = 0; w < P; ++w) {
            const int64_t a = first[(size_t)w], b = first[(size_t)w + 1];
            const int64_t z = std::min(b * W, C.nnz) - std::min(a * W, C.nnz);
            mx = mx < 0 ? z : std::max(mx, z);
            mn = mn < 0 ? z : std::min(mn, z);
        }
    } else {
    for (int64_t w = 0; w < P; ++w) {
        const int64_t j1 = j0 + (w < big ? q + 1 : q);
        const int64_t z = ptr[j1] - ptr[j0];
        mx = mx < 0 ? z : std::max(mx, z);
        mn = mn < 0 ? z : std::min(mn, z);
        // chunks whose first position's column lies in [j0, j1)
        first[(size_t)w] = (int32_t)c;
        while (c < nch && C.zp.jlo[(size_t)c] < j1) ++c;
        j0 = j1;
    }
    }
    first[(size_t)P] = (int32_t)nch;
    C.worker_max_nnz = mx;
    C.worker_min_nnz = mn;
    spw_status st;
    if ((st = dev_alloc(A, &C.d_wchunks, P + 1, "worker chunk runs"))) return st;
    if ((st = h2d(C.d_wchunks, first.data(), first.size() * 4, "worker chunk runs"))) return st;
    return SPW_OK;
}

// Row panels, wave row sets and blocks of the scatter product (see
// spw_internal.h and the scatter kernel).  rowi holds the internal
// (renumbered) rows.
spw_status build_mv_storage(spw_matrix_s &A, const int64_t *ptr, const int32_t *rowi, const double *val,
                            int64_t panel_rows_opt)
{
    const spw_dtype storage = A.value_storage;
    const int64_t es = storage_bytes(storage), GV = 16 / es;
    const int64_t rows = A.rows, cols = A.cols, nnz = A.nnz;
    const int64_t BLK = mv_block_nnz();
    const int64_t NB = mv_waves();
    const int64_t SPAN = 65536;                 // columns a block may span (16-bit offsets)
    const int64_t limit = mv_lds_rows_limit(SPW_F64, 1);
    int64_t R = rows;
    if (panel_rows_opt > 0) R = std::min<int64_t>(panel_rows_opt, limit);
    else if (rows > limit) {
        const int64_t P = (rows + limit - 1) / limit;
        R = (rows + P - 1) / P;
    }
    R = std::max<int64_t>(std::min(R, rows), 1);
    const int64_t P = (rows + R - 1) / R;
    A.panel_rows = R;
    A.n_panels = P;
    auto row_of = [&](int64_t p) -> int64_t { return (int64_t)rowi[p]; };

    // 1. Column-major order inside each panel: (panel, column) counts, then a
    //    stable scatter of the source positions.
    std::vector<int64_t> pptr((size_t)(P * (cols + 1)), 0);
    std::vector<int64_t> order;
    if (P == 1) {
        for (int64_t j = 0; j <= cols; ++j) pptr[(size_t)j] = ptr[j];
    } else {
        std::vector<int32_t> cnt((size_t)(P * cols), 0);
        parallel_for(cols, [&](int64_t a, int64_t b) {
            for (int64_t j = a; j < b; ++j)
                for (int64_t p = ptr[j]; p < ptr[j + 1]; ++p) cnt[(size_t)(row_of(p) % P * cols + j)]++;
        });
        int64_t run = 0;
        for (int64_t q = 0; q < P; ++q) {
            int64_t *pp = pptr.data() + q * (cols + 1);
            for (int64_t j = 0; j < cols; ++j) {
                pp[j] = run;
                run += cnt[(size_t)(q * cols + j)];
            }
            pp[cols] = run;
        }
        cnt.clear();
        cnt.shrink_to_fit();
        order.resize((size_t)nnz);
        parallel_for(cols, [&](int64_t a, int64_t b) {
            std::vector<int64_t> cur((size_t)P);
            for (int64_t j = a; j < b; ++j) {
                for (int64_t q = 0; q < P; ++q) cur[(size_t)q] = pptr[(size_t)(q * (cols + 1) + j)];
                for (int64_t p = ptr[j]; p < ptr[j + 1]; ++p) order[(size_t)cur[(size_t)(row_of(p) % P)]++] = p;
            }
        });
    }
    auto src_of = [&](int64_t pos) -> int64_t { return P == 1 ? pos : order[(size_t)pos]; };

    // 2. Deal each panel's rows to the NB waves, heaviest first onto the lightest wave.
    std::vector<uint8_t> wave_of((size_t)rows, 0);
    {
        std::vector<int64_t> rc((size_t)rows, 0);
        for (int64_t p = 0; p < nnz; ++p) rc[(size_t)row_of(p)]++;
        for (int64_t q = 0; q < P; ++q) {
            std::vector<int32_t> rs;
            for (int64_t r = q; r < rows; r += P) rs.push_back((int32_t)r);
            std::stable_sort(rs.begin(), rs.end(), [&](int32_t a, int32_t b) { return rc[(size_t)a] > rc[(size_t)b]; });
            std::vector<int64_t> load((size_t)NB, 0);
            for (int32_t r : rs) {
                const int64_t wv = std::min_element(load.begin(), load.end()) - load.begin();
                wave_of[(size_t)r] = (uint8_t)wv;
                load[(size_t)wv] += rc[(size_t)r];
            }
        }
    }

    // 3. Workgroups: contiguous runs of one panel's column-ordered nonzeros, as
    //    many in total as the chip runs at once.
    const int cus = device_cu_count(A.device);
    const int64_t per_cu = std::max<int64_t>(1, std::min<int64_t>(2, (160 * 1024) / std::max<int64_t>(R * 8 + 256, 1)));
    const int64_t target = (int64_t)cus * per_cu;
    struct WgRange {
        int32_t panel;
        int64_t a, b;      // panel-ordered positions
    };
    std::vector<WgRange> wr;
    A.panels.clear();
    // workgroups per panel in proportion to its nonzeros, largest remainders
    // first, at least one per non-empty panel, no more than target in total
    // when the panels allow it (one more would run as a second wave)
    std::vector<int64_t> pnw((size_t)P, 0);
    {
        std::vector<std::pair<double, int64_t>> rem;
        int64_t used = 0;
        for (int64_t q = 0; q < P; ++q) {
            const int64_t qn = pptr[(size_t)(q * (cols + 1) + cols)] - pptr[(size_t)(q * (cols + 1))];
            if (qn == 0) continue;
            const double share = (double)target * (double)qn / (double)std::max<int64_t>(nnz, 1);
            pnw[(size_t)q] = std::max<int64_t>(1, (int64_t)share);
            used += pnw[(size_t)q];
            rem.push_back({share - (double)(int64_t)share, q});
        }
        std::stable_sort(rem.begin(), rem.end(), [](const auto &x, const auto &y) { return x.first > y.first; });
        for (size_t i = 0; i < rem.size() && used < target; ++i, ++used) pnw[(size_t)rem[i].second]++;
    }
    for (int64_t q = 0; q < P; ++q) {
        const int64_t qa = pptr[(size_t)(q * (cols + 1))], qb = pptr[(size_t)(q * (cols + 1) + cols)];
        PanelDesc pd;
        pd.row0 = (int32_t)q;
        pd.rows = (int32_t)((rows - q + P - 1) / P);
        pd.wg0 = (int32_t)wr.size();
        if (qb > qa) {
            const int64_t nw = pnw[(size_t)q];
            const int64_t *pq = pptr.data() + q * (cols + 1);
            int64_t j0 = 0;
            for (int64_t w = 0; w < nw; ++w) {
                int64_t a, b;
                if (A.partition == SPW_PART_COLUMN) {
                    // equal numbers of columns, the first cols mod nw one more
                    const int64_t j1 = j0 + cols / nw + (w < cols % nw ? 1 : 0);
                    a = pq[j0];
                    b = pq[j1];
                    j0 = j1;
                } else if (A.partition == SPW_PART_MERGE) {
                    // merge path over (columns, nonzeros): range w starts at
                    // diagonal d = w * (cols + panel nonzeros) / nw; i columns
                    // and d - i nonzeros lie before it, with i the largest
                    // count of whole columns that fits
                    auto split = [&](int64_t ww) -> int64_t {
                        const int64_t d = (cols + (qb - qa)) * ww / nw;
                        int64_t lo = 0, hi = cols;        // largest i with (pq[i] - qa) + i <= d
                        while (lo < hi) {
                            const int64_t mid = (lo + hi + 1) / 2;
                            if (pq[mid] - qa + mid <= d) lo = mid;
                            else hi = mid - 1;
                        }
                        const int64_t k = std::min(std::max(d - lo, pq[lo] - qa),
                                                   (lo < cols ? pq[lo + 1] : pq[cols]) - qa);
                        return qa + k;
                    };
                    a = split(w);
                    b = split(w + 1);
                } else {
                    a = qa + (qb - qa) * w / nw;
                    b = qa + (qb - qa) * (w + 1) / nw;
                }
                if (b > a) wr.push_back(WgRange{(int32_t)q, a, b});
            }
        }
        pd.nwg = (int32_t)(wr.size() - (size_t)pd.wg0);
        A.panels.push_back(pd);
    }
    const int64_t W = (int64_t)wr.size();

    // 4. Blocks per (workgroup, wave): nonzeros of that wave's rows in column
    //    order, at most BLK per block and spanning fewer than SPAN columns.
    struct Blk {
        int32_t col_base, count;
        uint32_t packed[1024];
        double val[1024];
    };
    if (BLK > 1024 || BLK % 256) return fail(SPW_ERR_UNSUPPORTED, "scatter block size mismatch");
    std::vector<std::vector<std::vector<Blk>>> wblocks((size_t)W);
    parallel_for(W, [&](int64_t wa, int64_t wb) {
        for (int64_t w = wa; w < wb; ++w) {
            const WgRange &g = wr[(size_t)w];
            const int64_t *pp = pptr.data() + (int64_t)g.panel * (cols + 1);
            std::vector<std::vector<Blk>> &bl = wblocks[(size_t)w];
            bl.assign((size_t)NB, {});
            int64_t j = std::upper_bound(pp, pp + cols + 1, g.a) - pp - 1;
            for (int64_t pos = g.a; pos < g.b; ++pos) {
                while (pp[j + 1] <= pos) ++j;
                const int64_t sp = src_of(pos);
                const int64_t r = row_of(sp);
                std::vector<Blk> &v = bl[wave_of[(size_t)r]];
                if (v.empty() || v.back().count == BLK || j - v.back().col_base >= SPAN) {
                    v.emplace_back();
                    Blk &nb = v.back();
                    nb.col_base = (int32_t)j;
                    nb.count = 0;
                    std::memset(nb.packed, 0, (size_t)BLK * sizeof(uint32_t));
                    std::memset(nb.val, 0, (size_t)BLK * sizeof(double));
                }
                Blk &cb = v.back();
                // logical nonzero l = jj*64 + ln goes to the interleaved slots the kernel reads
                const int32_t l = cb.count++;
                const int32_t jj = l / 64, ln = l % 64;
                cb.packed[((jj / 4) * 64 + ln) * 4 + jj % 4] =
                    ((uint32_t)(r / P) << 16) | (uint32_t)(j - cb.col_base);
                cb.val[((jj / GV) * 64 + ln) * GV + jj % GV] = val[sp];
            }
        }
    });
    order.clear();
    order.shrink_to_fit();
    std::vector<int32_t> wg_blk((size_t)(W * (NB + 1)), 0);
    int64_t nblk = 0;
    for (int64_t w = 0; w < W; ++w)
        for (int64_t b = 0; b < NB; ++b) {
            wg_blk[(size_t)(w * (NB + 1) + b)] = (int32_t)nblk;
            nblk += (int64_t)wblocks[(size_t)w][(size_t)b].size();
            wg_blk[(size_t)(w * (NB + 1) + b + 1)] = (int32_t)nblk;
        }
    if (nblk * BLK >= ((int64_t)1 << 31)) return fail(SPW_ERR_UNSUPPORTED, "scatter-product storage exceeds 2^31 slots");
    const int64_t nslots = std::max<int64_t>(nblk, 1) * BLK;
    std::vector<uint32_t> packed((size_t)nslots, 0u);
    std::vector<uint8_t> mval((size_t)(nslots * es), 0);
    std::vector<int32_t> bdesc((size_t)(2 * std::max<int64_t>(nblk, 1)), 0);
    parallel_for(W, [&](int64_t wa, int64_t wb) {
        for (int64_t w = wa; w < wb; ++w)
            for (int64_t b = 0; b < NB; ++b) {
                int64_t id = wg_blk[(size_t)(w * (NB + 1) + b)];
                for (const Blk &bk : wblocks[(size_t)w][(size_t)b]) {
                    bdesc[(size_t)(2 * id)] = bk.col_base;
                    bdesc[(size_t)(2 * id + 1)] = bk.count;
                    std::memcpy(&packed[(size_t)(id * BLK)], bk.packed, (size_t)BLK * sizeof(uint32_t));
                    for (int64_t q = 0; q < BLK; ++q) put_value(storage, mval.data(), id * BLK + q, bk.val[q]);
                    ++id;
                }
            }
    });
    wblocks.clear();
    A.n_mblocks = nblk;
    A.mv_wgs = W;
    spw_status st;
    if ((st = dev_alloc(A, &A.d_mpacked, nslots, "block words"))) return st;
    if ((st = h2d(A.d_mpacked, packed.data(), (size_t)nslots * 4, "block words"))) return st;
    {
        uint8_t *d = nullptr;
        if ((st = dev_alloc(A, &d, nslots * es, "block values"))) return st;
        if ((st = h2d(d, mval.data(), mval.size(), "block values"))) return st;
        A.d_mval = d;
    }
    if ((st = dev_alloc(A, &A.d_mblocks, (int64_t)bdesc.size(), "block table"))) return st;
    if ((st = h2d(A.d_mblocks, bdesc.data(), bdesc.size() * 4, "block table"))) return st;
    if ((st = dev_alloc(A, &A.d_wg_blk, std::max<int64_t>((int64_t)wg_blk.size(), 1), "workgroup table"))) return st;
    if ((st = h2d(A.d_wg_blk, wg_blk.data(), wg_blk.size() * 4, "workgroup table"))) return st;
    if ((st = dev_alloc(A, &A.d_panels, P, "panels"))) return st;
    if ((st = h2d(A.d_panels, A.panels.data(), A.panels.size() * sizeof(PanelDesc), "panels"))) return st;
    return SPW_OK;
}

}  // namespace

spw_status grow_scratch(spw_matrix_s &A, int32_t k)
{
    spw_status st;
    if (!A.scratch.partial) {
        // partial sums of the scatter product: one column at a time
        if ((st = dev_alloc(A, &A.scratch.partial, std::max<int64_t>(A.mv_wgs, 1) * A.panel_rows, "partial sums")))
            return st;
    }
    const int64_t nch = std::max<int64_t>(A.cd.zp.n_chunks, A.cdt.zp.n_chunks);
    if (A.scratch.kcap >= k && A.scratch.carry_chunks >= nch) return SPW_OK;
    k = std::max<int32_t>(k, A.scratch.kcap);
    // grow the k-wide buffers: free the old ones once the device is idle
    auto drop = [&](double *&p) {
        if (!p) return;
        for (size_t i = 0; i < A.allocations.size(); ++i)
            if (A.allocations[i].first == p) {
                A.device_bytes -= A.allocations[i].second;
                A.allocations.erase(A.allocations.begin() + (long)i);
                break;
            }
        (void)hipFree(p);
        p = nullptr;
    };
    if (A.scratch.kcap > 0) {
        if (hipDeviceSynchronize() != hipSuccess) {
            (void)hipGetLastError();
            return fail(SPW_ERR_DEVICE, "hipDeviceSynchronize failed while growing scratch");
        }
    }
    drop(A.scratch.carry);
    drop(A.scratch.vperm);
    A.scratch.kcap = 0;
    A.scratch.carry_chunks = 0;
    if ((st = dev_alloc(A, &A.scratch.carry, std::max<int64_t>(2 * nch, 1) * k, "carries"))) return st;
    if ((st = dev_alloc(A, &A.scratch.vperm, std::max<int64_t>(A.rows, 1) * k, "renumbered vector"))) return st;
    A.scratch.kcap = k;
    A.scratch.carry_chunks = nch;
    return SPW_OK;
}

// ------------------------------------------------------------------ tuner
namespace {

// Median time in ms of `reps` runs of fn on stream s, after `warm` untimed
// runs; fn returns a HIP error code.  *err receives the first error.
template <typename F>
double time_median(hipStream_t s, F &&fn, int warm, int reps, int *err)
{
    *err = 0;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess) {
        (void)hipGetLastError();
        if (e0) (void)hipEventDestroy(e0);
        *err = (int)hipErrorOutOfMemory;
        return 0.0;
    }
    std::vector<float> t;
    for (int i = 0; i < warm + reps && !*err; ++i) {
        if (i >= warm) (void)hipEventRecord(e0, s);
        *err = fn();
        if (*err) break;
        if (i >= warm) {
            (void)hipEventRecord(e1, s);
            if (hipEventSynchronize(e1) != hipSuccess) {
                *err = (int)hipGetLastError();
                break;
            }
            float ms = 0.f;
            (void)hipEventElapsedTime(&ms, e0, e1);
            t.push_back(ms);
        }
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if (*err || t.empty()) return 0.0;
    std::sort(t.begin(), t.end());
    return (double)t[t.size() / 2];
}

const char *vdt_tag(spw_dtype vdt) { return vdt == SPW_F64 ? "f64" : "f32"; }

}  // namespace

// The host arrays a column-dot storage is built from (kept by spw_create
// while it runs, so the tuner can build other chunk sizes).
struct ColdotSource {
    int64_t rows, cols;
    const int64_t *ptr;
    const int32_t *rowi;
    const double *val;
};

// Chooses the column-dot chunk size and the workgroup size per vector type
// by timing spw_vtm-shaped column dots (u = B^T v) on scratch vectors, or
// takes the choices recorded for this matrix's fingerprint.  fixed_chunk /
// fixed_wg (non-zero) are the caller's and are not varied.  On return A.cd
// holds the storage of the chosen chunk size.
spw_status tune_coldot(spw_matrix_s &A, const ColdotSource &src, int32_t fixed_chunk, int32_t fixed_wg)
{
    spw_status st;
    const bool small_vals = A.value_storage != SPW_F64;
    // 1,024 threads fit with binary32 vectors and 4- or 2-byte values, or with chunks of 512
    auto wg_ok = [&](int32_t w, bool f32, int64_t chunk) {
        return w == 256 || w == 512 || (w == 1024 && ((f32 && small_vals) || chunk == 512));
    };
    auto use_chunk = [&](int64_t chunk) -> spw_status {
        if (A.cd.zp.chunk == chunk) return SPW_OK;
        if (hipDeviceSynchronize() != hipSuccess) {
            (void)hipGetLastError();
            return fail(SPW_ERR_DEVICE, "spw_create: device error while tuning");
        }
        free_coldot(A, A.cd);
        spw_status s2 = build_coldot(A, A.cd, src.rows, src.cols, src.ptr, src.rowi, src.val, A.value_storage, chunk);
        if (!s2) s2 = plan_workers(A, A.cd, src.ptr, SPW_PART_NONZERO);
        if (!s2) s2 = grow_scratch(A, 1);
        if (!s2 && t_uploader) s2 = t_uploader->finish();     // the arrays are on the device before timing
        return s2;
    };
    int32_t rc = 0, r64 = 0, r32 = 0;
    if (tune_get(A.fingerprint, "coldot.chunk", &rc) && tune_get(A.fingerprint, "coldot.wg.f64", &r64) &&
        tune_get(A.fingerprint, "coldot.wg.f32", &r32) && vtm_chunk_supported(rc) && wg_ok(r64, false, rc) &&
        wg_ok(r32, true, rc) && (fixed_chunk == 0 || fixed_chunk == rc)) {
        if ((st = use_chunk(rc))) return st;
        A.vtm_block[0] = fixed_wg ? fixed_wg : r64;
        A.vtm_block[1] = fixed_wg ? fixed_wg : r32;
        A.tuned = 1;
        return SPW_OK;
    }
    // scratch vectors: v (rows entries), u (cols entries), 8 bytes each
    void *dv = nullptr, *du = nullptr;
    hipStream_t s = nullptr;
    if (hipMalloc(&dv, (size_t)std::max<int64_t>(A.rows, 1) * 8) != hipSuccess ||
        hipMalloc(&du, (size_t)std::max<int64_t>(A.cols, 1) * 8) != hipSuccess ||
        hipMemset(dv, 0, (size_t)std::max<int64_t>(A.rows, 1) * 8) != hipSuccess ||
        hipStreamCreateWithFlags(&s, hipStreamNonBlocking) != hipSuccess) {
        (void)hipGetLastError();
        if (dv) (void)hipFree(dv);
        if (du) (void)hipFree(du);
        return fail(SPW_ERR_OUT_OF_MEMORY, "spw_create: no device memory for tuning");
    }
    struct Release {
        void *a, *b;
        hipStream_t s;
        ~Release()
        {
            (void)hipStreamSynchronize(s);
            (void)hipStreamDestroy(s);
            (void)hipFree(a);
            (void)hipFree(b);
        }
    } rel{dv, du, s};
    std::vector<int64_t> chunks = fixed_chunk ? std::vector<int64_t>{fixed_chunk} : std::vector<int64_t>{1024, 512};
    auto candidates = [&](bool f32, int64_t chunk) {
        if (fixed_wg) return std::vector<int32_t>{fixed_wg};
        std::vector<int32_t> w{256, 512};
        if (wg_ok(1024, f32, chunk)) w.push_back(1024);
        return w;
    };
    double best = -1.0;
    int64_t best_chunk = A.cd.zp.chunk;
    int32_t best64 = fixed_wg ? fixed_wg : 512, best32 = fixed_wg ? fixed_wg : 512;
    int err = 0;
    for (int64_t ch : chunks) {
        if ((st = use_chunk(ch))) return st;
        for (int32_t w : candidates(false, ch)) {
            A.vtm_block[0] = w;
            const double t = time_median(s, [&] { return launch_vtm(A, SPW_F64, dv, du, s); }, 2, 5, &err);
            if (err) return fail(SPW_ERR_DEVICE, "spw_create: a kernel failed while tuning");
            if (best < 0 || t < best) {
                best = t;
                best_chunk = ch;
                best64 = w;
            }
        }
    }
    if ((st = use_chunk(best_chunk))) return st;
    A.vtm_block[0] = best64;
    best = -1.0;
    for (int32_t w : candidates(true, best_chunk)) {
        A.vtm_block[1] = w;
        const double t = time_median(s, [&] { return launch_vtm(A, SPW_F32, dv, du, s); }, 2, 5, &err);
        if (err) return fail(SPW_ERR_DEVICE, "spw_create: a kernel failed while tuning");
        if (best < 0 || t < best) {
            best = t;
            best32 = w;
        }
    }
    A.vtm_block[1] = best32;
    A.tuned = 1;
    // a cache file that cannot be written keeps the records in memory
    (void)tune_put(A.fingerprint, "coldot.chunk", (int32_t)best_chunk);
    (void)tune_put(A.fingerprint, "coldot.wg.f64", best64);
    (void)tune_put(A.fingerprint, "coldot.wg.f32", best32);
    return SPW_OK;
}

spw_status grow_partial_cols(spw_matrix_s &A, int32_t cols)
{
    if (A.scratch.pcols >= cols || A.mv_wgs == 0) return SPW_OK;
    if (A.scratch.partial_cols) {
        if (hipDeviceSynchronize() != hipSuccess) {
            (void)hipGetLastError();
            return fail(SPW_ERR_DEVICE, "hipDeviceSynchronize failed while growing scratch");
        }
        for (size_t i = 0; i < A.allocations.size(); ++i)
            if (A.allocations[i].first == A.scratch.partial_cols) {
                A.device_bytes -= A.allocations[i].second;
                A.allocations.erase(A.allocations.begin() + (long)i);
                break;
            }
        (void)hipFree(A.scratch.partial_cols);
        A.scratch.partial_cols = nullptr;
        A.scratch.pcols = 0;
    }
    spw_status st;
    if ((st = dev_alloc(A, &A.scratch.partial_cols, (int64_t)cols * A.mv_wgs * A.panel_rows, "multi-column partial sums")))
        return st;
    A.scratch.pcols = cols;
    return SPW_OK;
}

// The CGLS workspace: r, q (m), s, p (n), partial sums, scalars, and a history
// of at least hist_len entries (a longer history replaces the old one once the
// device is idle).
spw_status grow_cgls(spw_matrix_s &A, int64_t hist_len)
{
    CglsScratch &W = A.cgls;
    spw_status st;
    if (!W.r) {
        if ((st = dev_alloc(A, &W.r, std::max<int64_t>(A.m, 1), "CGLS r"))) return st;
        if ((st = dev_alloc(A, &W.q, std::max<int64_t>(A.m, 1), "CGLS q"))) return st;
        if ((st = dev_alloc(A, &W.t, std::max<int64_t>(A.m, 1), "CGLS t"))) return st;
        if ((st = dev_alloc(A, &W.s, std::max<int64_t>(A.n, 1), "CGLS s"))) return st;
        if ((st = dev_alloc(A, &W.p, std::max<int64_t>(A.n, 1), "CGLS p"))) return st;
        if ((st = dev_alloc(A, &W.partial, cgls_dot_parts(), "CGLS partial sums"))) return st;
        if ((st = dev_alloc(A, &W.scal, 4, "CGLS scalars"))) return st;
    }
    if (W.hist_cap >= hist_len) return SPW_OK;
    if (W.hist) {
        if (hipDeviceSynchronize() != hipSuccess) {
            (void)hipGetLastError();
            return fail(SPW_ERR_DEVICE, "hipDeviceSynchronize failed while growing the CGLS history");
        }
        for (size_t i = 0; i < A.allocations.size(); ++i)
            if (A.allocations[i].first == W.hist) {
                A.device_bytes -= A.allocations[i].second;
                A.allocations.erase(A.allocations.begin() + (long)i);
                break;
            }
        (void)hipFree(W.hist);
        W.hist = nullptr;
        W.hist_cap = 0;
    }
    const int64_t cap = std::max<int64_t>(hist_len, 64);
    if ((st = dev_alloc(A, &W.hist, cap, "CGLS history"))) return st;
    W.hist_cap = cap;
    return SPW_OK;
}

// Sorts every line (column of a CSC, row of a CSR) by index and sums the
// values of a repeated index in the order the positions were given.  ptr must
// be valid and every index in [0, n_inner).  Fills the compressed output.
void canonical_lines(int64_t n_outer, const int64_t *ptr, const int32_t *idx, const double *val,
                     std::vector<int64_t> &optr, std::vector<int32_t> &oidx, std::vector<double> &oval)
{
    const int64_t nnz = ptr[n_outer];
    std::vector<int64_t> cnt((size_t)n_outer, 0), order((size_t)nnz);
    parallel_for(n_outer, [&](int64_t a, int64_t b) {
        for (int64_t j = a; j < b; ++j) {
            int64_t *o0 = order.data() + ptr[j], *o1 = order.data() + ptr[j + 1];
            std::iota(o0, o1, ptr[j]);
            std::stable_sort(o0, o1, [&](int64_t x, int64_t y) { return idx[x] < idx[y]; });
            int64_t distinct = 0;
            for (int64_t *q = o0; q < o1; ++q)
                if (q == o0 || idx[*q] != idx[*(q - 1)]) ++distinct;
            cnt[(size_t)j] = distinct;
        }
    });
    optr.assign((size_t)n_outer + 1, 0);
    for (int64_t j = 0; j < n_outer; ++j) optr[(size_t)j + 1] = optr[(size_t)j] + cnt[(size_t)j];
    oidx.resize((size_t)optr[(size_t)n_outer]);
    oval.resize((size_t)optr[(size_t)n_outer]);
    parallel_for(n_outer, [&](int64_t a, int64_t b) {
        for (int64_t j = a; j < b; ++j) {
            int64_t w = optr[(size_t)j] - 1;
            for (int64_t q = ptr[j]; q < ptr[j + 1]; ++q) {
                const int64_t p = order[(size_t)q];
                if (q == ptr[j] || idx[p] != oidx[(size_t)w]) {
                    ++w;
                    oidx[(size_t)w] = idx[p];
                    oval[(size_t)w] = val[p];
                } else {
                    oval[(size_t)w] = oval[(size_t)w] + val[p];
                }
            }
        }
    });
}

}  // namespace spw

using namespace spw;

extern "C" {

const char *spw_last_error(void) { return t_err.c_str(); }

const char *spw_status_string(spw_status s)
{
    switch (s) {
    case SPW_OK: return "SPW_OK";
    case SPW_ERR_INVALID_ARG: return "SPW_ERR_INVALID_ARG";
    case SPW_ERR_BAD_MATRIX: return "SPW_ERR_BAD_MATRIX";
    case SPW_ERR_OUT_OF_MEMORY: return "SPW_ERR_OUT_OF_MEMORY";
    case SPW_ERR_BUDGET: return "SPW_ERR_BUDGET";
    case SPW_ERR_DEVICE: return "SPW_ERR_DEVICE";
    case SPW_ERR_UNSUPPORTED: return "SPW_ERR_UNSUPPORTED";
    case SPW_ERR_BUSY: return "SPW_ERR_BUSY";
    case SPW_ERR_TIMEOUT: return "SPW_ERR_TIMEOUT";
    case SPW_ERR_SHUTDOWN: return "SPW_ERR_SHUTDOWN";
    }
    return "SPW_UNKNOWN_STATUS";
}

static spw_status spw_create_opts_default_impl(spw_create_opts *o)
{
    if (!o) return fail(SPW_ERR_INVALID_ARG, "spw_create_opts_default: NULL opts");
    std::memset(o, 0, sizeof(*o));
    o->struct_size = sizeof(*o);
    o->value_storage = SPW_F64;
    o->chunk_nnz = 0;
    o->relabel = -1;
    o->validate = 1;
    o->panel_rows = 0;
    o->device = -1;
    o->transpose = -1;
    o->wg_size = 0;
    o->autotune = 0;
    return SPW_OK;
}

spw_status spw_create_opts_default(spw_create_opts *o)
{
    return guarded("spw_create_opts_default", [&] { return spw_create_opts_default_impl(o); });
}

static spw_status spw_create_impl(spw_matrix *out, spw_format fmt, int64_t m, int64_t n, int64_t nnz,
                                  const int64_t *ptr, const int32_t *idx, const double *val,
                                  const spw_create_opts *opts_in)
{
    if (!out) return fail(SPW_ERR_INVALID_ARG, "spw_create: NULL out");
    *out = nullptr;
    if (fmt != SPW_CSC && fmt != SPW_CSR) return fail(SPW_ERR_INVALID_ARG, "spw_create: bad format");
    if (m < 0 || n < 0 || nnz < 0) return fail(SPW_ERR_INVALID_ARG, "spw_create: negative size");
    if (!ptr) return fail(SPW_ERR_INVALID_ARG, "spw_create: NULL ptr");
    if (nnz > 0 && (!idx || !val)) return fail(SPW_ERR_INVALID_ARG, "spw_create: NULL idx or val with nnz > 0");
    spw_create_opts opts;
    spw_create_opts_default(&opts);
    if (opts_in) {
        if (opts_in->struct_size != sizeof(spw_create_opts))
            return fail(SPW_ERR_INVALID_ARG, "spw_create: opts.struct_size must be sizeof(spw_create_opts)");
        opts = *opts_in;
    }
    if (opts.value_storage != SPW_F64 && opts.value_storage != SPW_F32 && opts.value_storage != SPW_BF16)
        return fail(SPW_ERR_INVALID_ARG, "spw_create: bad value_storage");
    if (opts.partition != SPW_PART_NONZERO && opts.partition != SPW_PART_COLUMN &&
        opts.partition != SPW_PART_MERGE)
        return fail(SPW_ERR_INVALID_ARG, "spw_create: bad partition");
    const int64_t chunk = opts.chunk_nnz > 0 ? opts.chunk_nnz : vtm_chunk_default();
    if (opts.chunk_nnz < 0 || !vtm_chunk_supported(chunk))
        return fail(SPW_ERR_UNSUPPORTED, "spw_create: chunk_nnz must be 0, 512 or 1024");
    if (opts.wg_size != 0 && opts.wg_size != 256 && opts.wg_size != 512 && opts.wg_size != 1024)
        return fail(SPW_ERR_UNSUPPORTED, "spw_create: wg_size must be 0, 256, 512 or 1024");
    if (opts.autotune != 0 && opts.autotune != 1) return fail(SPW_ERR_INVALID_ARG, "spw_create: autotune must be 0 or 1");

    const int64_t rows = fmt == SPW_CSC ? m : n;
    const int64_t cols = fmt == SPW_CSC ? n : m;
    const int64_t pad = 4096;
    if (nnz + pad >= ((int64_t)1 << 31) || cols >= ((int64_t)1 << 31) - 1 || rows >= ((int64_t)1 << 31))
        return fail(SPW_ERR_UNSUPPORTED, "spw_create: nnz and dimensions must stay below 2^31");
    if (opts.canonicalize) {
        // checks of the pointer and of the index range (order and repeats are fixed here)
        if (ptr[0] != 0 || ptr[cols] != nnz)
            return fail(SPW_ERR_BAD_MATRIX, "ptr must start at 0 and end at nnz");
        for (int64_t j = 0; j < cols; ++j)
            if (ptr[j + 1] < ptr[j])
                return fail(SPW_ERR_BAD_MATRIX, "ptr decreases at " + std::to_string(j));
        for (int64_t p = 0; p < nnz; ++p)
            if (idx[p] < 0 || idx[p] >= rows)
                return fail(SPW_ERR_BAD_MATRIX, "index out of range at position " + std::to_string(p));
        std::vector<int64_t> cptr;
        std::vector<int32_t> cidx;
        std::vector<double> cval;
        canonical_lines(cols, ptr, idx, val, cptr, cidx, cval);
        spw_create_opts o2 = opts;
        o2.canonicalize = 0;
        o2.validate = 0;
        return spw_create(out, fmt, m, n, (int64_t)cidx.size(), cptr.data(), cidx.data(), cval.data(), &o2);
    }
    if (opts.validate) {
        spw_status st = validate(cols, rows, nnz, ptr, idx, fmt == SPW_CSC ? "column" : "row");
        if (st) return st;
    } else if (ptr[cols] != nnz) {
        return fail(SPW_ERR_BAD_MATRIX, "ptr[last] must equal nnz");
    }

    // values as stored (rounded once), promoted back to binary64 for the builders
    std::vector<double> rounded;
    if (opts.value_storage != SPW_F64 && nnz > 0) {
        rounded.resize((size_t)nnz);
        const int64_t bad = round_values(opts.value_storage, nnz, val, rounded.data());
        if (bad >= 0)
            return fail(SPW_ERR_BAD_MATRIX, "position " + std::to_string(bad) + ": value " + std::to_string(val[bad]) +
                                                " overflows the value storage type");
        val = rounded.data();
    }

    DeviceGuard dg(opts.device);
    if (dg.st) return dg.st;
    std::unique_ptr<spw_matrix_s> A(new spw_matrix_s());
    A->format = fmt;
    A->value_storage = opts.value_storage;
    A->partition = opts.partition;
    A->m = m;
    A->n = n;
    A->nnz = nnz;
    A->rows = rows;
    A->cols = cols;
    (void)hipGetDevice(&A->device);
    A->relabeled = opts.relabel < 0 ? (rows > 4096 ? 1 : 0) : (opts.relabel ? 1 : 0);
    if (rows == 0) A->relabeled = 0;

    struct Cleanup {
        spw_matrix_s *a;
        bool armed = true;
        ~Cleanup()
        {
            if (armed) free_all(a);
        }
    } cleanup{A.get()};
    // large host-to-device copies go through pinned staging, overlapped with
    // the host work that follows them; declared after `cleanup`, so it waits
    // for its copies before the device buffers can be freed
    Uploader up;
    struct UploaderScope {
        Uploader *prev;
        explicit UploaderScope(Uploader *u) : prev(t_uploader) { t_uploader = u; }
        ~UploaderScope() { t_uploader = prev; }
    } up_scope(&up);

    spw_status st;
    // Row renumbering by descending count (ties by row), so that the busiest
    // entries of the short vector are adjacent.
    std::vector<int32_t> rank, inv;
    if (A->relabeled) {
        std::vector<int64_t> cnt((size_t)rows, 0);
        for (int64_t p = 0; p < nnz; ++p) cnt[(size_t)idx[p]]++;
        inv.resize((size_t)rows);
        std::iota(inv.begin(), inv.end(), 0);
        std::stable_sort(inv.begin(), inv.end(), [&](int32_t a, int32_t b) { return cnt[(size_t)a] > cnt[(size_t)b]; });
        rank.resize((size_t)rows);
        for (int64_t r = 0; r < rows; ++r) rank[(size_t)inv[(size_t)r]] = (int32_t)r;
        if ((st = dev_alloc(*A, &A->d_rank, rows, "row renumbering"))) return st;
        if ((st = h2d(A->d_rank, rank.data(), (size_t)rows * 4, "row renumbering"))) return st;
        if ((st = dev_alloc(*A, &A->d_inv, rows, "row renumbering"))) return st;
        if ((st = h2d(A->d_inv, inv.data(), (size_t)rows * 4, "row renumbering"))) return st;
    }
    std::vector<int32_t> rowi((size_t)std::max<int64_t>(nnz, 1), 0);
    {
        const bool rl = A->relabeled != 0;
        parallel_for(nnz, [&](int64_t a, int64_t b) {
            for (int64_t p = a; p < b; ++p) rowi[(size_t)p] = rl ? rank[(size_t)idx[p]] : idx[p];
        });
    }
    A->vtm_block[0] = A->vtm_block[1] = opts.wg_size;
    A->autotune = opts.autotune;
    A->fingerprint = matrix_fingerprint(fmt, opts.value_storage, m, n, nnz, ptr, idx);
    if ((st = build_coldot(*A, A->cd, rows, cols, ptr, rowi.data(), val, A->value_storage, chunk))) return st;
    if ((st = plan_workers(*A, A->cd, ptr, A->partition))) return st;

    // The transpose (caller's numbering), used by the tiled multi-RHS scatter
    // products: its column dots are the rows of B.  It is kept in blocks of
    // TRANSPOSE_BLOCK_ROWS of B's columns: column b*rows + i holds B's row i
    // within block b, so the chunks of one block, which the workgroups take
    // about together, gather only that block's rows of the input.
    if ((opts.transpose > 0 || (opts.transpose < 0 && opts.autotune)) && nnz > 0) {
        const int64_t R = TRANSPOSE_BLOCK_ROWS;
        const int64_t nb = std::max<int64_t>(1, (cols + R - 1) / R);
        const int64_t vcols = nb * rows;
        std::vector<int64_t> tptr((size_t)vcols + 1, 0);
        for (int64_t j = 0; j < cols; ++j) {
            const int64_t off = (j / R) * rows + 1;
            for (int64_t p = ptr[j]; p < ptr[j + 1]; ++p) tptr[(size_t)(off + idx[p])]++;
        }
        for (int64_t r = 0; r < vcols; ++r) tptr[(size_t)r + 1] += tptr[(size_t)r];
        std::vector<int32_t> tidx((size_t)nnz);
        std::vector<double> tval((size_t)nnz);
        {
            std::vector<int64_t> cur(tptr.begin(), tptr.end() - 1);
            for (int64_t j = 0; j < cols; ++j) {
                const int64_t off = (j / R) * rows;
                for (int64_t p = ptr[j]; p < ptr[j + 1]; ++p) {
                    const int64_t dst = cur[(size_t)(off + idx[p])]++;
                    tidx[(size_t)dst] = (int32_t)j;
                    tval[(size_t)dst] = val[p];
                }
            }
        }
        if ((st = build_coldot(*A, A->cdt, cols, vcols, tptr.data(), tidx.data(), tval.data(), A->value_storage,
                               vtm_chunk_default())))
            return st;
        A->cdt_blocks = nb;
    }

    // Scatter-product storage.
    if (rows > 0) {
        if ((st = build_mv_storage(*A, ptr, rowi.data(), val, opts.panel_rows))) return st;
    }
    if ((st = grow_scratch(*A, 1))) return st;
    if ((st = up.finish())) return st;
    if (opts.autotune && nnz > 0 && rows > 0 && A->partition == SPW_PART_NONZERO) {
        ColdotSource src{rows, cols, ptr, rowi.data(), val};
        if ((st = tune_coldot(*A, src, opts.chunk_nnz, opts.wg_size))) return st;
    }
    if (hipDeviceSynchronize() != hipSuccess) {
        (void)hipGetLastError();
        return fail(SPW_ERR_DEVICE, "device error during spw_create");
    }
    cleanup.armed = false;
    *out = A.release();
    return SPW_OK;
}

spw_status spw_create(spw_matrix *out, spw_format fmt, int64_t m, int64_t n, int64_t nnz, const int64_t *ptr,
                      const int32_t *idx, const double *val, const spw_create_opts *opts_in)
{
    return guarded("spw_create", [&] { return spw_create_impl(out, fmt, m, n, nnz, ptr, idx, val, opts_in); });
}

static spw_status spw_create_coo_impl(spw_matrix *out, spw_format fmt, int64_t m, int64_t n, int64_t nnz,
                                      const int32_t *rows, const int32_t *cols, const double *val,
                                      const spw_create_opts *opts)
{
    if (!out) return fail(SPW_ERR_INVALID_ARG, "spw_create_coo: NULL out");
    *out = nullptr;
    if (fmt != SPW_CSC && fmt != SPW_CSR) return fail(SPW_ERR_INVALID_ARG, "spw_create_coo: bad format");
    if (m < 0 || n < 0 || nnz < 0) return fail(SPW_ERR_INVALID_ARG, "spw_create_coo: negative size");
    if (nnz > 0 && (!rows || !cols || !val)) return fail(SPW_ERR_INVALID_ARG, "spw_create_coo: NULL triples");
    if (nnz >= ((int64_t)1 << 31)) return fail(SPW_ERR_UNSUPPORTED, "spw_create_coo: nnz must be < 2^31");
    // compressed dimension (outer) and the one stored per entry (inner)
    const bool csc = fmt == SPW_CSC;
    const int32_t *outer = csc ? cols : rows, *inner = csc ? rows : cols;
    const int64_t n_outer = csc ? n : m, n_inner = csc ? m : n;
    for (int64_t p = 0; p < nnz; ++p)
        if (rows[p] < 0 || rows[p] >= m || cols[p] < 0 || cols[p] >= n)
            return fail(SPW_ERR_BAD_MATRIX, "spw_create_coo: triple " + std::to_string(p) + " (" +
                                                std::to_string(rows[p]) + ", " + std::to_string(cols[p]) +
                                                ") lies outside the " + std::to_string(m) + " x " +
                                                std::to_string(n) + " matrix");
    (void)n_inner;
    // counting sort by the outer index (stable), then each outer line by inner index
    std::vector<int64_t> ptr((size_t)n_outer + 1, 0);
    for (int64_t p = 0; p < nnz; ++p) ptr[(size_t)outer[p] + 1]++;
    for (int64_t j = 0; j < n_outer; ++j) ptr[(size_t)j + 1] += ptr[(size_t)j];
    std::vector<int64_t> order((size_t)nnz);
    {
        std::vector<int64_t> cur(ptr.begin(), ptr.end() - 1);
        for (int64_t p = 0; p < nnz; ++p) order[(size_t)cur[(size_t)outer[p]]++] = p;
    }
    std::vector<int32_t> idx((size_t)nnz);
    std::vector<double> v((size_t)nnz);
    std::atomic<int64_t> dup{-1};
    parallel_for(n_outer, [&](int64_t a, int64_t b) {
        for (int64_t j = a; j < b; ++j) {
            int64_t *o0 = order.data() + ptr[(size_t)j], *o1 = order.data() + ptr[(size_t)j + 1];
            std::sort(o0, o1, [&](int64_t x, int64_t y) { return inner[x] < inner[y] || (inner[x] == inner[y] && x < y); });
            for (int64_t *q = o0; q < o1; ++q) {
                const int64_t pos = q - order.data();
                idx[(size_t)pos] = inner[*q];
                v[(size_t)pos] = val[*q];
                if (q > o0 && inner[*q] == inner[*(q - 1)]) {
                    int64_t none = -1;
                    dup.compare_exchange_strong(none, *q);
                }
            }
        }
    });
    const bool canon = opts && opts->struct_size == sizeof(spw_create_opts) && opts->canonicalize;
    if (dup.load() >= 0 && canon) {
        // repeats summed in the order given: the lines are sorted by (index, given position)
        std::vector<int64_t> cptr;
        std::vector<int32_t> cidx;
        std::vector<double> cval;
        canonical_lines(n_outer, ptr.data(), idx.data(), v.data(), cptr, cidx, cval);
        spw_create_opts o2 = *opts;
        o2.canonicalize = 0;
        return spw_create(out, fmt, m, n, (int64_t)cidx.size(), cptr.data(), cidx.data(), cval.data(), &o2);
    }
    if (dup.load() >= 0) {
        const int64_t p = dup.load();
        return fail(SPW_ERR_BAD_MATRIX, "spw_create_coo: (" + std::to_string(rows[p]) + ", " +
                                            std::to_string(cols[p]) + ") is given more than once");
    }
    order.clear();
    order.shrink_to_fit();
    return spw_create(out, fmt, m, n, nnz, ptr.data(), idx.data(), v.data(), opts);
}

spw_status spw_create_coo(spw_matrix *out, spw_format fmt, int64_t m, int64_t n, int64_t nnz, const int32_t *rows,
                          const int32_t *cols, const double *val, const spw_create_opts *opts)
{
    return guarded("spw_create_coo", [&] { return spw_create_coo_impl(out, fmt, m, n, nnz, rows, cols, val, opts); });
}

static spw_status spw_destroy_impl(spw_matrix A)
{
    if (!A) return SPW_OK;
    {
        DeviceGuard dg(A->device);
        (void)hipDeviceSynchronize();
        if (A->last_done) (void)hipEventDestroy((hipEvent_t)A->last_done);
        free_all(A);
    }
    delete A;
    return SPW_OK;
}

spw_status spw_destroy(spw_matrix A)
{
    return guarded("spw_destroy", [&] { return spw_destroy_impl(A); });
}

static spw_status spw_info_impl(spw_matrix A, spw_matrix_info *o)
{
    if (!A || !o) return fail(SPW_ERR_INVALID_ARG, "spw_info: NULL argument");
    if (o->struct_size != sizeof(spw_matrix_info))
        return fail(SPW_ERR_INVALID_ARG, "spw_info: out->struct_size must be sizeof(spw_matrix_info)");
    o->format = A->format;
    o->value_storage = A->value_storage;
    o->m = A->m;
    o->n = A->n;
    o->nnz = A->nnz;
    o->inner_rows = A->rows;
    o->inner_cols = A->cols;
    o->chunk_nnz = A->cd.zp.chunk;
    o->n_chunks = A->cd.zp.n_chunks;
    o->n_zones = A->cd.n_zones;
    o->n_panels = A->n_panels;
    o->panel_rows = A->panel_rows;
    o->mv_workgroups = A->mv_wgs;
    o->index_bytes = A->cd.idx_kind == IdxKind::U16 ? 2 : 4;
    o->has_transpose = A->cdt.built ? 1 : 0;
    o->partition = A->partition;
    o->workers = A->cd.n_workers;
    o->worker_max_nnz = A->cd.worker_max_nnz;
    o->worker_min_nnz = A->cd.worker_min_nnz;
    o->relabeled = A->relabeled;
    o->device = A->device;
    o->device_bytes = A->device_bytes;
    // the sizes the kernels run with (1,024 falls back to 512 where it does not fit)
    const bool c512 = A->cd.zp.chunk == 512;
    o->wg_size_f64 = A->vtm_block[0] ? A->vtm_block[0] : 512;
    o->wg_size_f32 = A->vtm_block[1] ? A->vtm_block[1] : (A->value_storage != SPW_F64 ? 1024 : 512);
    if (o->wg_size_f32 == 1024 && A->value_storage == SPW_F64 && !c512) o->wg_size_f32 = 512;
    if (o->wg_size_f64 == 1024 && !c512) o->wg_size_f64 = 512;
    o->tuned = A->tuned;
    o->fingerprint = A->fingerprint;
    return SPW_OK;
}

spw_status spw_info(spw_matrix A, spw_matrix_info *o)
{
    return guarded("spw_info", [&] { return spw_info_impl(A, o); });
}

// ---------------------------------------------------------- multi-RHS plans
namespace spw {
namespace {

// The fixed rule (see spw_plan in spw.h).  Scatter direction: passes of up to
// 8 columns below 16 columns (they beat the tiled column dots over the
// transpose there, whose gathers of the caller's k-wide rows of X cross cache
// lines unless k is a power of two), tiles from 16.  Column dots: each chunk
// read once and reduced per column up to 6 columns, tiles from about 7 on.
static int32_t rule_plan(const spw_matrix_s &A, bool scatter, int32_t k, int64_t ldo)
{
    if (scatter) return (k < 16 || !A.cdt.built) ? SPW_PLAN_PASSES : SPW_PLAN_TILE;
    return (k <= 6 && ldo < CHUNK_OUT_LD_LIMIT) ? SPW_PLAN_PASSES : SPW_PLAN_TILE;
}

static bool plan_runs(const spw_matrix_s &A, bool scatter, int32_t plan, int64_t ldo)
{
    if (plan < SPW_PLAN_SINGLE || plan > SPW_PLAN_TILE) return false;
    if (scatter) return plan != SPW_PLAN_TILE || A.cdt.built;
    // the chunk-per-wave column dots address outputs through a 2^31-byte view
    return plan == SPW_PLAN_TILE || ldo < CHUNK_OUT_LD_LIMIT;
}

static int64_t plan_slot(bool scatter, spw_dtype vdt, int32_t k)
{
    return ((int64_t)(scatter ? 1 : 0) << 40) | ((int64_t)vdt << 32) | (int64_t)k;
}

static std::string plan_cache_key(bool scatter, spw_dtype vdt, int32_t k)
{
    return std::string("plan.") + (scatter ? "sc." : "cd.") + vdt_tag(vdt) + ".k" + std::to_string(k);
}

// The binary64 partial sums of the blocked transpose for k columns; grown
// once the device is idle.  Returns a HIP error code.
static int grow_cdt_partial(spw_matrix_s &A, int32_t k)
{
    const int64_t need = A.cdt.cols * (int64_t)k;
    if (A.cdt_partial_elems >= need) return 0;
    if (A.cdt_partial) {
        if (hipDeviceSynchronize() != hipSuccess) return (int)hipGetLastError();
        for (size_t i = 0; i < A.allocations.size(); ++i)
            if (A.allocations[i].first == A.cdt_partial) {
                A.device_bytes -= A.allocations[i].second;
                A.allocations.erase(A.allocations.begin() + (long)i);
                break;
            }
        (void)hipFree(A.cdt_partial);
        A.cdt_partial = nullptr;
        A.cdt_partial_elems = 0;
    }
    if (dev_alloc(A, &A.cdt_partial, need, "partial sums of the blocked transpose")) return (int)hipErrorOutOfMemory;
    A.cdt_partial_elems = need;
    return 0;
}

// Runs a k-column product with one plan; returns a HIP error code.
static int run_plan(spw_matrix_s &A, int32_t plan, bool scatter, spw_dtype vdt, int32_t k, const void *in,
                    int64_t ldi, void *out, int64_t ldo, void *stream)
{
    const size_t es = vdt == SPW_F64 ? 8 : 4;
    if (plan == SPW_PLAN_TILE) {
        if (scatter) {
            if (A.nnz == 0) return launch_zero_fill(vdt, k, out, ldo, A.rows, stream);   // all outputs are zero
            if (A.cdt_blocks <= 1) return launch_coldot_batch(A, A.cdt, nullptr, vdt, k, in, ldi, out, ldo, stream);
            // one launch over every block into binary64 partial sums, then their sum in block order
            int e = grow_cdt_partial(A, k);
            if (!e) e = launch_coldot_batch(A, A.cdt, nullptr, vdt, k, in, ldi, A.cdt_partial, k, stream, true);
            if (!e) e = launch_sum_blocks(vdt, A.cdt_blocks, A.rows, k, A.cdt_partial, out, ldo, stream);
            return e;
        }
        return launch_coldot_batch(A, A.cd, A.relabeled ? A.d_inv : nullptr, vdt, k, in, ldi, out, ldo, stream);
    }
    if (plan == SPW_PLAN_SINGLE) {
        for (int32_t c = 0; c < k; ++c) {
            const void *ic = (const char *)in + (size_t)c * es;
            void *oc = (char *)out + (size_t)c * es;
            const int e = scatter ? launch_mv(A, vdt, 1, ic, ldi, oc, ldo, stream)
                                  : launch_vtm_cols(A, vdt, 1, &ic, &ldi, &oc, &ldo, stream);
            if (e) return e;
        }
        return 0;
    }
    return scatter ? launch_mv(A, vdt, k, in, ldi, out, ldo, stream)
                   : launch_vtm_multi(A, vdt, k, in, ldi, out, ldo, stream);
}

// Times every plan that can run on the caller's buffers and stream (the
// output is overwritten by each) and returns the fastest; 0 on a kernel error.
static int32_t tune_plan(spw_matrix_s &A, bool scatter, spw_dtype vdt, int32_t k, const void *in, int64_t ldi,
                         void *out, int64_t ldo, void *stream, int *err)
{
    double best = -1.0;
    int32_t choice = 0;
    for (int32_t plan : {SPW_PLAN_SINGLE, SPW_PLAN_PASSES, SPW_PLAN_TILE}) {
        if (!plan_runs(A, scatter, plan, ldo)) continue;
        const double t = time_median((hipStream_t)stream,
                                     [&] { return run_plan(A, plan, scatter, vdt, k, in, ldi, out, ldo, stream); },
                                     1, 3, err);
        if (*err) return 0;
        if (best < 0 || t < best) {
            best = t;
            choice = plan;
        }
    }
    return choice;
}

}  // namespace
}  // namespace spw

static spw_status run_product(spw_matrix A, bool want_mv, spw_dtype vdt, int32_t k, const void *in, int64_t ldi,
                              void *out, int64_t ldo, void *stream, const char *fname)
{
    if (!A) return fail(SPW_ERR_INVALID_ARG, std::string(fname) + ": NULL matrix");
    if (vdt != SPW_F64 && vdt != SPW_F32) return fail(SPW_ERR_INVALID_ARG, std::string(fname) + ": bad vector dtype");
    if (k < 1 || k > 64) return fail(SPW_ERR_INVALID_ARG, std::string(fname) + ": k must be in [1, 64]");
    if (ldi < k || ldo < k) return fail(SPW_ERR_INVALID_ARG, std::string(fname) + ": leading dimension < k");
    // short/long lengths of the input and output for this op
    const bool scatter = (A->format == SPW_CSC) == want_mv;   // B x  vs  v^T B
    const int64_t in_len = scatter ? A->cols : A->rows;
    const int64_t out_len = scatter ? A->rows : A->cols;
    if ((in_len > 0 && !in) || (out_len > 0 && !out))
        return fail(SPW_ERR_INVALID_ARG, std::string(fname) + ": NULL vector");
    DeviceGuard dg(A->device);
    if (dg.st) return dg.st;
    spw_status st = claim_stream(*A, stream, fname);
    if (st) return st;
    if ((st = grow_scratch(*A, coldot_tile_width(k)))) return st;
    int e = 0;
    if (k == 1) {
        if (ldi == 1 && ldo == 1) {
            e = scatter ? launch_mv(*A, vdt, 1, in, 1, out, 1, stream) : launch_vtm(*A, vdt, in, out, stream);
        } else if (scatter) {
            e = launch_mv(*A, vdt, 1, in, ldi, out, ldo, stream);
        } else if (ldo < CHUNK_OUT_LD_LIMIT) {
            e = launch_vtm_multi(*A, vdt, 1, in, ldi, out, ldo, stream);
        } else {
            e = launch_coldot_batch(*A, A->cd, A->relabeled ? A->d_inv : nullptr, vdt, 1, in, ldi, out, ldo, stream);
        }
    } else {
        // the plan: set by the caller or the tuner, recorded for this matrix, timed now, or the fixed rule
        const int64_t slot = plan_slot(scatter, vdt, k);
        int32_t plan = 0;
        {
            std::lock_guard<std::mutex> lk(A->plan_mu);
            const auto it = A->plans.find(slot);
            if (it != A->plans.end()) plan = it->second;
        }
        if (!plan_runs(*A, scatter, plan, ldo)) plan = 0;
        if (!plan && A->autotune) {
            int32_t rec = 0;
            if (tune_get(A->fingerprint, plan_cache_key(scatter, vdt, k), &rec) && plan_runs(*A, scatter, rec, ldo))
                plan = rec;
            if (scatter && (st = grow_partial_cols(*A, std::min<int32_t>(k, 8)))) return st;
            if (!plan && !capturing(stream)) {
                plan = tune_plan(*A, scatter, vdt, k, in, ldi, out, ldo, stream, &e);
                if (e) return fail(SPW_ERR_DEVICE, std::string(fname) + ": a kernel failed while tuning: " +
                                                       hipGetErrorString((hipError_t)e));
                if (plan) (void)tune_put(A->fingerprint, plan_cache_key(scatter, vdt, k), plan);
            }
            if (plan) {
                std::lock_guard<std::mutex> lk(A->plan_mu);
                A->plans[slot] = plan;
            }
        }
        if (!plan) plan = rule_plan(*A, scatter, k, ldo);
        if (scatter && plan == SPW_PLAN_PASSES && (st = grow_partial_cols(*A, std::min<int32_t>(k, 8)))) return st;
        e = run_plan(*A, plan, scatter, vdt, k, in, ldi, out, ldo, stream);
    }
    if (e == (int)hipErrorNotSupported)
        return fail(SPW_ERR_UNSUPPORTED, std::string(fname) + ": this dtype / k / storage combination is not available");
    if (e) return fail(SPW_ERR_DEVICE, std::string(fname) + ": kernel launch failed: " + hipGetErrorString((hipError_t)e));
    return release_stream(*A, stream, fname);
}

static spw_status batch_plan_impl(spw_matrix A, spw_op op, spw_dtype vdt, int32_t k, spw_plan *plan, int32_t *tuned)
{
    if (!A || !plan || !tuned) return fail(SPW_ERR_INVALID_ARG, "spw_batch_plan: NULL argument");
    if ((op != SPW_OP_MV && op != SPW_OP_VTM) || (vdt != SPW_F64 && vdt != SPW_F32) || k < 1 || k > 64)
        return fail(SPW_ERR_INVALID_ARG, "spw_batch_plan: bad op, vector type or k");
    const bool scatter = (A->format == SPW_CSC) == (op == SPW_OP_MV);
    *tuned = 0;
    if (k == 1) {
        *plan = SPW_PLAN_SINGLE;
        return SPW_OK;
    }
    int32_t p = 0;
    {
        std::lock_guard<std::mutex> lk(A->plan_mu);
        const auto it = A->plans.find(plan_slot(scatter, vdt, k));
        if (it != A->plans.end()) p = it->second;
    }
    if (!plan_runs(*A, scatter, p, k)) p = 0;
    if (!p && A->autotune) {
        int32_t rec = 0;
        if (tune_get(A->fingerprint, plan_cache_key(scatter, vdt, k), &rec) && plan_runs(*A, scatter, rec, k)) p = rec;
    }
    *tuned = p ? 1 : 0;
    *plan = (spw_plan)(p ? p : rule_plan(*A, scatter, k, k));
    return SPW_OK;
}

spw_status spw_batch_plan(spw_matrix A, spw_op op, spw_dtype vdt, int32_t k, spw_plan *plan, int32_t *tuned)
{
    return guarded("spw_batch_plan", [&] { return batch_plan_impl(A, op, vdt, k, plan, tuned); });
}

static spw_status set_batch_plan_impl(spw_matrix A, spw_op op, spw_dtype vdt, int32_t k, spw_plan plan)
{
    if (!A) return fail(SPW_ERR_INVALID_ARG, "spw_set_batch_plan: NULL matrix");
    if ((op != SPW_OP_MV && op != SPW_OP_VTM) || (vdt != SPW_F64 && vdt != SPW_F32) || k < 2 || k > 64 ||
        plan < SPW_PLAN_AUTO || plan > SPW_PLAN_TILE)
        return fail(SPW_ERR_INVALID_ARG, "spw_set_batch_plan: bad op, vector type, k (2..64) or plan");
    const bool scatter = (A->format == SPW_CSC) == (op == SPW_OP_MV);
    if (plan == SPW_PLAN_TILE && scatter && !A->cdt.built)
        return fail(SPW_ERR_UNSUPPORTED, "spw_set_batch_plan: the tiled plan of this direction needs the kept transpose");
    std::lock_guard<std::mutex> lk(A->plan_mu);
    if (plan == SPW_PLAN_AUTO) A->plans.erase(plan_slot(scatter, vdt, k));
    else A->plans[plan_slot(scatter, vdt, k)] = plan;
    return SPW_OK;
}

spw_status spw_set_batch_plan(spw_matrix A, spw_op op, spw_dtype vdt, int32_t k, spw_plan plan)
{
    return guarded("spw_set_batch_plan", [&] { return set_batch_plan_impl(A, op, vdt, k, plan); });
}

static spw_status spw_mv_impl(spw_matrix A, spw_dtype vdt, const void *x, void *y, void *stream)
{
    return run_product(A, true, vdt, 1, x, 1, y, 1, stream, "spw_mv");
}

spw_status spw_mv(spw_matrix A, spw_dtype vdt, const void *x, void *y, void *stream)
{
    return guarded("spw_mv", [&] { return spw_mv_impl(A, vdt, x, y, stream); });
}

static spw_status spw_vtm_impl(spw_matrix A, spw_dtype vdt, const void *v, void *u, void *stream)
{
    return run_product(A, false, vdt, 1, v, 1, u, 1, stream, "spw_vtm");
}

spw_status spw_vtm(spw_matrix A, spw_dtype vdt, const void *v, void *u, void *stream)
{
    return guarded("spw_vtm", [&] { return spw_vtm_impl(A, vdt, v, u, stream); });
}

static spw_status spw_mv_batch_impl(spw_matrix A, spw_dtype vdt, int32_t k, const void *X, int64_t ldx, void *Y,
                                    int64_t ldy, void *stream)
{
    return run_product(A, true, vdt, k, X, ldx, Y, ldy, stream, "spw_mv_batch");
}

spw_status spw_mv_batch(spw_matrix A, spw_dtype vdt, int32_t k, const void *X, int64_t ldx, void *Y, int64_t ldy,
                        void *stream)
{
    return guarded("spw_mv_batch", [&] { return spw_mv_batch_impl(A, vdt, k, X, ldx, Y, ldy, stream); });
}

static spw_status spw_vtm_batch_impl(spw_matrix A, spw_dtype vdt, int32_t k, const void *V, int64_t ldv, void *U,
                                     int64_t ldu, void *stream)
{
    return run_product(A, false, vdt, k, V, ldv, U, ldu, stream, "spw_vtm_batch");
}

spw_status spw_vtm_batch(spw_matrix A, spw_dtype vdt, int32_t k, const void *V, int64_t ldv, void *U, int64_t ldu,
                         void *stream)
{
    return guarded("spw_vtm_batch", [&] { return spw_vtm_batch_impl(A, vdt, k, V, ldv, U, ldu, stream); });
}

// Iterations between direct products q = A p in the CGLS loop.
constexpr int64_t CGLS_REFRESH = 50;

static spw_status spw_cgls_impl(spw_matrix A, spw_dtype vdt, const void *b, void *x, int32_t iters, double *hist,
                                void *stream)
{
    if (!A) return fail(SPW_ERR_INVALID_ARG, "spw_cgls: NULL matrix");
    if (vdt != SPW_F64) return fail(SPW_ERR_UNSUPPORTED, "spw_cgls: binary64 vectors only");
    if (iters < 0) return fail(SPW_ERR_INVALID_ARG, "spw_cgls: iters must be >= 0");
    if ((A->m > 0 && !b) || (A->n > 0 && !x)) return fail(SPW_ERR_INVALID_ARG, "spw_cgls: NULL vector");
    DeviceGuard dg(A->device);
    if (dg.st) return dg.st;
    // refuse a busy matrix before any workspace is reallocated
    spw_status st = claim_stream(*A, stream, "spw_cgls");
    if (st) return st;
    if ((st = grow_scratch(*A, 1))) return st;
    const int64_t hl = 2 * ((int64_t)iters + 1);
    if ((st = grow_cgls(*A, hl))) return st;
    CglsScratch &W = A->cgls;
    CglsWork w;
    w.m = A->m;
    w.n = A->n;
    w.b = (const double *)b;
    w.x = (double *)x;
    w.r = W.r;
    w.q = W.q;
    w.t = W.t;
    w.s = W.s;
    w.p = W.p;
    w.partial = W.partial;
    w.scal = W.scal;
    w.hist_gamma = W.hist;
    w.hist_rho = W.hist + iters + 1;
    auto vec = [&](CglsVecOp op) -> spw_status {
        const int e = launch_cgls_vec(op, w, stream);
        if (e) return fail(SPW_ERR_DEVICE, std::string("spw_cgls: kernel launch failed: ") +
                                               hipGetErrorString((hipError_t)e));
        return SPW_OK;
    };
    // one iteration k: t = A s_k, q_k = t + beta_k q_{k-1} (= A p_k), alpha_k, r_{k+1};
    // p_k = s_k + beta_k p_{k-1}, x_{k+1} = x_k + alpha_k p_k; s_{k+1} = A^T r_{k+1}, gamma_{k+1},
    // beta_{k+1}.  The first iteration takes q_0 = t and p_0 = s_0.  Every CGLS_REFRESH-th
    // iteration forms p_k first and takes q_k = A p_k with a product of its own, so the
    // rounding that the linear recurrence for q gathers is dropped at that point.
    auto iteration = [&](bool first, bool refresh) -> spw_status {
        spw_status s2;
        if (refresh) {
            if ((s2 = vec(CglsVecOp::P))) return s2;                                                   // p = s + beta p
            if ((s2 = run_product(A, true, SPW_F64, 1, w.p, 1, w.t, 1, stream, "spw_cgls"))) return s2;  // t = A p
            if ((s2 = vec(CglsVecOp::ALPHA_R0))) return s2;                                            // q = t
            if ((s2 = vec(CglsVecOp::X))) return s2;
        } else {
            if ((s2 = run_product(A, true, SPW_F64, 1, w.s, 1, w.t, 1, stream, "spw_cgls"))) return s2;   // t = A s
            if ((s2 = vec(first ? CglsVecOp::ALPHA_R0 : CglsVecOp::ALPHA_R))) return s2;
            if ((s2 = vec(first ? CglsVecOp::PX0 : CglsVecOp::PX))) return s2;
        }
        if ((s2 = run_product(A, false, SPW_F64, 1, w.r, 1, w.s, 1, stream, "spw_cgls"))) return s2;  // s = A^T r
        return vec(CglsVecOp::GAMMA);
    };
    // r_0 = b - A x_0, s_0 = A^T r_0, gamma_0 = ||s_0||^2
    if ((st = run_product(A, true, SPW_F64, 1, x, 1, w.q, 1, stream, "spw_cgls"))) return st;
    if ((st = vec(CglsVecOp::R_INIT))) return st;
    if ((st = run_product(A, false, SPW_F64, 1, w.r, 1, w.s, 1, stream, "spw_cgls"))) return st;
    if ((st = vec(CglsVecOp::GAMMA0))) return st;
    // Every iteration after the first launches the same kernels with the same
    // arguments (the history index lives on the device), so a caller may
    // capture a whole call without a history in a graph and replay it.
    for (int64_t k = 1; k <= iters; ++k)
        if ((st = iteration(k == 1, k > 1 && k % CGLS_REFRESH == 0))) return st;
    if ((st = release_stream(*A, stream, "spw_cgls"))) return st;
    if (hist) {
        if (hipMemcpyAsync(hist, W.hist, (size_t)hl * sizeof(double), hipMemcpyDeviceToHost, (hipStream_t)stream) !=
                hipSuccess ||
            hipStreamSynchronize((hipStream_t)stream) != hipSuccess) {
            (void)hipGetLastError();
            return fail(SPW_ERR_DEVICE, "spw_cgls: copying the history failed");
        }
    }
    return SPW_OK;
}

spw_status spw_cgls(spw_matrix A, spw_dtype vdt, const void *b, void *x, int32_t iters, double *hist, void *stream)
{
    return guarded("spw_cgls", [&] { return spw_cgls_impl(A, vdt, b, x, iters, hist, stream); });
}

static spw_status spw_round_values_impl(spw_dtype storage, int64_t n, const double *in, double *out)
{
    if (storage != SPW_F64 && storage != SPW_F32 && storage != SPW_BF16)
        return fail(SPW_ERR_INVALID_ARG, "spw_round_values: bad storage type");
    if (n < 0 || (n > 0 && (!in || !out))) return fail(SPW_ERR_INVALID_ARG, "spw_round_values: bad argument");
    const int64_t bad = round_values(storage, n, in, out);
    if (bad >= 0)
        return fail(SPW_ERR_BAD_MATRIX, "position " + std::to_string(bad) + ": value overflows the storage type");
    return SPW_OK;
}

spw_status spw_round_values(spw_dtype storage, int64_t n, const double *in, double *out)
{
    return guarded("spw_round_values", [&] { return spw_round_values_impl(storage, n, in, out); });
}

static spw_status spw_plan_zones_impl(int64_t n, const int64_t *ptr, int64_t chunk_nnz, int64_t *n_chunks,
                                      int64_t *n_zones, int64_t *chunk_owned, int64_t *zone_col, int64_t *zone_first,
                                      int64_t *zone_last)
{
    if (n < 0 || !ptr || chunk_nnz <= 0 || !n_chunks || !n_zones)
        return fail(SPW_ERR_INVALID_ARG, "spw_plan_zones: bad argument");
    if (ptr[0] != 0) return fail(SPW_ERR_BAD_MATRIX, "spw_plan_zones: ptr[0] must be 0");
    for (int64_t j = 0; j < n; ++j)
        if (ptr[j + 1] < ptr[j]) return fail(SPW_ERR_BAD_MATRIX, "spw_plan_zones: ptr decreases at " + std::to_string(j));
    if (ptr[n] >= ((int64_t)1 << 31) || n >= ((int64_t)1 << 31) - 1)
        return fail(SPW_ERR_UNSUPPORTED, "spw_plan_zones: sizes must stay below 2^31");
    ZonePlan zp;
    build_zone_plan(n, ptr, chunk_nnz, zp);
    *n_chunks = zp.n_chunks;
    *n_zones = (int64_t)zp.zone_col.size();
    if (chunk_owned)
        for (size_t c = 0; c < zp.owned.size(); ++c) chunk_owned[c] = zp.owned[c];
    for (size_t k = 0; k < zp.zone_col.size(); ++k) {
        if (zone_col) zone_col[k] = zp.zone_col[k];
        if (zone_first) zone_first[k] = zp.zone_first[k];
        if (zone_last) zone_last[k] = zp.zone_last[k];
    }
    return SPW_OK;
}

spw_status spw_plan_zones(int64_t n, const int64_t *ptr, int64_t chunk_nnz, int64_t *n_chunks, int64_t *n_zones,
                          int64_t *chunk_owned, int64_t *zone_col, int64_t *zone_first, int64_t *zone_last)
{
    return guarded("spw_plan_zones", [&] {
        return spw_plan_zones_impl(n, ptr, chunk_nnz, n_chunks, n_zones, chunk_owned, zone_col, zone_first, zone_last);
    });
}

}  // extern "C"
