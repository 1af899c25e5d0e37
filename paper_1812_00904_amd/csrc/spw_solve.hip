// Vector kernels of the CGLS loop (conjugate gradients on min ||b - A x||_2),
// the first-order use of the two products that the paper's closing section
// describes: each iteration is one product with A, one with A^T, and a few
// passes of vector updates and inner products, which this file fuses.
//
// The product with A is taken of s = A^T r, and q = A p is formed from it by
// linearity (p = s + beta p, so q = A s + beta q).  This leaves the update of
// the two long vectors (p, then x) free to run right before the A^T r product,
// whose scattered gathers leave memory bandwidth to spare for writing them
// back, instead of right before the A p product, whose streaming they slowed.
//
// Every inner product is formed in a fixed order, so a solve is bit-identical
// from run to run: DOT_PARTS workgroups each sum a fixed contiguous range
// (thread t adds elements t, t + BLOCK, ... of the range in order, then a
// fixed butterfly inside each wave and the waves in ascending order), and one
// workgroup adds the DOT_PARTS partial sums the same way.  The step sizes stay
// on the device: the scalar kernel that finishes an inner product also forms
// alpha or beta, so the loop never waits for the host.
//
// Scalars slot layout (binary64): [0] gamma = ||A^T r||^2 of the current
// iterate, [1] alpha, [2] beta, [3] the iteration the history is at (an
// integer, so one captured iteration can be replayed unchanged).
#include <hip/hip_runtime.h>

#include <cstdint>

#include "spw_internal.h"

namespace spw {
namespace {

constexpr int SV_BLOCK = 256;
constexpr int SV_WAVE = 64;
constexpr int DOT_PARTS = 1024;          // partial sums per inner product (one per workgroup)
constexpr int S_GAMMA = 0, S_ALPHA = 1, S_BETA = 2, S_ITER = 3;

// Sum of one value per thread over a workgroup of SV_BLOCK threads, in a fixed
// order: butterfly inside each wave, then the waves in ascending order.  The
// result is valid in thread 0.
__device__ __forceinline__ double block_sum(double v, double *lds)
{
    for (int off = SV_WAVE / 2; off > 0; off >>= 1) v += __shfl_xor(v, off, SV_WAVE);
    const int wave = threadIdx.x / SV_WAVE, lane = threadIdx.x % SV_WAVE;
    if (lane == 0) lds[wave] = v;
    __syncthreads();
    double s = 0.0;
    if (threadIdx.x == 0)
        for (int w = 0; w < SV_BLOCK / SV_WAVE; ++w) s += lds[w];
    return s;
}

// Range of workgroup g out of DOT_PARTS over len elements.
__device__ __forceinline__ void part_range(int64_t len, int64_t &a, int64_t &e)
{
    a = len * (int64_t)blockIdx.x / DOT_PARTS;
    e = len * ((int64_t)blockIdx.x + 1) / DOT_PARTS;
}

// partial[g] = sum over workgroup g's range of a_i * a_i.  Eight loads are
// issued before their squares are added (in the same order as one at a time),
// so that more bytes are in flight.
__global__ __launch_bounds__(SV_BLOCK) void sq_part(const double *__restrict__ a, int64_t len,
                                                    double *__restrict__ partial)
{
    __shared__ double lds[SV_BLOCK / SV_WAVE];
    int64_t s, e;
    part_range(len, s, e);
    double acc = 0.0;
    int64_t i = s + threadIdx.x;
    for (; i + 7 * SV_BLOCK < e; i += 8 * SV_BLOCK) {
        double t[8];
#pragma unroll
        for (int u = 0; u < 8; ++u) t[u] = a[i + u * SV_BLOCK];
#pragma unroll
        for (int u = 0; u < 8; ++u) acc += t[u] * t[u];
    }
    for (; i < e; i += SV_BLOCK) acc += a[i] * a[i];
    const double t = block_sum(acc, lds);
    if (threadIdx.x == 0) partial[blockIdx.x] = t;
}

// FIRST: q = t.  Otherwise q = t + beta q.  Either way partial[g] = sum of
// q_i * q_i of the new q over workgroup g's range.
template <bool FIRST>
__global__ __launch_bounds__(SV_BLOCK) void q_step(double *__restrict__ q, const double *__restrict__ t, int64_t len,
                                                   const double *__restrict__ scal, double *__restrict__ partial)
{
    __shared__ double lds[SV_BLOCK / SV_WAVE];
    const double beta = FIRST ? 0.0 : scal[S_BETA];
    int64_t s, e;
    part_range(len, s, e);
    double acc = 0.0;
    for (int64_t i = s + threadIdx.x; i < e; i += SV_BLOCK) {
        const double qi = FIRST ? t[i] : t[i] + beta * q[i];
        q[i] = qi;
        acc += qi * qi;
    }
    const double sum = block_sum(acc, lds);
    if (threadIdx.x == 0) partial[blockIdx.x] = sum;
}

// INIT: r = b - q.  UPDATE: r = r - alpha q.  Either way partial[g] = sum of
// r_i * r_i of the new r over workgroup g's range.
template <bool INIT>
__global__ __launch_bounds__(SV_BLOCK) void r_step(double *__restrict__ r, const double *__restrict__ b,
                                                   const double *__restrict__ q, int64_t len,
                                                   const double *__restrict__ scal, double *__restrict__ partial)
{
    __shared__ double lds[SV_BLOCK / SV_WAVE];
    const double alpha = INIT ? 0.0 : scal[S_ALPHA];
    int64_t s, e;
    part_range(len, s, e);
    double acc = 0.0;
    for (int64_t i = s + threadIdx.x; i < e; i += SV_BLOCK) {
        const double ri = INIT ? b[i] - q[i] : r[i] - alpha * q[i];
        r[i] = ri;
        acc += ri * ri;
    }
    const double t = block_sum(acc, lds);
    if (threadIdx.x == 0) partial[blockIdx.x] = t;
}

// What the scalar kernel does with the finished inner product.  Iteration k
// (the history index) is scal[S_ITER]: 0 during the start-up, set to 1 by
// OP_GAMMA0 and advanced by OP_GAMMA, the last scalar step of an iteration.
enum ScalarOp : int {
    OP_GAMMA0 = 0,   // gamma = sum, hist_gamma[0] = sum, k = 1
    OP_ALPHA = 1,    // delta = sum, alpha = gamma / delta (0 when either is 0)
    OP_GAMMA = 2,    // gamma_new = sum, beta = gamma_new / gamma (0 when gamma is 0), gamma = gamma_new,
                     // hist_gamma[k] = sum, k = k + 1
    OP_RHO = 3,      // hist_rho[k] = sum
    OP_RHO0 = 4      // hist_rho[0] = sum, k = 0
};

// One workgroup: adds the DOT_PARTS partial sums in a fixed order and applies op.
__global__ __launch_bounds__(SV_BLOCK) void scalar_step(const double *__restrict__ partial, int op,
                                                        double *__restrict__ scal, double *__restrict__ hist_gamma,
                                                        double *__restrict__ hist_rho)
{
    __shared__ double lds[SV_BLOCK / SV_WAVE];
    double acc = 0.0;
    for (int i = threadIdx.x; i < DOT_PARTS; i += SV_BLOCK) acc += partial[i];
    const double sum = block_sum(acc, lds);
    if (threadIdx.x != 0) return;
    const int64_t k = (int64_t)scal[S_ITER];
    if (op == OP_RHO0) {
        scal[S_ITER] = 0.0;
        hist_rho[0] = sum;
    } else if (op == OP_GAMMA0) {
        scal[S_GAMMA] = sum;
        hist_gamma[0] = sum;
        scal[S_ITER] = 1.0;
    } else if (op == OP_ALPHA) {
        const double gamma = scal[S_GAMMA];
        scal[S_ALPHA] = (gamma > 0.0 && sum > 0.0) ? gamma / sum : 0.0;
    } else if (op == OP_GAMMA) {
        const double gamma = scal[S_GAMMA];
        scal[S_BETA] = gamma > 0.0 ? sum / gamma : 0.0;
        scal[S_GAMMA] = sum;
        hist_gamma[k] = sum;
        scal[S_ITER] = (double)(k + 1);
    } else {
        hist_rho[k] = sum;
    }
}

// p = s + beta p (FIRST: p = s), then x = x + alpha p with the new p: one
// pass over the three long vectors.
template <bool FIRST>
__global__ __launch_bounds__(SV_BLOCK) void px_step(double *__restrict__ x, double *__restrict__ p,
                                                    const double *__restrict__ s, int64_t len,
                                                    const double *__restrict__ scal)
{
    const double alpha = scal[S_ALPHA], beta = FIRST ? 0.0 : scal[S_BETA];
    const int64_t stride = (int64_t)gridDim.x * SV_BLOCK;
    for (int64_t i = blockIdx.x * (int64_t)SV_BLOCK + threadIdx.x; i < len; i += stride) {
        const double pi = FIRST ? s[i] : s[i] + beta * p[i];
        p[i] = pi;
        x[i] = x[i] + alpha * pi;
    }
}

// The two halves of px_step for an iteration that forms q = A p directly:
// p = s + beta p before the product, x = x + alpha p after alpha is known.
__global__ __launch_bounds__(SV_BLOCK) void p_step(double *__restrict__ p, const double *__restrict__ s, int64_t len,
                                                   const double *__restrict__ scal)
{
    const double beta = scal[S_BETA];
    const int64_t stride = (int64_t)gridDim.x * SV_BLOCK;
    for (int64_t i = blockIdx.x * (int64_t)SV_BLOCK + threadIdx.x; i < len; i += stride) p[i] = s[i] + beta * p[i];
}

__global__ __launch_bounds__(SV_BLOCK) void x_step(double *__restrict__ x, const double *__restrict__ p, int64_t len,
                                                   const double *__restrict__ scal)
{
    const double alpha = scal[S_ALPHA];
    const int64_t stride = (int64_t)gridDim.x * SV_BLOCK;
    for (int64_t i = blockIdx.x * (int64_t)SV_BLOCK + threadIdx.x; i < len; i += stride) x[i] = x[i] + alpha * p[i];
}

unsigned stream_grid(int64_t len)
{
    const int64_t g = (len + SV_BLOCK - 1) / SV_BLOCK;
    return (unsigned)(g < 1 ? 1 : (g > 16384 ? 16384 : g));
}

}  // namespace

int64_t cgls_dot_parts() { return DOT_PARTS; }

int launch_cgls_vec(CglsVecOp op, const CglsWork &w, void *stream)
{
    hipStream_t st = (hipStream_t)stream;
    auto scalar = [&](ScalarOp sop) {
        hipLaunchKernelGGL(scalar_step, dim3(1), dim3(SV_BLOCK), 0, st, w.partial, (int)sop, w.scal, w.hist_gamma,
                           w.hist_rho);
    };
    switch (op) {
    case CglsVecOp::R_INIT:     // r = b - q, rho_0
        hipLaunchKernelGGL(r_step<true>, dim3(DOT_PARTS), dim3(SV_BLOCK), 0, st, w.r, w.b, w.q, w.m, w.scal, w.partial);
        scalar(OP_RHO0);
        break;
    case CglsVecOp::GAMMA0:     // gamma_0 = ||s||^2
        hipLaunchKernelGGL(sq_part, dim3(DOT_PARTS), dim3(SV_BLOCK), 0, st, w.s, w.n, w.partial);
        scalar(OP_GAMMA0);
        break;
    case CglsVecOp::ALPHA_R0:   // q = t, alpha = gamma / ||q||^2, r = r - alpha q, rho_k
    case CglsVecOp::ALPHA_R:    // q = t + beta q, the same
        if (op == CglsVecOp::ALPHA_R0)
            hipLaunchKernelGGL(q_step<true>, dim3(DOT_PARTS), dim3(SV_BLOCK), 0, st, w.q, w.t, w.m, w.scal, w.partial);
        else
            hipLaunchKernelGGL(q_step<false>, dim3(DOT_PARTS), dim3(SV_BLOCK), 0, st, w.q, w.t, w.m, w.scal, w.partial);
        scalar(OP_ALPHA);
        hipLaunchKernelGGL(r_step<false>, dim3(DOT_PARTS), dim3(SV_BLOCK), 0, st, w.r, w.b, w.q, w.m, w.scal, w.partial);
        scalar(OP_RHO);
        break;
    case CglsVecOp::PX0:        // p = s, x = x + alpha p
        hipLaunchKernelGGL(px_step<true>, dim3(stream_grid(w.n)), dim3(SV_BLOCK), 0, st, w.x, w.p, w.s, w.n, w.scal);
        break;
    case CglsVecOp::PX:         // p = s + beta p, x = x + alpha p
        hipLaunchKernelGGL(px_step<false>, dim3(stream_grid(w.n)), dim3(SV_BLOCK), 0, st, w.x, w.p, w.s, w.n, w.scal);
        break;
    case CglsVecOp::P:          // p = s + beta p
        hipLaunchKernelGGL(p_step, dim3(stream_grid(w.n)), dim3(SV_BLOCK), 0, st, w.p, w.s, w.n, w.scal);
        break;
    case CglsVecOp::X:          // x = x + alpha p
        hipLaunchKernelGGL(x_step, dim3(stream_grid(w.n)), dim3(SV_BLOCK), 0, st, w.x, w.p, w.n, w.scal);
        break;
    case CglsVecOp::GAMMA:      // gamma_k = ||s||^2, beta
        hipLaunchKernelGGL(sq_part, dim3(DOT_PARTS), dim3(SV_BLOCK), 0, st, w.s, w.n, w.partial);
        scalar(OP_GAMMA);
        break;
    }
    return (int)hipGetLastError();
}

}  // namespace spw
