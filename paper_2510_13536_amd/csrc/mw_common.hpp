// mw_common.hpp -- launch geometry, reductions and host helpers shared by
// the libmwcg kernels (gfx950, wave64).
#pragma once

#include <hip/hip_ext.h>
#include <hip/hip_runtime.h>

#include <cstdint>
#include <cstdio>

#include "mw.h"
#include "mw_arith.hpp"

namespace mwk {

constexpr int NT = 256;          // threads per workgroup of the streaming kernels
constexpr int NWAVE = NT / 64;   // wavefronts per workgroup
constexpr int FIN_NT = 1024;     // threads of the one-workgroup finalisers
constexpr int MAX_GRID = 2048;   // workgroups of the persistent streaming kernels
constexpr int NXCD = 8;          // XCDs per MI355X; workgroups are dealt to them round-robin

// ------------------------------------------------------- tile scheduling
//
// Persistent streaming kernels walk "tiles" (units of NT rows).  The tile
// range is split into NXCD contiguous parts; workgroup b runs on XCD b % 8
// and takes the tiles of that XCD's part with a stride equal to the number
// of workgroups on that XCD.  Neighbouring rows are thus handled inside one
// XCD and share its L2.  The assignment is static, so any per-workgroup
// partial sum has a fixed association.  Requires gridDim.x >= min(8, ntiles).
struct TileRange {
    int first, end, step;
};

__device__ __forceinline__ TileRange xcd_tiles(int ntiles)
{
    const int G = gridDim.x;
    const int xcd = blockIdx.x & (NXCD - 1), j = blockIdx.x / NXCD;
    const int nbx = G / NXCD + (xcd < (G & (NXCD - 1)) ? 1 : 0);
    const int q = ntiles / NXCD, rem = ntiles & (NXCD - 1);
    const int t0 = xcd * q + (xcd < rem ? xcd : rem);
    const int t1 = t0 + q + (xcd < rem ? 1 : 0);
    return TileRange{t0 + j, t1, nbx};
}

// The m-th tile of the range, walking the XCD's part forwards (rev = 0) or
// backwards (rev = 1).  Consecutive kernels that walk in opposite
// directions start on the rows the previous kernel touched last, which are
// the most likely to still be in the Infinity Cache.
struct TileWalk {
    int base, count, step, rev;
    __device__ __forceinline__ int operator[](int m) const { return rev ? base - m * step : base + m * step; }
};

__device__ __forceinline__ TileWalk xcd_walk(int ntiles, int rev)
{
    const TileRange r = xcd_tiles(ntiles);
    const int t0 = r.first - (int)(blockIdx.x / NXCD);  // first tile of the XCD's part
    const int len = r.end - t0;
    const int j = (int)(blockIdx.x / NXCD);
    const int count = (j < len) ? (len - j + r.step - 1) / r.step : 0;
    return TileWalk{rev ? r.end - 1 - j : r.first, count, r.step, rev};
}

// Index of the calling wavefront inside its workgroup, as a wave-uniform
// (scalar) value, so per-slice bounds are scalar loads and loops over a
// slice are scalar loops.
__device__ __forceinline__ int wave_id() { return __builtin_amdgcn_readfirstlane(threadIdx.x >> 6); }

// Grid size of a persistent streaming kernel over ntiles tiles.
inline int persistent_grid(long ntiles)
{
    return (int)(ntiles < MAX_GRID ? (ntiles > 0 ? ntiles : 1) : MAX_GRID);
}

// Workgroup index remap for one-tile-per-workgroup kernels: XCD x gets the
// x-th contiguous range of logical workgroups.
__device__ __forceinline__ int xcd_remap(int bid, int nb)
{
    const int q = nb / NXCD, rem = nb & (NXCD - 1);
    const int x = bid & (NXCD - 1), j = bid / NXCD;
    return x * q + (x < rem ? x : rem) + j;
}

// ------------------------------------------------------------ reductions

// Sum over a workgroup of NTHR threads; result valid in thread 0.  Order:
// shuffle tree inside each wavefront (offsets 32, 16, ..., 1), then the
// wavefront sums pairwise (a fixed binary tree over wavefront index).
template <int A, int NTHR>
__device__ __forceinline__ Num<A> block_sum(Num<A> v)
{
    constexpr int NW = NTHR / 64;
    __shared__ Num<A> part[NW];
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v = add<A>(v, shfl_down<A>(v, off));
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    if (lane == 0) part[wid] = v;
    __syncthreads();
    if (threadIdx.x == 0) {
#pragma unroll
        for (int s = 1; s < NW; s <<= 1)
#pragma unroll
            for (int i = 0; i + s < NW; i += 2 * s) part[i] = add<A>(part[i], part[i + s]);
        v = part[0];
    }
    __syncthreads();
    return v;
}

// Sum of nslots k-word partials (slot s at slots + s*K) by one FIN_NT
// workgroup: thread t adds slots t, t + FIN_NT, ... in order (loads issued
// ahead of the dependent adds), then block_sum.
template <int A, int NTHR = FIN_NT>
__device__ __forceinline__ Num<A> reduce_slots(int nslots, const double *__restrict__ slots)
{
    constexpr int K = words(A);
    constexpr int B = 4;
    Num<A> acc = zero<A>();
    for (int s0 = threadIdx.x; s0 < nslots; s0 += NTHR * B) {
        Num<A> v[B];
#pragma unroll
        for (int u = 0; u < B; ++u) {
            const int s = s0 + u * NTHR;
            v[u] = (s < nslots) ? load_scalar<A>(slots + (long)s * K) : zero<A>();
        }
#pragma unroll
        for (int u = 0; u < B; ++u)
            if (s0 + u * NTHR < nslots) acc = add<A>(acc, v[u]);
    }
    return block_sum<A, NTHR>(acc);
}

// acc + x*y as a dot-product step (FP64: one fma).
template <int A>
__device__ __forceinline__ Num<A> dot_step(const Num<A> &acc, const Num<A> &x, const Num<A> &y)
{
    if constexpr (A == FP64) return promote<A>(__builtin_fma(x.w[0], y.w[0], acc.w[0]));
    else return add<A>(acc, mul<A>(x, y));
}

// One step of a row sum: acc + a*x (FP64: fma; else FP64 x multi-word).
template <int A>
__device__ __forceinline__ Num<A> row_step(const Num<A> &acc, double a, const Num<A> &x)
{
    if constexpr (A == FP64) return promote<A>(__builtin_fma(a, x.w[0], acc.w[0]));
    else return add<A>(acc, dxmul<A>(a, x));
}

}  // namespace mwk

// ------------------------------------------------------------ host side

namespace mwh {

int hip_fail(hipError_t e, const char *what);
void set_error(const char *msg);
void clear_error();  // at the entry of every status-returning ABI call

inline int blocks_for(long n, long per) { return (int)((n + per - 1) / per); }
inline size_t align256(size_t b) { return (b + 255) & ~(size_t)255; }
inline bool valid_arith(int a) { return a >= MW_FP64 && a <= MW_MXQTW; }
inline bool mixed_arith(int a) { return a == MW_MXDW || a == MW_MXQTW; }
// A size the library takes (0 .. MW_MAX_N); a larger one also leaves a
// message for mw_last_error.
inline bool size_ok(long n)
{
    if (n > MW_MAX_N) set_error("n or nnz exceeds MW_MAX_N (2^31 - 2^16)");
    return n >= 0 && n <= MW_MAX_N;
}
inline bool valid_csr(const mw_csr_t *A)
{
    return A && A->n > 0 && A->nnz >= 0 && size_ok(A->n) && size_ok(A->nnz) && A->row_ptr && A->col_idx && A->val;
}

// The library's own stream for the calling thread on the current device
// (default priority, non-blocking: graph capture is not possible on the
// legacy default stream a caller may pass).  One per (thread, device, use),
// created at first use; nullptr when it cannot be created.
constexpr int MAX_DEVICES = 64;
template <int USE>
hipStream_t thread_stream()
{
    thread_local hipStream_t s[MAX_DEVICES] = {};
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= MAX_DEVICES) {
        (void)hipGetLastError();
        return nullptr;
    }
    if (!s[dev] && hipStreamCreateWithFlags(&s[dev], hipStreamNonBlocking) != hipSuccess) {
        (void)hipGetLastError();
        s[dev] = nullptr;
    }
    return s[dev];
}

}  // namespace mwh

#define HIP_TRY(call)                                              \
    do {                                                           \
        hipError_t e_ = (call);                                    \
        if (e_ != hipSuccess) return mwh::hip_fail(e_, #call);     \
    } while (0)

// The events that order a solve after the caller's stream (`in`) and time
// it (t0, t1); destroyed on every return path of the solve.
struct SolveEvents {
    hipEvent_t in = nullptr, t0 = nullptr, t1 = nullptr;
    SolveEvents() = default;
    SolveEvents(const SolveEvents &) = delete;
    SolveEvents &operator=(const SolveEvents &) = delete;
    ~SolveEvents()
    {
        if (in) (void)hipEventDestroy(in);
        if (t0) (void)hipEventDestroy(t0);
        if (t1) (void)hipEventDestroy(t1);
    }
    // Creates the three events, makes `own` wait for the work enqueued on
    // `user` so far and records t0 on `own`.
    int start(hipStream_t user, hipStream_t own)
    {
        HIP_TRY(hipEventCreateWithFlags(&in, hipEventDisableTiming));
        HIP_TRY(hipEventCreate(&t0));
        HIP_TRY(hipEventCreate(&t1));
        HIP_TRY(hipEventRecord(in, user));
        HIP_TRY(hipStreamWaitEvent(own, in, 0));
        HIP_TRY(hipEventRecord(t0, own));
        return 0;
    }
};

// Kernel launch; given a pair of events, they are attached to the dispatch
// itself (hipExtLaunchKernelGGL), so their elapsed time is the kernel's
// execution alone.
#define MW_LAUNCH(kern, grid, block, stream, ev0, ev1, ...)                                  \
    do {                                                                                       \
        if (ev0) hipExtLaunchKernelGGL(kern, grid, block, 0, stream, ev0, ev1, 0, __VA_ARGS__); \
        else hipLaunchKernelGGL(kern, grid, block, 0, stream, __VA_ARGS__);                     \
    } while (0)

// Every arithmetic but the mixed ones (callers reject those first).
#define MW_DISPATCH_WORDS(a, fn, ...)                    \
    switch (a) {                                         \
    case MW_FP64: return fn<mwk::FP64>(__VA_ARGS__);     \
    case MW_DW: return fn<mwk::DW>(__VA_ARGS__);         \
    case MW_QDW: return fn<mwk::QDW>(__VA_ARGS__);       \
    case MW_TW: return fn<mwk::TW>(__VA_ARGS__);         \
    case MW_QTW: return fn<mwk::QTW>(__VA_ARGS__);       \
    case MW_QTWE: return fn<mwk::QTWE>(__VA_ARGS__);     \
    case MW_QW: return fn<mwk::QW>(__VA_ARGS__);         \
    default: return fn<mwk::QQW>(__VA_ARGS__);           \
    }

// Every arithmetic.
#define MW_DISPATCH(a, fn, ...)                          \
    switch (a) {                                         \
    case MW_MXDW: return fn<mwk::MXDW>(__VA_ARGS__);     \
    case MW_MXQTW: return fn<mwk::MXQTW>(__VA_ARGS__);   \
    default: MW_DISPATCH_WORDS(a, fn, __VA_ARGS__)       \
    }
