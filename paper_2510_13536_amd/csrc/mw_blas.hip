// mw_blas.hip -- element-wise operations, AXPY, DOT and SpMV of libmwcg
// (gfx950).  Method: Mukunoki & Ozaki, arXiv 2510.13536, Sec. III (the
// multi-word algorithms) and Sec. IV-B (CSR SpMV, DOT, AXPY).
//
// SpMV kernels
//   mw_csr_spmv_kernel   CSR input as given.  A workgroup owns NT rows;
//                        its nonzeros are streamed through LDS in coalesced
//                        chunks (each thread forms FP64 x multi-word
//                        products), then every row's thread adds its own
//                        products in CSR order.
//   mw_sell_spmv_kernel  the planned form (SELL-64): slices of 64 rows, one
//                        wavefront per slice and one lane per row, entries
//                        stored in pairs so every wavefront load of values
//                        (and column indices) is contiguous.  A slice whose
//                        rows fit diagonal slots (one column offset per
//                        slot, stencil and banded rows) stores no column
//                        indices: the gather address is row + offset, the
//                        slot's lane mask skips rows without that entry.
//                        Other slices keep explicit columns; padding
//                        entries (col -1) are skipped, not added as zeros.
// Both sum every row sequentially from zero in CSR order, so both are
// bit-identical to that definition, whatever the launch shape.
//   mw_vec_spmv_kernel   the vector-row plan (MW_FMT_CSRVEC), for matrices
//                        with few, long rows: L lanes per row, lane t adds
//                        the row's entries t, t + L, t + 2L, ... in order
//                        from zero, then the L partial sums are combined by
//                        a fixed halving tree.  Deterministic; the row's
//                        sum is associated differently from CSR order
//                        (longest accumulation path ceil(len / L) + log2 L
//                        operations instead of len).
#include "mw_blas.hpp"

#include <cstdlib>
#include <cstring>
#include <mutex>

using namespace mwk;

// ================================================================ host errors

namespace mwh {

thread_local char g_err[256] = "";

int hip_fail(hipError_t e, const char *what)
{
    snprintf(g_err, sizeof(g_err), "%s: %s", what, hipGetErrorString(e));
    return MW_EHIP;
}

void set_error(const char *msg) { snprintf(g_err, sizeof(g_err), "%s", msg); }

void clear_error() { g_err[0] = 0; }

}  // namespace mwh

namespace {

using namespace mwh;


constexpr int DOT_EPT = 8;        // elements per thread in the standalone dot
constexpr int CSR_NPT = 4;        // nonzeros per thread per LDS chunk (CSR SpMV)

// ------------------------------------------------------------ element-wise

template <int A, int OP>
__global__ void __launch_bounds__(NT) mw_elementwise_kernel(int n, const double *u, const double *v, double *w)
{
    const long i = (long)blockIdx.x * NT + threadIdx.x;
    if (i >= n) return;
    if constexpr (OP == MW_OP_TOFP64) {
        const double r = to_fp64<A>(load<A>(u, n, i));
        w[i] = r;
    } else if constexpr (OP == MW_OP_DXMUL) {
        const double a = u[i];
        const Num<A> r = dxmul<A>(a, load<A>(v, n, i));
        store<A>(w, n, i, r);
    } else {
        const Num<A> a = load<A>(u, n, i);
        Num<A> r;
        if constexpr (OP == MW_OP_ADD) r = add<A>(a, load<A>(v, n, i));
        else if constexpr (OP == MW_OP_MUL) r = mul<A>(a, load<A>(v, n, i));
        else if constexpr (OP == MW_OP_DIV) r = div<A>(a, load<A>(v, n, i));
        else if constexpr (OP == MW_OP_NORM) r = normalise<A>(a);
        else r = neg<A>(a);
        store<A>(w, n, i, r);
    }
}

template <int A>
__global__ void __launch_bounds__(NT) mw_axpy_kernel(int n, const double *__restrict__ alpha,
                                                     const double *__restrict__ x, double *__restrict__ y)
{
    const long i = (long)xcd_remap(blockIdx.x, gridDim.x) * NT + threadIdx.x;
    if (i >= n) return;
    const Num<A> al = load_scalar<A>(alpha);
    store<A>(y, n, i, axpy_term<A>(al, load<A>(x, n, i), load<A>(y, n, i)));
}

// --------------------------------------------------------------------- dot

template <int A>
__global__ void __launch_bounds__(NT) mw_dot_partial_kernel(int n, const double *__restrict__ x,
                                                            const double *__restrict__ y, double *__restrict__ slots)
{
    constexpr int K = words(A);
    const long base = (long)blockIdx.x * NT * DOT_EPT + threadIdx.x;
    Num<A> acc = zero<A>();
#pragma unroll
    for (int j = 0; j < DOT_EPT; ++j) {
        const long i = base + (long)j * NT;
        if (i < n) acc = dot_step<A>(acc, load<A>(x, n, i), load<A>(y, n, i));
    }
    const Num<A> s = block_sum<A, NT>(acc);
    if (threadIdx.x == 0) store_scalar<A>(slots + (long)blockIdx.x * K, s);
}

template <int A>
__global__ void __launch_bounds__(FIN_NT) mw_reduce_slots_kernel(int nslots, const double *__restrict__ slots,
                                                                 double *__restrict__ result)
{
    const Num<A> s = reduce_slots<A>(nslots, slots);
    if (threadIdx.x == 0) store_scalar<A>(result, s);
}

// --------------------------------------------------------------- CSR SpMV
//
// One workgroup owns NT consecutive rows (one per thread).  Its nonzeros
// [row_ptr[r0], row_ptr[r0 + NT]) are processed in chunks of CH = NT *
// CSR_NPT: thread t loads nonzeros t, t + NT, ... of the chunk (coalesced
// val/col streams, gathered x_j) and leaves the FP64 x multi-word product
// in LDS (FP64: the pair (a_ij, x_j), whose accumulation is one fma); then
// every thread adds the products of its own row that fall in the chunk, in
// CSR order, into a register accumulator that persists across chunks.
// MODE 1 (CG): x is p, kept in the gather layout (load_il) by the solver; also the
// partial of p^T q into slots[logical workgroup].
template <int A, int MODE>
__global__ void __launch_bounds__(NT) mw_csr_spmv_kernel(int n, const int32_t *__restrict__ row_ptr,
                                                         const int32_t *__restrict__ col,
                                                         const double *__restrict__ val,
                                                         const double *__restrict__ x, double *__restrict__ y,
                                                         double *__restrict__ slots, const int32_t *__restrict__ run_prev,
                                                         int32_t *__restrict__ run_cur)
{
    constexpr int K = words(A);
    constexpr int CH = NT * CSR_NPT;
    constexpr int LW = (A == FP64) ? 2 : K;
    __shared__ double lds[LW][CH];

    if constexpr (MODE == 1) {
        if (!*run_prev) {
            if (blockIdx.x == 0 && threadIdx.x == 0) *run_cur = 0;
            return;
        }
    }
    const int lb = xcd_remap(blockIdx.x, gridDim.x);
    const int r0 = lb * NT;
    const int r1 = min(r0 + NT, n);
    const int row = r0 + (int)threadIdx.x;
    const int z0 = row_ptr[r0];
    const int z1 = row_ptr[r1];
    int rs = 0, re = 0;
    if (row < n) {
        rs = row_ptr[row];
        re = row_ptr[row + 1];
    }
    Num<A> acc = zero<A>();
    for (int c0 = z0; c0 < z1; c0 += CH) {
        const int cn = min(CH, z1 - c0);
#pragma unroll
        for (int j = 0; j < CSR_NPT; ++j) {
            const int t = (int)threadIdx.x + j * NT;
            if (t < cn) {
                const double a = val[c0 + t];
                const Num<A> xj = load_v<A, MODE>(x, n, col[c0 + t]);
                if constexpr (A == FP64) {
                    lds[0][t] = a;
                    lds[1][t] = xj.w[0];
                } else {
                    const Num<A> pr = dxmul<A>(a, xj);
#pragma unroll
                    for (int w = 0; w < K; ++w) lds[w][t] = pr.w[w];
                }
            }
        }
        __syncthreads();
        const int zb = max(rs, c0), ze = min(re, c0 + cn);
        for (int z = zb; z < ze; ++z) {
            const int t = z - c0;
            if constexpr (A == FP64) {
                acc.w[0] = __builtin_fma(lds[0][t], lds[1][t], acc.w[0]);
            } else {
                Num<A> pr;
#pragma unroll
                for (int w = 0; w < K; ++w) pr.w[w] = lds[w][t];
                acc = add<A>(acc, pr);
            }
        }
        __syncthreads();
    }
    if (row < n) store<A>(y, n, row, acc);
    if constexpr (MODE == 1) {
        Num<A> c = zero<A>();
        if (row < n) c = dot_step<A>(c, load_il<A>(x, n, row), acc);
        const Num<A> sum = block_sum<A, NT>(c);
        if (threadIdx.x == 0) store_scalar<A>(slots + (long)lb * K, sum);
    }
}

// -------------------------------------------------------------- SELL SpMV
//
// Persistent workgroups of NWAVE wavefronts walk tiles of NWAVE slices
// (xcd_tiles); wavefront w of a tile takes slice 4t + w, lane l its row
// 64 s + l (entry positions: sell_row_sum).
// MODE 1 (CG): x is p, kept in the gather layout (load_il) by the solver, y is q; each
// thread accumulates p_i q_i over its rows in tile order, and the
// workgroup sum goes to slots[blockIdx.x].
template <int A, int MODE>
__global__ void __launch_bounds__(NT) mw_sell_spmv_kernel(int n, int ns, const int32_t *__restrict__ sp,
                                                          const int32_t *__restrict__ sc,
                                                          const int32_t *__restrict__ soff,
                                                          const uint64_t *__restrict__ smask,
                                                          const double *__restrict__ sv,
                                                          const double *__restrict__ x, double *__restrict__ y,
                                                          double *__restrict__ slots, const int32_t *__restrict__ run_prev,
                                                          int32_t *__restrict__ run_cur, int rev)
{
    constexpr int K = words(A);
    if constexpr (MODE == 1) {
        if (!*run_prev) {
            if (blockIdx.x == 0 && threadIdx.x == 0) *run_cur = 0;
            return;
        }
    }
    const int lane = threadIdx.x & 63, wave = wave_id();
    const TileWalk tw = xcd_walk((ns + NWAVE - 1) / NWAVE, rev);
    __shared__ double xwin[dia_window<A>() ? NWAVE * K * WIN_ROWS : 1];
    double *wv = xwin + (dia_window<A>() ? wave * K * WIN_ROWS : 0);
    Num<A> part = zero<A>();
    for (int m = 0; m < tw.count; ++m) {
        const int s = tw[m] * NWAVE + wave;
        if (s >= ns) continue;  // whole wavefront
        const int row = s * 64 + lane;
        const int b = sp[s];
        const int w = (sp[s + 1] - b) >> 6;
        Num<A> acc;
        if (slice_is_diag(b, w, smask)) {
            // x[row]: the offset-0 slot, the source of the +-1 slots and,
            // in CG mode, p_i of p^T q
            const Num<A> xc = row < n ? load_v<A, MODE>(x, n, row) : zero<A>();
            const int32_t *so = soff + (b >> 6);
            if (dia_window<A>() && w >= WIN_MIN_W && offsets_in_window(so, w)) {
                stage_window<A, MODE>(wv, lane, row, xc, x, n);
                acc = dia_row_sum<A, MODE, true>(b, w, lane, row, so, smask + (b >> 6), sv, x, n, xc, xc, wv);
            } else {
                Num<A> xe = zero<A>();
                if constexpr (neighbour_moves<A>()) {
                    const long re = lane == 0 ? (long)row - 1 : (long)row + 1;
                    if ((lane == 0 || lane == 63) && re >= 0 && re < n) xe = load_v<A, MODE>(x, n, re);
                }
                acc = dia_row_sum<A, MODE, false>(b, w, lane, row, so, smask + (b >> 6), sv, x, n, xc, xe, wv);
            }
            if (row < n) {
                store<A>(y, n, row, acc);
                if constexpr (MODE == 1) part = dot_step<A>(part, xc, acc);
            }
        } else {
            acc = sell_row_sum<A, MODE>(b, w, lane, sc, sv, x, n);
            if (row < n) {
                store<A>(y, n, row, acc);
                if constexpr (MODE == 1) part = dot_step<A>(part, load_il<A>(x, n, row), acc);
            }
        }
    }
    if constexpr (MODE == 1) {
        const Num<A> sum = block_sum<A, NT>(part);
        if (threadIdx.x == 0) store_scalar<A>(slots + (long)blockIdx.x * K, sum);
    }
}

// Vector-row SpMV (plan format MW_FMT_CSRVEC): L lanes per row, 64 / L
// rows per wavefront, NWAVE * 64 / L rows per tile of the persistent walk.
// MODE 1 (CG): x is p in the gather layout; the row group's first lane
// forms p_i q_i, and the workgroup sum of those goes to slots[blockIdx.x].
template <int A, int MODE, int L>
__global__ void __launch_bounds__(NT) mw_vec_spmv_kernel(int n, const int32_t *__restrict__ row_ptr,
                                                         const int32_t *__restrict__ col,
                                                         const double *__restrict__ val,
                                                         const double *__restrict__ x, double *__restrict__ y,
                                                         double *__restrict__ slots, const int32_t *__restrict__ run_prev,
                                                         int32_t *__restrict__ run_cur, int rev)
{
    constexpr int K = words(A);
    constexpr int RPW = 64 / L;          // rows per wavefront
    constexpr int RPT = NWAVE * RPW;     // rows per tile
    if constexpr (MODE == 1) {
        if (!*run_prev) {
            if (blockIdx.x == 0 && threadIdx.x == 0) *run_cur = 0;
            return;
        }
    }
    const int lane = threadIdx.x & 63, wave = wave_id();
    const int t = lane % L;
    const TileWalk tw = xcd_walk((n + RPT - 1) / RPT, rev);
    Num<A> part = zero<A>();
    for (int m = 0; m < tw.count; ++m) {
        const long row = (long)tw[m] * RPT + wave * RPW + lane / L;
        Num<A> acc = zero<A>();
        if (row < n) {
            const int re = row_ptr[row + 1];
            int j = row_ptr[row] + t;
            // U entries' loads in flight per lane before their products are
            // added in order (the same association as one at a time): on
            // MI355X 5-16 % faster CG iterations on long rows; four cost the
            // 3- and 4-word types more in registers than they gain
            constexpr int U = words(A) >= 3 ? 2 : 4;
            for (; j + (U - 1) * L < re; j += U * L) {
                double a[U];
                int c[U];
                Num<A> xv[U];
#pragma unroll
                for (int u = 0; u < U; ++u) {
                    a[u] = val[j + u * L];
                    c[u] = col[j + u * L];
                }
#pragma unroll
                for (int u = 0; u < U; ++u) xv[u] = load_v<A, MODE>(x, n, c[u]);
#pragma unroll
                for (int u = 0; u < U; ++u) acc = row_step<A>(acc, a[u], xv[u]);
            }
            for (; j < re; j += L) acc = row_step<A>(acc, val[j], load_v<A, MODE>(x, n, col[j]));
        }
        // fixed halving tree inside the row's group of L lanes (the whole
        // wavefront takes part in every shuffle)
#pragma unroll
        for (int d = L / 2; d > 0; d >>= 1) {
            const Num<A> o = shfl_down<A>(acc, d);
            if (t < d) acc = add<A>(acc, o);
        }
        if (t == 0 && row < n) {
            store<A>(y, n, row, acc);
            if constexpr (MODE == 1) part = dot_step<A>(part, load_v<A, MODE>(x, n, row), acc);
        }
    }
    if constexpr (MODE == 1) {
        const Num<A> sum = block_sum<A, NT>(part);
        if (threadIdx.x == 0) store_scalar<A>(slots + (long)blockIdx.x * K, sum);
    }
}

// ------------------------------------------------- gradient on a pattern
//
// grad_val[k] = -(lam_i * x_j) for the k-th stored entry (i, j): the
// derivative of a loss with respect to A_ij when x = A^-1 b and lam solves
// A^T lam = dL/dx.  The product is formed in the arithmetic and rounded
// to FP64 (FP64: -(lam_i * x_j), one rounding).  One wavefront per block
// of 64 rows: the block's entries are contiguous in the CSR arrays, so the
// lanes walk them 64 at a time (coalesced column loads and gradient
// stores); a lane finds its entry's row by a binary search over the
// block's row starts, which the lanes hold one each.
template <int A>
__global__ void __launch_bounds__(NT) mw_csr_grad_kernel(int n, const int32_t *__restrict__ row_ptr,
                                                         const int32_t *__restrict__ col,
                                                         const double *__restrict__ lam,
                                                         const double *__restrict__ x, double *__restrict__ grad)
{
    // XCD x takes the x-th contiguous range of row blocks, so the gathers
    // of x for a block's neighbours hit that XCD's L2
    const long r0 = ((long)xcd_remap(blockIdx.x, gridDim.x) * NWAVE + wave_id()) * 64;
    if (r0 >= n) return;
    const int lane = threadIdx.x & 63;
    // row starts of the block; lanes past the last row hold a start no
    // entry index reaches
    const int start = r0 + lane < n ? row_ptr[r0 + lane] : 0x7fffffff;
    // lam of the block's rows, one per lane (coalesced), passed to the
    // entries' lanes by shuffles
    const Num<A> lrow = r0 + lane < n ? load<A>(lam, n, r0 + lane) : zero<A>();
    const int e0 = row_ptr[r0];
    const int e1 = row_ptr[r0 + 64 < n ? r0 + 64 : n];
    // two 64-entry chunks per pass: their searches and loads are independent
    for (int z0 = e0; z0 < e1; z0 += 128) {
        const int za = z0 + lane, zb = z0 + 64 + lane;
        // the last row whose start is <= z (a row with entries: an empty
        // row's start equals the next row's); all lanes take part
        int la = 0, lb = 0;
#pragma unroll
        for (int step = 32; step > 0; step >>= 1) {
            if (__shfl(start, la + step, 64) <= za) la += step;
            if (__shfl(start, lb + step, 64) <= zb) lb += step;
        }
        Num<A> lia, lib;
#pragma unroll
        for (int w = 0; w < words(A); ++w) {
            lia.w[w] = __shfl(lrow.w[w], la, 64);
            lib.w[w] = __shfl(lrow.w[w], lb, 64);
        }
        if (za < e1) grad[za] = -to_fp64<A>(mul<A>(lia, load<A>(x, n, col[za])));
        if (zb < e1) grad[zb] = -to_fp64<A>(mul<A>(lib, load<A>(x, n, col[zb])));
    }
}

// ------------------------------------------------------------- CSR check
//
// Flags (pinned host memory, written by the device): [0] row_ptr[0] != 0 or
// row_ptr[n] != nnz, [1] row_ptr decreases somewhere, [2] a column index
// outside [0, n).  Reads row_ptr[0 .. n] and col[0 .. nnz) only, so it is
// safe on any arrays of those lengths, whatever they hold.
__global__ void __launch_bounds__(NT) mw_csr_check_kernel(int n, int nnz, const int32_t *__restrict__ row_ptr,
                                                          const int32_t *__restrict__ col, int32_t *flags)
{
    const long tid = (long)blockIdx.x * NT + threadIdx.x, stride = (long)gridDim.x * NT;
    if (tid == 0 && (row_ptr[0] != 0 || row_ptr[n] != nnz)) flags[0] = 1;
    bool dec = false, out = false;
    for (long i = tid; i < n; i += stride) dec = dec || row_ptr[i + 1] < row_ptr[i];
    for (long j = tid; j < nnz; j += stride) {
        const int c = col[j];
        out = out || c < 0 || c >= n;
    }
    if (dec) flags[1] = 1;
    if (out) flags[2] = 1;
}

// ------------------------------------------------------ Jacobi reciprocal
//
// d_i = fl(1 / a_ii) from the CSR rows (the last stored entry in column i;
// none: 1 / 0 = inf, which ends a preconditioned solve with a breakdown).
__global__ void __launch_bounds__(NT) mw_jacobi_dinv_kernel(int n, const int32_t *__restrict__ row_ptr,
                                                            const int32_t *__restrict__ col,
                                                            const double *__restrict__ val, double *__restrict__ dinv)
{
    const long i = (long)blockIdx.x * NT + threadIdx.x;
    if (i >= n) return;
    double aii = 0.0;
    for (int j = row_ptr[i]; j < row_ptr[i + 1]; ++j)
        if (col[j] == i) aii = val[j];
    dinv[i] = 1.0 / aii;
}

// -------------------------------------------------------------- SELL plan

// Width (longest row) of every 64-row slice: one wavefront per slice.
__global__ void __launch_bounds__(NT) mw_sell_width_kernel(int n, int ns, const int32_t *__restrict__ row_ptr,
                                                           int32_t *__restrict__ width)
{
    const int s = blockIdx.x * NWAVE + wave_id();
    const int lane = threadIdx.x & 63;
    if (s >= ns) return;
    const int row = s * 64 + lane;
    int len = row < n ? row_ptr[row + 1] - row_ptr[row] : 0;
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) len = max(len, __shfl_xor(len, off, 64));
    if (lane == 0) width[s] = len;
}

// Exclusive scan of 64 * width into slice_ptr (one workgroup of FIN_NT
// threads, each owning a contiguous range of slices).  The 64-bit total is
// written to *total; slice_ptr is meaningful only if the total fits int32.
__global__ void __launch_bounds__(FIN_NT) mw_sell_scan_kernel(int ns, const int32_t *__restrict__ width,
                                                              int32_t *__restrict__ slice_ptr,
                                                              long long *__restrict__ total)
{
    __shared__ long long sums[FIN_NT];
    const int t = threadIdx.x;
    const int per = (ns + FIN_NT - 1) / FIN_NT;
    const int lo = min(t * per, ns), hi = min(lo + per, ns);
    long long s = 0;
    // unrolled so that the loads of a thread's contiguous range are issued
    // together, not one round trip after another
#pragma unroll 16
    for (int i = lo; i < hi; ++i) s += 64LL * width[i];
    sums[t] = s;
    __syncthreads();
    // Hillis-Steele inclusive scan over the FIN_NT thread sums
    for (int off = 1; off < FIN_NT; off <<= 1) {
        const long long v = (t >= off) ? sums[t - off] : 0;
        __syncthreads();
        sums[t] += v;
        __syncthreads();
    }
    long long run = sums[t] - s;
#pragma unroll 16
    for (int i = lo; i < hi; ++i) {
        slice_ptr[i] = (int32_t)run;
        run += 64LL * width[i];
    }
    if (t == FIN_NT - 1) {
        slice_ptr[ns] = (int32_t)sums[t];
        *total = sums[t];
    }
}

// Scatter the CSR rows into the slices (fill_slice); counts the slices
// stored as diagonal slots.
__global__ void __launch_bounds__(NT) mw_sell_fill_kernel(int n, int ns, const int32_t *__restrict__ row_ptr,
                                                          const int32_t *__restrict__ col,
                                                          const double *__restrict__ val,
                                                          const int32_t *__restrict__ slice_ptr,
                                                          int32_t *__restrict__ scol, double *__restrict__ sval,
                                                          int32_t *__restrict__ soff, uint64_t *__restrict__ smask,
                                                          int32_t *__restrict__ is_diag)
{
    const int s = blockIdx.x * NWAVE + wave_id();
    const int lane = threadIdx.x & 63;
    if (s >= ns) return;
    const int row = s * 64 + lane;
    const int b = slice_ptr[s];
    const int w = (slice_ptr[s + 1] - b) / 64;
    const int rs = row < n ? row_ptr[row] : 0;
    const int len = row < n ? row_ptr[row + 1] - rs : 0;
    const bool diag = fill_slice(b, w, lane, row, rs, len, col, val, scol, sval, soff, smask);
    if (lane == 0) is_diag[s] = diag ? 1 : 0;
}

// *out = number of non-zero flags[0 .. ns) (one workgroup of FIN_NT
// threads; a single counter bumped by every slice serialises on it).
__global__ void __launch_bounds__(FIN_NT) mw_flag_count_kernel(int ns, const int32_t *__restrict__ flags,
                                                               int32_t *__restrict__ out)
{
    __shared__ int part[FIN_NT / 64];
    int c = 0;
    for (int i = threadIdx.x; i < ns; i += FIN_NT) c += flags[i] != 0;
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) c += __shfl_xor(c, off, 64);
    if ((threadIdx.x & 63) == 0) part[threadIdx.x >> 6] = c;
    __syncthreads();
    if (threadIdx.x == 0) {
        int t = 0;
        for (int w = 0; w < FIN_NT / 64; ++w) t += part[w];
        *out = t;
    }
}

// Plan buffer: slice_ptr, the width scratch, the 64-bit total and the
// diagonal-slice count, then per 64-entry slot the offset and lane mask,
// then columns and values.
struct PlanLayout {
    size_t slice_ptr, width, total, ndiag, soff, smask, col, val, bytes;
    long long cap;  // entries the buffer can hold
};

PlanLayout plan_layout(int32_t n, int32_t nnz)
{
    const long long ns = (n + 63) / 64;
    PlanLayout L;
    L.cap = (long long)nnz + (long long)nnz / 4 + 64 * ns;
    const long long slots = L.cap / 64 + 1;
    L.slice_ptr = 0;
    L.width = align256(sizeof(int32_t) * (ns + 1));
    L.total = L.width + align256(sizeof(int32_t) * ns);
    L.ndiag = L.total + 8;
    L.soff = L.total + 256;
    L.smask = L.soff + align256(sizeof(int32_t) * slots);
    L.col = L.smask + align256(sizeof(uint64_t) * slots);
    L.val = L.col + align256(sizeof(int32_t) * L.cap);
    L.bytes = L.val + align256(sizeof(double) * L.cap);
    return L;
}

long long *pinned_total()
{
    thread_local long long *buf = nullptr;
    if (!buf && hipHostMalloc((void **)&buf, 64, hipHostMallocDefault) != hipSuccess) buf = nullptr;
    return buf;
}

}  // namespace

// ============================================================ internal API

namespace mwh {

int launch_sell_scan(int ns, const int32_t *width, int32_t *slice_ptr, long long *total, hipStream_t s)
{
    hipLaunchKernelGGL(mw_sell_scan_kernel, dim3(1), dim3(FIN_NT), 0, s, ns, width, slice_ptr, total);
    HIP_TRY(hipGetLastError());
    return MW_OK;
}

template <int A, int L>
void rc_launch_vec(const mw_csr_t *M, const double *x, double *y, double *slots, const int32_t *run_prev,
                   int32_t *run_cur, int mode, hipStream_t s, int rev, hipEvent_t ev0, hipEvent_t ev1, int g)
{
    if (mode == 0)
        MW_LAUNCH((mw_vec_spmv_kernel<A, 0, L>), dim3(g), dim3(NT), s, ev0, ev1, M->n, M->row_ptr, M->col_idx,
                  M->val, x, y, slots, run_prev, run_cur, rev);
    else
        MW_LAUNCH((mw_vec_spmv_kernel<A, 1, L>), dim3(g), dim3(NT), s, ev0, ev1, M->n, M->row_ptr, M->col_idx,
                  M->val, x, y, slots, run_prev, run_cur, rev);
}

int spmv_tiles(const mw_spmv_plan_t *plan)
{
    if (plan->format == MW_FMT_CSRVEC) {
        const long rpt = (long)NWAVE * (64 / plan->lanes);
        return (int)((plan->n + rpt - 1) / rpt);
    }
    return blocks_for(plan->nslices, NWAVE);
}

int plan_rows(const mw_csr_t *A, int lanes, mw_spmv_plan_t *plan)
{
    if (lanes == 0) {
        // about eight entries per lane for the average row
        const double avg = A->n > 0 ? (double)A->nnz / A->n : 0.0;
        lanes = 2;
        while (lanes < 64 && lanes * 8 < avg) lanes *= 2;
    }
    if (lanes != 2 && lanes != 4 && lanes != 8 && lanes != 16 && lanes != 32 && lanes != 64) return MW_EINVAL;
    memset(plan, 0, sizeof(*plan));
    plan->n = A->n;
    plan->nnz = A->nnz;
    plan->format = MW_FMT_CSRVEC;
    plan->nslices = (A->n + 63) / 64;
    plan->lanes = lanes;
    plan->csr = *A;
    return MW_OK;
}

bool plan_valid(const mw_spmv_plan_t *plan)
{
    if (!plan || !valid_csr(&plan->csr) || plan->n != plan->csr.n) return false;
    const int L = plan->lanes;
    switch (plan->format) {
    case MW_FMT_CSR: return true;
    case MW_FMT_SELL64: return plan->slice_ptr && plan->col && plan->val && plan->nslices == (plan->n + 63) / 64;
    case MW_FMT_CSRVEC: return L >= 2 && L <= 64 && (L & (L - 1)) == 0;
    default: return false;
    }
}

// Measured on MI355X (SpMV alone, SELL-64 against vector rows of 2 .. 64
// lanes): SELL-64 is faster for n >= 1M whatever the row length (16K or
// more slices fill the GPU), vector rows for n <= 83K with 73 .. 400
// entries per row (2 .. 7x) and for irregular rows whose SELL padding
// forces the CSR fallback (6 .. 20x at 25 .. 280 entries per row).  The
// best lanes per row: about 8 entries per lane in FP64, 16 in the
// multi-word arithmetics (within 15 % of the best of 2 .. 64).
bool rows_by_size(int n, int nnz) { return n <= (1 << 18) && (long)nnz >= 32L * n; }

int rows_lanes(int a, int n, int nnz, int lanes)
{
    if (lanes > 0) return lanes;
    const double avg = n > 0 ? (double)nnz / n : 0.0;
    const int per = words(a) == 1 ? 8 : 16;
    int L = 2;
    while (L < 64 && L * per < avg) L *= 2;
    return L;
}

int plan_auto(int a, const mw_csr_t *A, int lanes, void *buffer, size_t bytes, mw_spmv_plan_t *plan, hipStream_t s)
{
    if (rows_by_size(A->n, A->nnz)) return plan_rows(A, rows_lanes(a, A->n, A->nnz, lanes), plan);
    const int rc = plan_build(A, buffer, bytes, plan, s);
    if (rc == MW_OK && plan->format == MW_FMT_CSR && (long)A->nnz >= 16L * A->n)
        return plan_rows(A, rows_lanes(a, A->n, A->nnz, lanes), plan);
    return rc;
}

int csr_check(const mw_csr_t *A, hipStream_t s)
{
    if (!valid_csr(A)) return MW_EINVAL;
    thread_local int32_t *flags = nullptr;
    if (!flags && hipHostMalloc((void **)&flags, 64, hipHostMallocCoherent) != hipSuccess) flags = nullptr;
    if (!flags) return hip_fail(hipErrorOutOfMemory, "hipHostMalloc");
    int32_t *dflags = nullptr;
    HIP_TRY(hipHostGetDevicePointer((void **)&dflags, flags, 0));
    flags[0] = flags[1] = flags[2] = 0;
    const long work = A->n > A->nnz ? A->n : A->nnz;
    const int g = blocks_for(work, NT) < 1024 ? blocks_for(work, NT) : 1024;
    hipLaunchKernelGGL(mw_csr_check_kernel, dim3(g > 0 ? g : 1), dim3(NT), 0, s, A->n, A->nnz, A->row_ptr, A->col_idx,
                       dflags);
    HIP_TRY(hipGetLastError());
    HIP_TRY(hipStreamSynchronize(s));
    if (flags[0]) set_error("CSR check: row_ptr[0] is not 0 or row_ptr[n] is not nnz");
    else if (flags[1]) set_error("CSR check: row_ptr decreases");
    else if (flags[2]) set_error("CSR check: a column index is outside [0, n)");
    return flags[0] || flags[1] || flags[2] ? MW_EINVAL : MW_OK;
}

bool csr_check_on()
{
    static const bool on = [] {
        const char *e = getenv("MW_CHECK_CSR");
        return e && atoi(e) != 0;
    }();
    return on;
}

void launch_jacobi_dinv(const mw_csr_t *A, double *dinv, hipStream_t s)
{
    hipLaunchKernelGGL(mw_jacobi_dinv_kernel, dim3(blocks_for(A->n, NT)), dim3(NT), 0, s, A->n, A->row_ptr,
                       A->col_idx, A->val, dinv);
}

int spmv_max_slots(int32_t n)
{
    const int csr = blocks_for(n, NT);
    return csr > MAX_GRID ? csr : MAX_GRID;
}

template <int A>
int spmv_launch(const mw_csr_t *M, const mw_spmv_plan_t *plan, const double *x, double *y, double *slots,
                const int32_t *run_prev, int32_t *run_cur, int mode, hipStream_t s, int *nslots, int rev,
                hipEvent_t ev0, hipEvent_t ev1, int grid)
{
    if (plan && plan->format == MW_FMT_CSRVEC) {
        const int g = grid > 0 ? grid : cg_shape(A, M->n, M->nnz, spmv_tiles(plan), nullptr, 0).sgrid;
        switch (plan->lanes) {
        case 2: rc_launch_vec<A, 2>(M, x, y, slots, run_prev, run_cur, mode, s, rev, ev0, ev1, g); break;
        case 4: rc_launch_vec<A, 4>(M, x, y, slots, run_prev, run_cur, mode, s, rev, ev0, ev1, g); break;
        case 8: rc_launch_vec<A, 8>(M, x, y, slots, run_prev, run_cur, mode, s, rev, ev0, ev1, g); break;
        case 16: rc_launch_vec<A, 16>(M, x, y, slots, run_prev, run_cur, mode, s, rev, ev0, ev1, g); break;
        case 32: rc_launch_vec<A, 32>(M, x, y, slots, run_prev, run_cur, mode, s, rev, ev0, ev1, g); break;
        default: rc_launch_vec<A, 64>(M, x, y, slots, run_prev, run_cur, mode, s, rev, ev0, ev1, g); break;
        }
        if (nslots) *nslots = g;
    } else if (plan && plan->format == MW_FMT_SELL64) {
        const int ns = plan->nslices;
        const int g = grid > 0 ? grid : cg_shape(A, M->n, M->nnz, spmv_tiles(plan), nullptr, 0).sgrid;
        if (mode == 0)
            MW_LAUNCH((mw_sell_spmv_kernel<A, 0>), dim3(g), dim3(NT), s, ev0, ev1, M->n, ns, plan->slice_ptr,
                      plan->col, plan->slot_off, plan->slot_mask, plan->val, x, y, slots, run_prev, run_cur, rev);
        else
            MW_LAUNCH((mw_sell_spmv_kernel<A, 1>), dim3(g), dim3(NT), s, ev0, ev1, M->n, ns, plan->slice_ptr,
                      plan->col, plan->slot_off, plan->slot_mask, plan->val, x, y, slots, run_prev, run_cur, rev);
        if (nslots) *nslots = g;
    } else {
        const int nb = blocks_for(M->n, NT);
        if (mode == 0)
            MW_LAUNCH((mw_csr_spmv_kernel<A, 0>), dim3(nb), dim3(NT), s, ev0, ev1, M->n, M->row_ptr, M->col_idx,
                      M->val, x, y, slots, run_prev, run_cur);
        else
            MW_LAUNCH((mw_csr_spmv_kernel<A, 1>), dim3(nb), dim3(NT), s, ev0, ev1, M->n, M->row_ptr, M->col_idx,
                      M->val, x, y, slots, run_prev, run_cur);
        if (nslots) *nslots = nb;
    }
    HIP_TRY(hipGetLastError());
    return MW_OK;
}

template int spmv_launch<FP64>(const mw_csr_t *, const mw_spmv_plan_t *, const double *, double *, double *,
                               const int32_t *, int32_t *, int, hipStream_t, int *, int, hipEvent_t, hipEvent_t, int);
template int spmv_launch<DW>(const mw_csr_t *, const mw_spmv_plan_t *, const double *, double *, double *,
                             const int32_t *, int32_t *, int, hipStream_t, int *, int, hipEvent_t, hipEvent_t, int);
template int spmv_launch<QDW>(const mw_csr_t *, const mw_spmv_plan_t *, const double *, double *, double *,
                              const int32_t *, int32_t *, int, hipStream_t, int *, int, hipEvent_t, hipEvent_t, int);
template int spmv_launch<TW>(const mw_csr_t *, const mw_spmv_plan_t *, const double *, double *, double *,
                             const int32_t *, int32_t *, int, hipStream_t, int *, int, hipEvent_t, hipEvent_t, int);
template int spmv_launch<QTW>(const mw_csr_t *, const mw_spmv_plan_t *, const double *, double *, double *,
                              const int32_t *, int32_t *, int, hipStream_t, int *, int, hipEvent_t, hipEvent_t, int);
template int spmv_launch<QTWE>(const mw_csr_t *, const mw_spmv_plan_t *, const double *, double *, double *,
                               const int32_t *, int32_t *, int, hipStream_t, int *, int, hipEvent_t, hipEvent_t, int);
template int spmv_launch<QW>(const mw_csr_t *, const mw_spmv_plan_t *, const double *, double *, double *,
                             const int32_t *, int32_t *, int, hipStream_t, int *, int, hipEvent_t, hipEvent_t, int);
template int spmv_launch<QQW>(const mw_csr_t *, const mw_spmv_plan_t *, const double *, double *, double *,
                              const int32_t *, int32_t *, int, hipStream_t, int *, int, hipEvent_t, hipEvent_t, int);
template int spmv_launch<MXDW>(const mw_csr_t *, const mw_spmv_plan_t *, const double *, double *, double *,
                               const int32_t *, int32_t *, int, hipStream_t, int *, int, hipEvent_t, hipEvent_t, int);
template int spmv_launch<MXQTW>(const mw_csr_t *, const mw_spmv_plan_t *, const double *, double *, double *,
                                const int32_t *, int32_t *, int, hipStream_t, int *, int, hipEvent_t, hipEvent_t, int);

size_t plan_bytes(int32_t n, int32_t nnz) { return plan_layout(n, nnz).bytes; }

int plan_build(const mw_csr_t *A, void *buffer, size_t bytes, mw_spmv_plan_t *plan, hipStream_t s)
{
    const int n = A->n;
    const int ns = (n + 63) / 64;
    const PlanLayout L = plan_layout(n, A->nnz);
    if (bytes < L.bytes) return MW_EINVAL;
    char *base = (char *)buffer;
    int32_t *sp = (int32_t *)(base + L.slice_ptr);
    int32_t *width = (int32_t *)(base + L.width);
    long long *total = (long long *)(base + L.total);
    int32_t *ndiag = (int32_t *)(base + L.ndiag);
    int32_t *soff = (int32_t *)(base + L.soff);
    uint64_t *smask = (uint64_t *)(base + L.smask);
    int32_t *scol = (int32_t *)(base + L.col);
    double *sval = (double *)(base + L.val);
    long long *htot = pinned_total();
    if (!htot) return hip_fail(hipErrorOutOfMemory, "hipHostMalloc");

    memset(plan, 0, sizeof(*plan));
    plan->n = n;
    plan->nnz = A->nnz;
    plan->nslices = ns;
    plan->csr = *A;
    plan->format = MW_FMT_CSR;

    const int nbw = blocks_for(ns, NWAVE);
    hipLaunchKernelGGL(mw_sell_width_kernel, dim3(nbw), dim3(NT), 0, s, n, ns, A->row_ptr, width);
    hipLaunchKernelGGL(mw_sell_scan_kernel, dim3(1), dim3(FIN_NT), 0, s, ns, width, sp, total);
    HIP_TRY(hipGetLastError());
    HIP_TRY(hipMemcpyAsync(htot, total, sizeof(long long), hipMemcpyDeviceToHost, s));
    HIP_TRY(hipStreamSynchronize(s));
    const long long stored = htot[0];
    if (stored > L.cap || stored > 0x7fffffffLL) return MW_OK;  // CSR fallback
    // the width scratch, read by the scan only, takes the per-slice flags
    hipLaunchKernelGGL(mw_sell_fill_kernel, dim3(nbw), dim3(NT), 0, s, n, ns, A->row_ptr, A->col_idx, A->val, sp,
                       scol, sval, soff, smask, width);
    hipLaunchKernelGGL(mw_flag_count_kernel, dim3(1), dim3(FIN_NT), 0, s, ns, width, ndiag);
    HIP_TRY(hipGetLastError());
    HIP_TRY(hipMemcpyAsync(htot + 1, ndiag, sizeof(int32_t), hipMemcpyDeviceToHost, s));
    HIP_TRY(hipStreamSynchronize(s));
    plan->format = MW_FMT_SELL64;
    plan->stored = stored;
    plan->slice_ptr = sp;
    plan->col = scol;
    plan->val = sval;
    plan->slot_off = soff;
    plan->slot_mask = smask;
    plan->ndiag = (int32_t)htot[1];
    return MW_OK;
}

}  // namespace mwh

namespace {

template <int A, int OP>
int launch_elementwise(int32_t n, const double *u, const double *v, double *w, hipStream_t s)
{
    hipLaunchKernelGGL((mw_elementwise_kernel<A, OP>), dim3(blocks_for(n, NT)), dim3(NT), 0, s, n, u, v, w);
    HIP_TRY(hipGetLastError());
    return MW_OK;
}

template <int A>
int elementwise_a(int op, int32_t n, const double *u, const double *v, double *w, hipStream_t s)
{
    switch (op) {
    case MW_OP_ADD: return launch_elementwise<A, MW_OP_ADD>(n, u, v, w, s);
    case MW_OP_MUL: return launch_elementwise<A, MW_OP_MUL>(n, u, v, w, s);
    case MW_OP_DXMUL: return launch_elementwise<A, MW_OP_DXMUL>(n, u, v, w, s);
    case MW_OP_DIV: return launch_elementwise<A, MW_OP_DIV>(n, u, v, w, s);
    case MW_OP_NORM: return launch_elementwise<A, MW_OP_NORM>(n, u, v, w, s);
    case MW_OP_NEG: return launch_elementwise<A, MW_OP_NEG>(n, u, v, w, s);
    default: return launch_elementwise<A, MW_OP_TOFP64>(n, u, v, w, s);
    }
}

template <int A>
int axpy_a(int32_t n, const double *alpha, const double *x, double *y, hipStream_t s)
{
    hipLaunchKernelGGL((mw_axpy_kernel<A>), dim3(blocks_for(n, NT)), dim3(NT), 0, s, n, alpha, x, y);
    HIP_TRY(hipGetLastError());
    return MW_OK;
}

template <int A>
int dot_a(int32_t n, const double *x, const double *y, double *res, void *ws, hipStream_t s)
{
    const int nb = n > 0 ? blocks_for(n, (long)NT * DOT_EPT) : 0;
    double *slots = (double *)ws;
    if (nb > 0) {
        hipLaunchKernelGGL((mw_dot_partial_kernel<A>), dim3(nb), dim3(NT), 0, s, n, x, y, slots);
        HIP_TRY(hipGetLastError());
    }
    hipLaunchKernelGGL((mw_reduce_slots_kernel<A>), dim3(1), dim3(FIN_NT), 0, s, nb, slots, res);
    HIP_TRY(hipGetLastError());
    return MW_OK;
}

// ------------------------------------------- dot without a workspace
//
// mw_dot_noalloc keeps the per-workgroup partial sums in `scratch`, a
// file-scope device array that every GPU the library runs on holds until
// the process ends.  On the host `scratch` is only a stand-in for the
// symbol, not a device address: the address is looked up once per device
// (hipGetSymbolAddress, with that device current) and that pointer is what
// the kernels receive.  Every slot the reduction reads is written by the
// partial kernel of the same call, so nothing needs clearing between calls;
// calls that overlap on one GPU share the array and race.
constexpr int NOALLOC_SLOTS = MW_DOT_NOALLOC_MAX_N / (NT * DOT_EPT);
static_assert((long)NOALLOC_SLOTS * NT * DOT_EPT == MW_DOT_NOALLOC_MAX_N, "whole workgroups");
constexpr int MAX_DEVICES = 64;

static __device__ __align__(256) double scratch[4 * NOALLOC_SLOTS];

std::mutex g_scratch_mu;
double *g_scratch_ptr[MAX_DEVICES] = {};

// The current device's copy of `scratch`.
int scratch_slots(double **out)
{
    int dev = -1;
    HIP_TRY(hipGetDevice(&dev));
    if (dev < 0 || dev >= MAX_DEVICES) {
        set_error("mw_dot_noalloc: device ordinal beyond the 64 this library keeps scratch addresses for");
        return MW_EINVAL;
    }
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void *p = nullptr;
        HIP_TRY(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
        if (!p) {
            set_error("mw_dot_noalloc: hipGetSymbolAddress returned a null address for the scratch array");
            return MW_EHIP;
        }
        g_scratch_ptr[dev] = (double *)p;
    }
    *out = g_scratch_ptr[dev];
    return MW_OK;
}

template <int A>
int grad_a(const mw_csr_t *M, const double *lam, const double *x, double *grad, hipStream_t s)
{
    hipLaunchKernelGGL((mw_csr_grad_kernel<A>), dim3(blocks_for(blocks_for(M->n, 64), NWAVE)), dim3(NT), 0, s, M->n,
                       M->row_ptr, M->col_idx, lam, x, grad);
    HIP_TRY(hipGetLastError());
    return MW_OK;
}

template <int A>
int spmv_csr_a(const mw_csr_t *M, const double *x, double *y, hipStream_t s)
{
    return mwh::spmv_launch<A>(M, nullptr, x, y, nullptr, nullptr, nullptr, 0, s);
}

template <int A>
int spmv_planned_a(const mw_spmv_plan_t *P, const double *x, double *y, hipStream_t s)
{
    return mwh::spmv_launch<A>(&P->csr, P, x, y, nullptr, nullptr, nullptr, 0, s);
}

}  // namespace

// ================================================================== C ABI

extern "C" {

int mw_words(mw_arith_t a) { return mwh::valid_arith(a) ? vwords(a) : -1; }

int mw_scalar_words(mw_arith_t a) { return mwh::valid_arith(a) ? words(a) : -1; }

const char *mw_status_string(int code)
{
    switch (code) {
    case MW_OK: return "ok";
    case MW_NOT_CONVERGED: return "not converged (maxit reached)";
    case MW_BREAKDOWN: return "breakdown (p^T A p <= 0 or non-finite scalar)";
    case MW_EINVAL: return "invalid argument";
    case MW_EHIP: return "HIP runtime error";
    default: return "unknown status";
    }
}

const char *mw_last_error(void) { return mwh::g_err; }

int mw_elementwise(mw_arith_t a, int op, int32_t n, const double *u, const double *v, double *w, void *stream)
{
    mwh::clear_error();
    if (!valid_arith(a) || mixed_arith(a) || op < MW_OP_ADD || op > MW_OP_TOFP64 || !size_ok(n) || (n > 0 && (!u || !w)))
        return MW_EINVAL;
    const bool needs_v = (op == MW_OP_ADD || op == MW_OP_MUL || op == MW_OP_DXMUL || op == MW_OP_DIV);
    if (needs_v && n > 0 && !v) return MW_EINVAL;
    if (n == 0) return MW_OK;
    hipStream_t s = (hipStream_t)stream;
    MW_DISPATCH_WORDS(a, elementwise_a, op, n, u, v, w, s);
}

int mw_axpy(mw_arith_t a, int32_t n, const double *alpha, const double *x, double *y, void *stream)
{
    mwh::clear_error();
    if (!valid_arith(a) || !size_ok(n) || (n > 0 && (!alpha || !x || !y))) return MW_EINVAL;
    if (n == 0) return MW_OK;
    hipStream_t s = (hipStream_t)stream;
    MW_DISPATCH(a, axpy_a, n, alpha, x, y, s);
}

size_t mw_dot_workspace_bytes(mw_arith_t a, int32_t n)
{
    if (!valid_arith(a) || !size_ok(n)) return 0;
    const size_t nb = (size_t)(n > 0 ? blocks_for(n, (long)NT * DOT_EPT) : 0);
    return align256(sizeof(double) * words(a) * (nb > 0 ? nb : 1));
}

int mw_dot(mw_arith_t a, int32_t n, const double *x, const double *y, double *result, void *workspace,
           void *stream)
{
    mwh::clear_error();
    if (!valid_arith(a) || !size_ok(n) || !result || !workspace || (n > 0 && (!x || !y))) return MW_EINVAL;
    hipStream_t s = (hipStream_t)stream;
    MW_DISPATCH(a, dot_a, n, x, y, result, workspace, s);
}

int mw_dot_noalloc(mw_arith_t a, int32_t n, const double *x, const double *y, double *result, void *stream)
{
    mwh::clear_error();
    if (!valid_arith(a) || n < 0 || !result || (n > 0 && (!x || !y))) return MW_EINVAL;
    if (n > MW_DOT_NOALLOC_MAX_N) {
        set_error("mw_dot_noalloc: n exceeds MW_DOT_NOALLOC_MAX_N (33554432); use mw_dot with a workspace");
        return MW_EINVAL;
    }
    double *slots = nullptr;
    const int rc = scratch_slots(&slots);
    if (rc != MW_OK) return rc;
    hipStream_t s = (hipStream_t)stream;
    MW_DISPATCH(a, dot_a, n, x, y, result, slots, s);
}

int mw_spmv(mw_arith_t a, const mw_csr_t *A, const double *x, double *y, void *stream)
{
    mwh::clear_error();
    if (!valid_arith(a) || !valid_csr(A) || !x || !y || x == y) return MW_EINVAL;
    MW_CSR_GUARD(A, stream);
    hipStream_t s = (hipStream_t)stream;
    MW_DISPATCH(a, spmv_csr_a, A, x, y, s);
}

int mw_csr_check(const mw_csr_t *A, void *stream)
{
    mwh::clear_error();
    return mwh::csr_check(A, (hipStream_t)stream);
}

int mw_csr_grad(mw_arith_t a, const mw_csr_t *A, const double *lam, const double *x, double *grad_val,
                void *stream)
{
    mwh::clear_error();
    if (!valid_arith(a) || mixed_arith(a) || !valid_csr(A) || !lam || !x || !grad_val) return MW_EINVAL;
    MW_CSR_GUARD(A, stream);
    hipStream_t s = (hipStream_t)stream;
    MW_DISPATCH_WORDS(a, grad_a, A, lam, x, grad_val, s);
}

size_t mw_spmv_plan_bytes(int32_t n, int32_t nnz)
{
    if (n <= 0 || !size_ok(n) || !size_ok(nnz)) return 0;
    return mwh::plan_bytes(n, nnz);
}

int mw_spmv_plan(const mw_csr_t *A, void *buffer, size_t bytes, mw_spmv_plan_t *plan, void *stream)
{
    mwh::clear_error();
    if (!valid_csr(A) || !buffer || !plan) return MW_EINVAL;
    MW_CSR_GUARD(A, stream);
    return mwh::plan_build(A, buffer, bytes, plan, (hipStream_t)stream);
}

int mw_spmv_plan_rows(const mw_csr_t *A, int32_t lanes, mw_spmv_plan_t *plan)
{
    mwh::clear_error();
    if (!valid_csr(A) || !plan) return MW_EINVAL;
    return mwh::plan_rows(A, lanes, plan);
}

int mw_spmv_planned(mw_arith_t a, const mw_spmv_plan_t *plan, const double *x, double *y, void *stream)
{
    mwh::clear_error();
    if (!valid_arith(a) || !plan_valid(plan) || !x || !y || x == y) return MW_EINVAL;
    MW_CSR_GUARD(&plan->csr, stream);
    hipStream_t s = (hipStream_t)stream;
    MW_DISPATCH(a, spmv_planned_a, plan, x, y, s);
}

}  // extern "C"
