// mw_kernels.hip -- gfx950 kernels, CG driver and C ABI of libmwcg.
//
// Method: Mukunoki & Ozaki, arXiv 2510.13536 (Alg. 1, Sec. III, Sec. IV).
// Declarations and argument contracts: include/mw.h.
//
// Kernel map (wave64, 256-thread workgroups, no MFMA: this is memory-bound
// FP64 vector work):
//   mw_spmv_kernel       CSR SpMV, one row per thread.  The workgroup's
//                        nonzeros are streamed through LDS in coalesced
//                        chunks: every thread forms FP64 x multi-word
//                        products of consecutive nonzeros, then each row's
//                        thread adds its own products in CSR order, which
//                        keeps every row bit-identical to the sequential
//                        definition.  In CG mode it also forms p_i * q_i
//                        and a workgroup partial of p^T q.
//   mw_dot_*             fixed-order dot: per-thread sequential over a few
//                        elements, wavefront shuffle tree, LDS tree across
//                        wavefronts, workgroup slots, one-workgroup
//                        finaliser (pairwise tree).
//   mw_cg_update_r       r = r - alpha q, x = x + alpha p, quasi
//                        normalisation of r, workgroup partial of r^T r.
//   mw_cg_final_*        one-workgroup finalisers: alpha = rho / sigma,
//                        and beta, the FP64 residual test and the stop flag.
//   mw_cg_update_p       p = r + beta p.
// Workgroup indices of the streaming kernels are remapped so each XCD
// (8 per MI355X, one L2 each, workgroups dealt round-robin) works on one
// contiguous range of rows, keeping the p_j gathers of neighbouring rows in
// the same L2.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdint>
#include <cstdio>
#include <cstring>

#include "mw.h"
#include "mw_arith.hpp"

using namespace mwk;

namespace {

constexpr int NT = 256;        // threads per workgroup
constexpr int NWAVE = NT / 64;
constexpr int DOT_EPT = 8;     // elements per thread in the standalone dot
constexpr int FIN_NT = 256;    // threads of the one-workgroup finalisers

// nonzeros staged per LDS chunk in the SpMV (per-thread share = SPMV_NPT)
template <int A>
constexpr int spmv_npt() { return 8; }

__device__ __forceinline__ int xcd_remap(int bid, int nb)
{
    const int q = nb >> 3, rem = nb & 7;
    const int x = bid & 7, j = bid >> 3;
    return x * q + (x < rem ? x : rem) + j;
}

// ------------------------------------------------------------ reductions

// Sum of v over the workgroup (NT threads); result valid in thread 0.
// Order: shuffle tree over each wavefront (offsets 32..1), then the
// wavefront sums pairwise: (w0 + w1) + (w2 + w3).
template <int A>
__device__ __forceinline__ Num<A> block_sum(Num<A> v)
{
    __shared__ Num<A> part[NWAVE];
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v = add<A>(v, shfl_down<A>(v, off));
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    if (lane == 0) part[wid] = v;
    __syncthreads();
    Num<A> r = v;
    if (threadIdx.x == 0) {
        r = add<A>(add<A>(part[0], part[1]), add<A>(part[2], part[3]));
    }
    return r;
}

// Sum of nslots k-word partials (slot-major: slot s at s*K) by one
// workgroup: thread t adds slots t, t+FIN_NT, ... in order, then block_sum.
template <int A>
__device__ __forceinline__ Num<A> reduce_slots(int nslots, const double *__restrict__ slots)
{
    constexpr int K = words(A);
    Num<A> acc = zero<A>();
    for (int s = threadIdx.x; s < nslots; s += FIN_NT) acc = add<A>(acc, load_scalar<A>(slots + (long)s * K));
    return block_sum<A>(acc);
}

template <int A>
__device__ __forceinline__ Num<A> dot_step(const Num<A> &acc, const Num<A> &x, const Num<A> &y)
{
    if constexpr (A == FP64) return promote<A>(__builtin_fma(x.w[0], y.w[0], acc.w[0]));
    else return add<A>(acc, mul<A>(x, y));
}

// ------------------------------------------------------------- CG state

struct CgState {
    double rho[3];
    double alpha[3];
    double beta[3];
    double nb;        // ||b||_2
    double tol;
    double rel_res;   // last relative residual
    double *history;  // optional per-iteration relative residuals
    int32_t active;   // 1 while iterating
    int32_t status;   // MW_OK / MW_NOT_CONVERGED / MW_BREAKDOWN
    int32_t iters;
    int32_t maxit;
    int32_t normalize;
    int32_t pad[3];
};

// ------------------------------------------------------- element-wise

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
    const int nb = gridDim.x;
    const long i = (long)xcd_remap(blockIdx.x, nb) * NT + threadIdx.x;
    if (i >= n) return;
    const Num<A> al = load_scalar<A>(alpha);
    store<A>(y, n, i, axpy_term<A>(al, load<A>(x, n, i), load<A>(y, n, i)));
}

// ----------------------------------------------------------------- dot

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
    const Num<A> s = block_sum<A>(acc);
    if (threadIdx.x == 0) store_scalar<A>(slots + (long)blockIdx.x * K, s);
}

template <int A>
__global__ void __launch_bounds__(FIN_NT) mw_dot_final_kernel(int nslots, const double *__restrict__ slots,
                                                              double *__restrict__ result)
{
    const Num<A> s = reduce_slots<A>(nslots, slots);
    if (threadIdx.x == 0) store_scalar<A>(result, s);
}

// ---------------------------------------------------------------- SpMV
//
// One workgroup owns NT consecutive rows (one per thread).  Its nonzeros
// [row_ptr[r0], row_ptr[r0 + NT]) are processed in chunks of CH = NT * NPT:
// phase 1 has thread t load nonzeros t, t + NT, ... of the chunk (coalesced
// val/col streams, gathered x_j) and leave the FP64 x multi-word product in
// LDS (FP64: the pair (a_ij, x_j), since its accumulation is one fma);
// phase 2 has every thread add the products of its own row that fall in the
// chunk, in CSR order, into a register accumulator that persists across
// chunks.
//
// MODE 0: y = A x.
// MODE 1 (CG): x is p, y is q; also the workgroup partial of p^T q
//              (mul(p_i, q_i) per row) into slots[logical block]; the whole
//              workgroup exits at once when the solve has stopped.
template <int A, int MODE>
__global__ void __launch_bounds__(NT) mw_spmv_kernel(int n, const int32_t *__restrict__ row_ptr,
                                                     const int32_t *__restrict__ col,
                                                     const double *__restrict__ val,
                                                     const double *__restrict__ x, double *__restrict__ y,
                                                     double *__restrict__ slots, const CgState *__restrict__ st)
{
    constexpr int K = words(A);
    constexpr int CH = NT * spmv_npt<A>();
    constexpr int LW = (A == FP64) ? 2 : K;  // LDS words per nonzero
    __shared__ double lds[LW][CH];

    if constexpr (MODE == 1) {
        if (!st->active) return;
    }
    const int nb = gridDim.x;
    const int lb = xcd_remap(blockIdx.x, nb);
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
        for (int j = 0; j < spmv_npt<A>(); ++j) {
            const int t = (int)threadIdx.x + j * NT;
            if (t < cn) {
                const double a = val[c0 + t];
                const int c = col[c0 + t];
                const Num<A> xj = load<A>(x, n, c);
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
        if (row < n) c = mul<A>(load<A>(x, n, row), acc);
        const Num<A> s = block_sum<A>(c);
        if (threadIdx.x == 0) store_scalar<A>(slots + (long)lb * K, s);
    }
}

// ------------------------------------------------------------ CG steps

// r = b - q (q = A x0), p = r, partials of r^T r and b^T b.
template <int A>
__global__ void __launch_bounds__(NT) mw_cg_init_kernel(int n, const double *__restrict__ b,
                                                        const double *__restrict__ q, double *__restrict__ r,
                                                        double *__restrict__ p, double *__restrict__ slots_rr,
                                                        double *__restrict__ slots_bb)
{
    constexpr int K = words(A);
    const int nb = gridDim.x;
    const int lb = xcd_remap(blockIdx.x, nb);
    const long i = (long)lb * NT + threadIdx.x;
    Num<A> rr = zero<A>(), bb = zero<A>();
    if (i < n) {
        const Num<A> bi = promote<A>(b[i]);
        Num<A> ri;
        if constexpr (A == FP64) ri = promote<A>(bi.w[0] - q[i]);
        else ri = add<A>(bi, neg<A>(load<A>(q, n, i)));
        store<A>(r, n, i, ri);
        store<A>(p, n, i, ri);
        rr = mul<A>(ri, ri);
        bb = mul<A>(bi, bi);
    }
    const Num<A> s1 = block_sum<A>(rr);
    __syncthreads();
    const Num<A> s2 = block_sum<A>(bb);
    if (threadIdx.x == 0) {
        store_scalar<A>(slots_rr + (long)lb * K, s1);
        store_scalar<A>(slots_bb + (long)lb * K, s2);
    }
}

template <int A>
__global__ void __launch_bounds__(FIN_NT) mw_cg_init_final_kernel(int nslots, const double *__restrict__ slots_rr,
                                                                  const double *__restrict__ slots_bb,
                                                                  CgState *__restrict__ st)
{
    const Num<A> rho = reduce_slots<A>(nslots, slots_rr);
    __syncthreads();
    const Num<A> bb = reduce_slots<A>(nslots, slots_bb);
    if (threadIdx.x == 0) {
        store_scalar<A>(st->rho, rho);
        st->nb = sqrt(to_fp64<A>(bb));
        st->iters = 0;
        st->status = MW_OK;
        const double r64 = to_fp64<A>(rho);
        st->rel_res = sqrt(r64) / st->nb;
        if (r64 == 0.0) {
            st->rel_res = 0.0;
            st->active = 0;
        } else if (st->maxit == 0) {
            st->status = MW_NOT_CONVERGED;
            st->active = 0;
        } else {
            st->active = 1;
        }
    }
}

// alpha = rho / sigma, with the breakdown test on sigma and alpha.
template <int A>
__global__ void __launch_bounds__(FIN_NT) mw_cg_final_alpha_kernel(int nslots, const double *__restrict__ slots,
                                                                   CgState *__restrict__ st)
{
    if (!st->active) return;
    const Num<A> sigma = reduce_slots<A>(nslots, slots);
    if (threadIdx.x == 0) {
        const double s64 = to_fp64<A>(sigma);
        if (!(s64 > 0.0) || !isfinite(s64)) {
            st->status = MW_BREAKDOWN;
            st->active = 0;
            return;
        }
        const Num<A> al = div<A>(load_scalar<A>(st->rho), sigma);
        if (!isfinite(to_fp64<A>(al))) {
            st->status = MW_BREAKDOWN;
            st->active = 0;
            return;
        }
        store_scalar<A>(st->alpha, al);
    }
}

// x = x + alpha p;  r = r - alpha q;  quasi: r = normalise(r);  partial of r^T r.
template <int A>
__global__ void __launch_bounds__(NT) mw_cg_update_r_kernel(int n, const double *__restrict__ q,
                                                            const double *__restrict__ p, double *__restrict__ r,
                                                            double *__restrict__ x, double *__restrict__ slots,
                                                            const CgState *__restrict__ st)
{
    constexpr int K = words(A);
    if (!st->active) return;
    const int nb = gridDim.x;
    const int lb = xcd_remap(blockIdx.x, nb);
    const long i = (long)lb * NT + threadIdx.x;
    Num<A> rr = zero<A>();
    if (i < n) {
        const Num<A> al = load_scalar<A>(st->alpha);
        store<A>(x, n, i, axpy_term<A>(al, load<A>(p, n, i), load<A>(x, n, i)));
        Num<A> ri = axmy_term<A>(al, load<A>(q, n, i), load<A>(r, n, i));
        if constexpr (is_quasi(A)) {
            if (st->normalize) ri = normalise<A>(ri);
        }
        store<A>(r, n, i, ri);
        rr = mul<A>(ri, ri);
    }
    const Num<A> s = block_sum<A>(rr);
    if (threadIdx.x == 0) store_scalar<A>(slots + (long)lb * K, s);
}

// rho' = sum of partials; iteration count; FP64 residual test; beta.
template <int A>
__global__ void __launch_bounds__(FIN_NT) mw_cg_final_beta_kernel(int nslots, const double *__restrict__ slots,
                                                                  CgState *__restrict__ st)
{
    if (!st->active) return;
    const Num<A> rho_new = reduce_slots<A>(nslots, slots);
    if (threadIdx.x == 0) {
        const int it = st->iters + 1;
        st->iters = it;
        const double rr = to_fp64<A>(rho_new);
        if (!isfinite(rr)) {
            st->status = MW_BREAKDOWN;
            st->active = 0;
            return;
        }
        const double rel = sqrt(rr) / st->nb;
        st->rel_res = rel;
        if (st->history) st->history[it - 1] = rel;
        if (rel < st->tol) {
            st->status = MW_OK;
            st->active = 0;
            return;
        }
        if (it >= st->maxit) {
            st->status = MW_NOT_CONVERGED;
            st->active = 0;
            return;
        }
        store_scalar<A>(st->beta, div<A>(rho_new, load_scalar<A>(st->rho)));
        store_scalar<A>(st->rho, rho_new);
    }
}

// p = r + beta p.
template <int A>
__global__ void __launch_bounds__(NT) mw_cg_update_p_kernel(int n, const double *__restrict__ r, double *__restrict__ p,
                                                            const CgState *__restrict__ st)
{
    if (!st->active) return;
    const int nb = gridDim.x;
    const long i = (long)xcd_remap(blockIdx.x, nb) * NT + threadIdx.x;
    if (i >= n) return;
    const Num<A> be = load_scalar<A>(st->beta);
    store<A>(p, n, i, axpy_term<A>(be, load<A>(p, n, i), load<A>(r, n, i)));
}

// ------------------------------------------------------------ host side

thread_local char g_err[256] = "";

int hip_fail(hipError_t e, const char *what)
{
    snprintf(g_err, sizeof(g_err), "%s: %s", what, hipGetErrorString(e));
    return MW_EHIP;
}

#define HIP_TRY(call)                                  \
    do {                                               \
        hipError_t e_ = (call);                        \
        if (e_ != hipSuccess) return hip_fail(e_, #call); \
    } while (0)

inline int blocks_for(long n, long per) { return (int)((n + per - 1) / per); }

inline size_t align256(size_t b) { return (b + 255) & ~(size_t)255; }

bool valid_arith(int a) { return a >= MW_FP64 && a <= MW_QTW; }

bool valid_csr(const mw_csr_t *A)
{
    return A && A->n > 0 && A->nnz >= 0 && A->row_ptr && A->col_idx && A->val;
}

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
int spmv_launch(const mw_csr_t *M, const double *x, double *y, double *slots, const CgState *st, int mode,
                hipStream_t s)
{
    const int nb = blocks_for(M->n, NT);
    if (mode == 0)
        hipLaunchKernelGGL((mw_spmv_kernel<A, 0>), dim3(nb), dim3(NT), 0, s, M->n, M->row_ptr, M->col_idx, M->val,
                           x, y, slots, st);
    else
        hipLaunchKernelGGL((mw_spmv_kernel<A, 1>), dim3(nb), dim3(NT), 0, s, M->n, M->row_ptr, M->col_idx, M->val,
                           x, y, slots, st);
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
    hipLaunchKernelGGL((mw_dot_final_kernel<A>), dim3(1), dim3(FIN_NT), 0, s, nb, slots, res);
    HIP_TRY(hipGetLastError());
    return MW_OK;
}

// Workspace of the solver: r, p, q (K planes each), two slot arrays, state.
struct CgLayout {
    size_t r, p, q, slots_a, slots_b, state, total;
};

CgLayout cg_layout(int a, int32_t n)
{
    const size_t K = (size_t)words(a);
    const size_t plane = align256(sizeof(double) * (size_t)n * K);
    const size_t nslot = (size_t)blocks_for(n, NT);
    const size_t slots = align256(sizeof(double) * nslot * K);
    CgLayout L;
    L.r = 0;
    L.p = L.r + plane;
    L.q = L.p + plane;
    L.slots_a = L.q + plane;
    L.slots_b = L.slots_a + slots;
    L.state = L.slots_b + slots;
    L.total = L.state + align256(sizeof(CgState));
    return L;
}

int *pinned_flags()
{
    thread_local int *buf = nullptr;
    if (!buf) {
        if (hipHostMalloc((void **)&buf, 4 * sizeof(int), hipHostMallocDefault) != hipSuccess) buf = nullptr;
    }
    return buf;
}

template <int A>
int cg_a(const mw_csr_t *M, const double *b, double *x, double tol, int32_t maxit, const mw_cg_opts_t *opts,
         void *ws, mw_cg_info_t *info, hipStream_t s)
{
    const int n = M->n;
    const CgLayout L = cg_layout(A, n);
    char *base = (char *)ws;
    double *r = (double *)(base + L.r);
    double *p = (double *)(base + L.p);
    double *q = (double *)(base + L.q);
    double *sa = (double *)(base + L.slots_a);
    double *sb = (double *)(base + L.slots_b);
    CgState *st = (CgState *)(base + L.state);
    const int nb = blocks_for(n, NT);
    const int chunk = (opts && opts->chunk > 0) ? opts->chunk : 32;

    CgState h;
    memset(&h, 0, sizeof(h));
    h.tol = tol;
    h.maxit = maxit;
    h.normalize = opts ? opts->normalize : 1;
    h.history = opts ? opts->history : nullptr;
    int *flags = pinned_flags();
    if (!flags) return hip_fail(hipErrorOutOfMemory, "hipHostMalloc");

    hipEvent_t e0, e1;
    HIP_TRY(hipEventCreate(&e0));
    HIP_TRY(hipEventCreate(&e1));
    HIP_TRY(hipEventRecord(e0, s));
    HIP_TRY(hipMemcpyAsync(st, &h, sizeof(CgState), hipMemcpyHostToDevice, s));

    int rc = spmv_launch<A>(M, x, q, nullptr, nullptr, 0, s);
    if (rc) return rc;
    hipLaunchKernelGGL((mw_cg_init_kernel<A>), dim3(nb), dim3(NT), 0, s, n, b, q, r, p, sa, sb);
    HIP_TRY(hipGetLastError());
    hipLaunchKernelGGL((mw_cg_init_final_kernel<A>), dim3(1), dim3(FIN_NT), 0, s, nb, sa, sb, st);
    HIP_TRY(hipGetLastError());
    HIP_TRY(hipMemcpyAsync(flags, &st->active, sizeof(int), hipMemcpyDeviceToHost, s));
    HIP_TRY(hipStreamSynchronize(s));

    while (flags[0]) {
        for (int it = 0; it < chunk; ++it) {
            rc = spmv_launch<A>(M, p, q, sa, st, 1, s);
            if (rc) return rc;
            hipLaunchKernelGGL((mw_cg_final_alpha_kernel<A>), dim3(1), dim3(FIN_NT), 0, s, nb, sa, st);
            hipLaunchKernelGGL((mw_cg_update_r_kernel<A>), dim3(nb), dim3(NT), 0, s, n, q, p, r, x, sa, st);
            hipLaunchKernelGGL((mw_cg_final_beta_kernel<A>), dim3(1), dim3(FIN_NT), 0, s, nb, sa, st);
            hipLaunchKernelGGL((mw_cg_update_p_kernel<A>), dim3(nb), dim3(NT), 0, s, n, r, p, st);
        }
        HIP_TRY(hipGetLastError());
        HIP_TRY(hipMemcpyAsync(flags, &st->active, sizeof(int), hipMemcpyDeviceToHost, s));
        HIP_TRY(hipStreamSynchronize(s));
    }
    HIP_TRY(hipMemcpyAsync(&h, st, sizeof(CgState), hipMemcpyDeviceToHost, s));
    HIP_TRY(hipEventRecord(e1, s));
    HIP_TRY(hipStreamSynchronize(s));
    float ms = 0.f;
    HIP_TRY(hipEventElapsedTime(&ms, e0, e1));
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if (info) {
        info->iters = h.iters;
        info->status = h.status;
        info->rel_res = h.rel_res;
        info->seconds = ms * 1e-3;
    }
    return h.status;
}

}  // namespace

// ================================================================ C ABI

extern "C" {

int mw_words(mw_arith_t a) { return valid_arith(a) ? words(a) : -1; }

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

const char *mw_last_error(void) { return g_err; }

#define DISPATCH(a, fn, ...)                              \
    switch (a) {                                          \
    case MW_FP64: return fn<FP64>(__VA_ARGS__);           \
    case MW_DW: return fn<DW>(__VA_ARGS__);               \
    case MW_QDW: return fn<QDW>(__VA_ARGS__);             \
    case MW_TW: return fn<TW>(__VA_ARGS__);               \
    default: return fn<QTW>(__VA_ARGS__);                 \
    }

int mw_elementwise(mw_arith_t a, int op, int32_t n, const double *u, const double *v, double *w, void *stream)
{
    if (!valid_arith(a) || op < MW_OP_ADD || op > MW_OP_TOFP64 || n < 0 || (n > 0 && (!u || !w)))
        return MW_EINVAL;
    const bool needs_v = (op == MW_OP_ADD || op == MW_OP_MUL || op == MW_OP_DXMUL || op == MW_OP_DIV);
    if (needs_v && n > 0 && !v) return MW_EINVAL;
    if (n == 0) return MW_OK;
    hipStream_t s = (hipStream_t)stream;
    DISPATCH(a, elementwise_a, op, n, u, v, w, s);
}

int mw_axpy(mw_arith_t a, int32_t n, const double *alpha, const double *x, double *y, void *stream)
{
    if (!valid_arith(a) || n < 0 || (n > 0 && (!alpha || !x || !y))) return MW_EINVAL;
    if (n == 0) return MW_OK;
    hipStream_t s = (hipStream_t)stream;
    switch (a) {
    case MW_FP64: hipLaunchKernelGGL((mw_axpy_kernel<FP64>), dim3(blocks_for(n, NT)), dim3(NT), 0, s, n, alpha, x, y); break;
    case MW_DW: hipLaunchKernelGGL((mw_axpy_kernel<DW>), dim3(blocks_for(n, NT)), dim3(NT), 0, s, n, alpha, x, y); break;
    case MW_QDW: hipLaunchKernelGGL((mw_axpy_kernel<QDW>), dim3(blocks_for(n, NT)), dim3(NT), 0, s, n, alpha, x, y); break;
    case MW_TW: hipLaunchKernelGGL((mw_axpy_kernel<TW>), dim3(blocks_for(n, NT)), dim3(NT), 0, s, n, alpha, x, y); break;
    default: hipLaunchKernelGGL((mw_axpy_kernel<QTW>), dim3(blocks_for(n, NT)), dim3(NT), 0, s, n, alpha, x, y); break;
    }
    HIP_TRY(hipGetLastError());
    return MW_OK;
}

size_t mw_dot_workspace_bytes(mw_arith_t a, int32_t n)
{
    if (!valid_arith(a) || n < 0) return 0;
    const size_t nb = (size_t)(n > 0 ? blocks_for(n, (long)NT * DOT_EPT) : 0);
    return align256(sizeof(double) * words(a) * (nb > 0 ? nb : 1));
}

int mw_dot(mw_arith_t a, int32_t n, const double *x, const double *y, double *result, void *workspace,
           void *stream)
{
    if (!valid_arith(a) || n < 0 || !result || !workspace || (n > 0 && (!x || !y))) return MW_EINVAL;
    hipStream_t s = (hipStream_t)stream;
    DISPATCH(a, dot_a, n, x, y, result, workspace, s);
}

int mw_spmv(mw_arith_t a, const mw_csr_t *A, const double *x, double *y, void *stream)
{
    if (!valid_arith(a) || !valid_csr(A) || !x || !y || x == y) return MW_EINVAL;
    hipStream_t s = (hipStream_t)stream;
    switch (a) {
    case MW_FP64: return spmv_launch<FP64>(A, x, y, nullptr, nullptr, 0, s);
    case MW_DW: return spmv_launch<DW>(A, x, y, nullptr, nullptr, 0, s);
    case MW_QDW: return spmv_launch<QDW>(A, x, y, nullptr, nullptr, 0, s);
    case MW_TW: return spmv_launch<TW>(A, x, y, nullptr, nullptr, 0, s);
    default: return spmv_launch<QTW>(A, x, y, nullptr, nullptr, 0, s);
    }
}

size_t mw_cg_workspace_bytes(mw_arith_t a, int32_t n, int32_t nnz)
{
    (void)nnz;
    if (!valid_arith(a) || n <= 0) return 0;
    return cg_layout(a, n).total;
}

int mw_cg_solve(mw_arith_t a, const mw_csr_t *A, const double *b, double *x, double tol, int32_t maxit,
                const mw_cg_opts_t *opts, void *workspace, mw_cg_info_t *info, void *stream)
{
    if (!valid_arith(a) || !valid_csr(A) || !b || !x || !workspace || !(tol >= 0.0) || maxit < 0)
        return MW_EINVAL;
    hipStream_t s = (hipStream_t)stream;
    DISPATCH(a, cg_a, A, b, x, tol, maxit, opts, workspace, info, s);
}

}  // extern "C"
