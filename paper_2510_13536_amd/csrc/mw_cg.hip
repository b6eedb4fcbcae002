// mw_cg.hip -- the CG driver of libmwcg (gfx950).
//
// Method: Mukunoki & Ozaki, arXiv 2510.13536, Alg. 1 with Sec. IV-C (A, b
// FP64; x, vectors and scalars in the arithmetic; FP64 residual test) and
// Sec. IV-D (QDW/QTW normalise r after its update, once per iteration).
//
// One iteration is five kernels on one stream; kernel boundaries are the
// only grid-wide synchronisation (cheaper on this GPU than a software grid
// barrier or a fence-and-counter "last workgroup" reduction):
//   1. q = A p and the workgroup partials of p^T q   (SpMV, SELL-64 plan)
//   2. alpha = rho / p^T q, breakdown test           (one workgroup)
//   3. r = r - alpha q, normalise r (quasi types), partials of r^T r
//   4. rho' = r^T r, FP64 residual test, beta         (one workgroup)
//   5. x = x + alpha p, p = r + beta p
// The x update of iteration i runs in kernel 5 with the p that kernel 1
// read (x is not read by anything else), which saves a pass over p; when
// the solve stops in kernel 4, the stopping iteration's x update is applied
// by one closing kernel.  Every kernel first reads the device flag and
// exits at once after the stop, so a chunk of iterations can be enqueued
// (or replayed from a captured hipGraph) and the host checks the flag once
// per chunk.  Partial sums use fixed slots and a fixed order: the solve is
// run-to-run reproducible.
#include "mw_blas.hpp"

#include <cstring>

using namespace mwk;
using namespace mwh;

namespace {

// r = b - q (q = A x0), p = r, partials of r^T r and b^T b.
template <int A>
__global__ void __launch_bounds__(NT) mw_cg_init_kernel(int n, const double *__restrict__ b,
                                                        const double *__restrict__ q, double *__restrict__ r,
                                                        double *__restrict__ p, double *__restrict__ slots_rr,
                                                        double *__restrict__ slots_bb)
{
    constexpr int K = words(A);
    const TileRange tr = xcd_tiles((n + NT - 1) / NT);
    Num<A> rr = zero<A>(), bb = zero<A>();
    for (int t = tr.first; t < tr.end; t += tr.step) {
        const long i = (long)t * NT + threadIdx.x;
        if (i >= n) continue;
        const Num<A> bi = promote<A>(b[i]);
        Num<A> ri;
        if constexpr (A == FP64) ri = promote<A>(bi.w[0] - q[i]);
        else ri = add<A>(bi, neg<A>(load<A>(q, n, i)));
        store<A>(r, n, i, ri);
        store<A>(p, n, i, ri);
        rr = dot_step<A>(rr, ri, ri);
        bb = dot_step<A>(bb, bi, bi);
    }
    const Num<A> s1 = block_sum<A, NT>(rr);
    const Num<A> s2 = block_sum<A, NT>(bb);
    if (threadIdx.x == 0) {
        store_scalar<A>(slots_rr + (long)blockIdx.x * K, s1);
        store_scalar<A>(slots_bb + (long)blockIdx.x * K, s2);
    }
}

template <int A>
__global__ void __launch_bounds__(FIN_NT) mw_cg_init_final_kernel(int nslots, const double *__restrict__ slots_rr,
                                                                  const double *__restrict__ slots_bb,
                                                                  CgState *__restrict__ st)
{
    const Num<A> rho = reduce_slots<A>(nslots, slots_rr);
    const Num<A> bb = reduce_slots<A>(nslots, slots_bb);
    if (threadIdx.x == 0) {
        store_scalar<A>(st->rho, rho);
        st->nb = sqrt(to_fp64<A>(bb));
        st->iters = 0;
        st->status = MW_OK;
        st->x_due = 0;
        const double r64 = to_fp64<A>(rho);
        if (r64 == 0.0) {
            st->rel_res = 0.0;
            st->active = 0;
        } else {
            st->rel_res = sqrt(r64) / st->nb;
            if (st->maxit == 0) {
                st->status = MW_NOT_CONVERGED;
                st->active = 0;
            } else {
                st->active = 1;
            }
        }
    }
}

// alpha = rho / sigma with the breakdown tests on sigma and alpha.
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

// r = r - alpha q; quasi: r = normalise(r); partials of r^T r.
template <int A>
__global__ void __launch_bounds__(NT) mw_cg_update_r_kernel(int n, const double *__restrict__ q, double *__restrict__ r,
                                                            double *__restrict__ slots, const CgState *__restrict__ st)
{
    constexpr int K = words(A);
    if (!st->active) return;
    const TileRange tr = xcd_tiles((n + NT - 1) / NT);
    const Num<A> al = load_scalar<A>(st->alpha);
    const bool norm = is_quasi(A) && st->normalize;
    Num<A> rr = zero<A>();
    for (int t = tr.first; t < tr.end; t += tr.step) {
        const long i = (long)t * NT + threadIdx.x;
        if (i >= n) continue;
        Num<A> ri = axmy_term<A>(al, load<A>(q, n, i), load<A>(r, n, i));
        if (norm) ri = normalise<A>(ri);
        store<A>(r, n, i, ri);
        rr = dot_step<A>(rr, ri, ri);
    }
    const Num<A> s = block_sum<A, NT>(rr);
    if (threadIdx.x == 0) store_scalar<A>(slots + (long)blockIdx.x * K, s);
}

// rho' = sum of partials; iteration count; FP64 test; beta.
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
            st->x_due = 1;
            return;
        }
        const double rel = sqrt(rr) / st->nb;
        st->rel_res = rel;
        if (st->history) st->history[it - 1] = rel;
        if (rel < st->tol || it >= st->maxit) {
            st->status = (rel < st->tol) ? MW_OK : MW_NOT_CONVERGED;
            st->active = 0;
            st->x_due = 1;
            return;
        }
        store_scalar<A>(st->beta, div<A>(rho_new, load_scalar<A>(st->rho)));
        store_scalar<A>(st->rho, rho_new);
    }
}

// x = x + alpha p;  p = r + beta p  (both with the p of this iteration).
template <int A>
__global__ void __launch_bounds__(NT) mw_cg_update_p_kernel(int n, const double *__restrict__ r, double *__restrict__ p,
                                                            double *__restrict__ x, const CgState *__restrict__ st)
{
    if (!st->active) return;
    const long i = (long)xcd_remap(blockIdx.x, gridDim.x) * NT + threadIdx.x;
    if (i >= n) return;
    const Num<A> al = load_scalar<A>(st->alpha);
    const Num<A> be = load_scalar<A>(st->beta);
    const Num<A> pi = load<A>(p, n, i);
    store<A>(x, n, i, axpy_term<A>(al, pi, load<A>(x, n, i)));
    store<A>(p, n, i, axpy_term<A>(be, pi, load<A>(r, n, i)));
}

// The stopping iteration's x = x + alpha p.
template <int A>
__global__ void __launch_bounds__(NT) mw_cg_final_x_kernel(int n, const double *__restrict__ p, double *__restrict__ x,
                                                           const CgState *__restrict__ st)
{
    if (!st->x_due) return;
    const long i = (long)xcd_remap(blockIdx.x, gridDim.x) * NT + threadIdx.x;
    if (i >= n) return;
    const Num<A> al = load_scalar<A>(st->alpha);
    store<A>(x, n, i, axpy_term<A>(al, load<A>(p, n, i), load<A>(x, n, i)));
}

// ------------------------------------------------------------ host side

struct CgLayout {
    size_t r, p, q, slots_a, slots_b, state, plan, total;
};

CgLayout cg_layout(int a, int32_t n, int32_t nnz)
{
    const size_t K = (size_t)words(a);
    const size_t plane = align256(sizeof(double) * (size_t)n * K);
    const size_t slots = align256(sizeof(double) * (size_t)spmv_max_slots(n) * K);
    CgLayout L;
    L.r = 0;
    L.p = L.r + plane;
    L.q = L.p + plane;
    L.slots_a = L.q + plane;
    L.slots_b = L.slots_a + slots;
    L.state = L.slots_b + slots;
    L.plan = L.state + align256(sizeof(CgState));
    L.total = L.plan + plan_bytes(n, nnz);
    return L;
}

int *pinned_flags()
{
    thread_local int *buf = nullptr;
    if (!buf && hipHostMalloc((void **)&buf, 64, hipHostMallocDefault) != hipSuccess) buf = nullptr;
    return buf;
}

// The library's own stream per thread (default priority): graph capture is
// not possible on the legacy default stream a caller may pass.
hipStream_t own_stream()
{
    thread_local hipStream_t s = nullptr;
    if (!s && hipStreamCreateWithFlags(&s, hipStreamNonBlocking) != hipSuccess) s = nullptr;
    return s;
}

struct EventPool {
    hipEvent_t *e = nullptr;
    int n = 0;
    int init(int count)
    {
        release();
        e = new hipEvent_t[count];
        for (; n < count; ++n) HIP_TRY(hipEventCreate(&e[n]));
        return MW_OK;
    }
    void release()
    {
        for (int i = 0; i < n; ++i) (void)hipEventDestroy(e[i]);
        delete[] e;
        e = nullptr;
        n = 0;
    }
    ~EventPool() { release(); }
};

constexpr int NKERN = 5;  // kernels per iteration
constexpr int KCLASS[NKERN] = {MW_PROF_SPMV, MW_PROF_FINAL, MW_PROF_UPDATE_R, MW_PROF_FINAL, MW_PROF_UPDATE_P};

// Everything one chunk of iterations needs.
struct ChunkArgs {
    int arith, n, nslots_sp, nslots_up, chunk, timed_mask;
    const mw_csr_t *M;
    const mw_spmv_plan_t *plan;
    double *r, *p, *q, *x, *slots;
    CgState *st;
};

bool same_key(const ChunkArgs &a, const ChunkArgs &b)
{
    return a.arith == b.arith && a.n == b.n && a.nslots_sp == b.nslots_sp && a.nslots_up == b.nslots_up &&
           a.chunk == b.chunk && a.timed_mask == b.timed_mask && a.r == b.r && a.p == b.p && a.q == b.q &&
           a.x == b.x && a.slots == b.slots && a.st == b.st && a.plan && b.plan &&
           a.plan->format == b.plan->format && a.plan->slice_ptr == b.plan->slice_ptr &&
           a.plan->col == b.plan->col && a.plan->val == b.plan->val && a.M->row_ptr == b.M->row_ptr &&
           a.M->col_idx == b.M->col_idx && a.M->val == b.M->val && a.M->n == b.M->n;
}

// Enqueues one chunk; with a mask, records events around the timed classes.
template <int A>
int enqueue_chunk(const ChunkArgs &c, EventPool *ev, hipStream_t s)
{
    const int nbp = blocks_for(c.n, NT);
    const int gup = persistent_grid(blocks_for(c.n, NT));
    for (int it = 0; it < c.chunk; ++it) {
        for (int k = 0; k < NKERN; ++k) {
            const bool timed = ev && (c.timed_mask & (1 << KCLASS[k]));
            if (timed) HIP_TRY(hipEventRecord(ev->e[(it * NKERN + k) * 2], s));
            switch (k) {
            case 0: {
                const int rc = spmv_launch<A>(c.M, c.plan, c.p, c.q, c.slots, c.st, 1, s);
                if (rc) return rc;
                break;
            }
            case 1:
                hipLaunchKernelGGL((mw_cg_final_alpha_kernel<A>), dim3(1), dim3(FIN_NT), 0, s, c.nslots_sp, c.slots,
                                   c.st);
                break;
            case 2:
                hipLaunchKernelGGL((mw_cg_update_r_kernel<A>), dim3(gup), dim3(NT), 0, s, c.n, c.q, c.r, c.slots,
                                   c.st);
                break;
            case 3:
                hipLaunchKernelGGL((mw_cg_final_beta_kernel<A>), dim3(1), dim3(FIN_NT), 0, s, c.nslots_up, c.slots,
                                   c.st);
                break;
            default:
                hipLaunchKernelGGL((mw_cg_update_p_kernel<A>), dim3(nbp), dim3(NT), 0, s, c.n, c.r, c.p, c.x, c.st);
                break;
            }
            if (timed) HIP_TRY(hipEventRecord(ev->e[(it * NKERN + k) * 2 + 1], s));
        }
    }
    HIP_TRY(hipGetLastError());
    return MW_OK;
}

// A captured chunk, kept per thread and reused while the arguments match.
struct GraphCache {
    bool valid = false;
    ChunkArgs key{};
    mw_csr_t M{};
    mw_spmv_plan_t plan{};
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    EventPool ev;
    void release()
    {
        if (exec) (void)hipGraphExecDestroy(exec);
        if (graph) (void)hipGraphDestroy(graph);
        exec = nullptr;
        graph = nullptr;
        ev.release();
        valid = false;
    }
};

// Heap-allocated and never freed: no HIP call may run during process
// teardown, after the runtime may already be gone.
GraphCache &graph_cache()
{
    thread_local GraphCache *g = new GraphCache();
    return *g;
}

template <int A>
int cg_a(const mw_csr_t *M, const double *b, double *x, double tol, int32_t maxit, const mw_cg_opts_t *opts,
         void *ws, mw_cg_info_t *info, hipStream_t user)
{
    const int n = M->n;
    const CgLayout L = cg_layout(A, n, M->nnz);
    char *base = (char *)ws;
    double *r = (double *)(base + L.r);
    double *p = (double *)(base + L.p);
    double *q = (double *)(base + L.q);
    double *sa = (double *)(base + L.slots_a);
    double *sb = (double *)(base + L.slots_b);
    CgState *st = (CgState *)(base + L.state);
    const int chunk = (opts && opts->chunk > 0) ? opts->chunk : 32;
    mw_cg_prof_t *prof = opts ? opts->prof : nullptr;
    const int mask = prof ? (prof->mask ? prof->mask : 0xF) : 0;
    // events recorded by graph nodes cannot be read back: timing uses direct launches
    const bool use_graph = !(opts && opts->no_graph) && !prof;

    hipStream_t s = own_stream();
    int *flags = pinned_flags();
    if (!s || !flags) return hip_fail(hipErrorOutOfMemory, "stream/pinned buffer");

    hipEvent_t e_in, e0, e1;
    HIP_TRY(hipEventCreateWithFlags(&e_in, hipEventDisableTiming));
    HIP_TRY(hipEventCreate(&e0));
    HIP_TRY(hipEventCreate(&e1));
    HIP_TRY(hipEventRecord(e_in, user));
    HIP_TRY(hipStreamWaitEvent(s, e_in, 0));
    HIP_TRY(hipEventRecord(e0, s));

    // SpMV plan: given by the caller or built here
    mw_spmv_plan_t own_plan;
    const mw_spmv_plan_t *plan = opts ? opts->plan : nullptr;
    if (!plan) {
        const int rc = plan_build(M, base + L.plan, L.total - L.plan, &own_plan, s);
        if (rc) return rc;
        plan = &own_plan;
    }

    CgState h;
    memset(&h, 0, sizeof(h));
    h.tol = tol;
    h.maxit = maxit;
    h.normalize = opts ? opts->normalize : 1;
    h.history = opts ? opts->history : nullptr;
    HIP_TRY(hipMemcpyAsync(st, &h, sizeof(CgState), hipMemcpyHostToDevice, s));

    // r0 = b - A x0, p0 = r0, rho0, ||b||
    int rc = spmv_launch<A>(M, plan, x, q, nullptr, nullptr, 0, s);
    if (rc) return rc;
    const int gi = persistent_grid(blocks_for(n, NT));
    hipLaunchKernelGGL((mw_cg_init_kernel<A>), dim3(gi), dim3(NT), 0, s, n, b, q, r, p, sa, sb);
    hipLaunchKernelGGL((mw_cg_init_final_kernel<A>), dim3(1), dim3(FIN_NT), 0, s, gi, sa, sb, st);
    HIP_TRY(hipGetLastError());
    HIP_TRY(hipMemcpyAsync(flags, &st->active, 3 * sizeof(int), hipMemcpyDeviceToHost, s));
    HIP_TRY(hipStreamSynchronize(s));

    ChunkArgs c{};
    c.arith = A;
    c.n = n;
    c.chunk = chunk;
    c.timed_mask = mask;
    c.M = M;
    c.plan = plan;
    c.r = r;
    c.p = p;
    c.q = q;
    c.x = x;
    c.slots = sa;
    c.st = st;
    c.nslots_up = persistent_grid(blocks_for(n, NT));
    c.nslots_sp = (plan->format == MW_FMT_SELL64) ? persistent_grid(blocks_for(plan->nslices, NWAVE))
                                                  : blocks_for(n, NT);

    EventPool local_ev;
    EventPool *ev = nullptr;
    if (flags[0]) {
        if (use_graph) {
            GraphCache &G = graph_cache();
            if (!(G.valid && same_key(G.key, c))) {
                G.release();
                if (mask && (rc = G.ev.init(2 * NKERN * chunk))) return rc;
                HIP_TRY(hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal));
                rc = enqueue_chunk<A>(c, mask ? &G.ev : nullptr, s);
                hipGraph_t g = nullptr;
                const hipError_t ce = hipStreamEndCapture(s, &g);
                if (rc) return rc;
                if (ce != hipSuccess) return hip_fail(ce, "hipStreamEndCapture");
                G.graph = g;
                HIP_TRY(hipGraphInstantiate(&G.exec, g, nullptr, nullptr, 0));
                G.key = c;
                G.M = *M;
                G.plan = *plan;
                G.key.M = &G.M;
                G.key.plan = &G.plan;
                G.valid = true;
            }
            ev = mask ? &G.ev : nullptr;
        } else if (mask) {
            if ((rc = local_ev.init(2 * NKERN * chunk))) return rc;
            ev = &local_ev;
        }
    }

    int iters_before = 0;
    while (flags[0]) {
        if (use_graph) {
            HIP_TRY(hipGraphLaunch(graph_cache().exec, s));
        } else {
            rc = enqueue_chunk<A>(c, ev, s);
            if (rc) return rc;
        }
        HIP_TRY(hipMemcpyAsync(flags, &st->active, 3 * sizeof(int), hipMemcpyDeviceToHost, s));
        HIP_TRY(hipStreamSynchronize(s));
        if (ev) {
            // iterations of this chunk that ran to completion (the one that
            // stopped the solve is left out: part of its launches exited)
            const int done = flags[2] - iters_before - (flags[0] ? 0 : 1);
            for (int it = 0; it < done && it < chunk; ++it)
                for (int k = 0; k < NKERN; ++k) {
                    if (!(mask & (1 << KCLASS[k]))) continue;
                    float ms = 0.f;
                    HIP_TRY(hipEventElapsedTime(&ms, ev->e[(it * NKERN + k) * 2], ev->e[(it * NKERN + k) * 2 + 1]));
                    prof->ms[KCLASS[k]] += ms;
                    prof->launches[KCLASS[k]] += 1;
                }
        }
        iters_before = flags[2];
    }
    hipLaunchKernelGGL((mw_cg_final_x_kernel<A>), dim3(blocks_for(n, NT)), dim3(NT), 0, s, n, p, x, st);
    HIP_TRY(hipGetLastError());
    HIP_TRY(hipMemcpyAsync(&h, st, sizeof(CgState), hipMemcpyDeviceToHost, s));
    HIP_TRY(hipEventRecord(e1, s));
    HIP_TRY(hipStreamSynchronize(s));
    float ms = 0.f;
    HIP_TRY(hipEventElapsedTime(&ms, e0, e1));
    (void)hipEventDestroy(e_in);
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

// ================================================================== C ABI

extern "C" {

size_t mw_cg_workspace_bytes(mw_arith_t a, int32_t n, int32_t nnz)
{
    if (!valid_arith(a) || n <= 0 || nnz < 0) return 0;
    return cg_layout(a, n, nnz).total;
}

int mw_cg_solve(mw_arith_t a, const mw_csr_t *A, const double *b, double *x, double tol, int32_t maxit,
                const mw_cg_opts_t *opts, void *workspace, mw_cg_info_t *info, void *stream)
{
    if (!valid_arith(a) || !valid_csr(A) || !b || !x || !workspace || !(tol >= 0.0) || maxit < 0)
        return MW_EINVAL;
    if (opts && opts->plan && (opts->plan->n != A->n || opts->plan->csr.row_ptr != A->row_ptr)) return MW_EINVAL;
    MW_DISPATCH(a, cg_a, A, b, x, tol, maxit, opts, workspace, info, (hipStream_t)stream);
}

}  // extern "C"
