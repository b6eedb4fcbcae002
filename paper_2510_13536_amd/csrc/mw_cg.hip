// mw_cg.hip -- the CG driver of libmwcg (gfx950).
//
// Method: Mukunoki & Ozaki, arXiv 2510.13536, Alg. 1 with Sec. IV-C (A, b
// FP64; x, vectors and scalars in the arithmetic; FP64 residual test) and
// Sec. IV-D (QDW/QTW normalise r after its update, once per iteration).
//
// One iteration is three kernels on one stream; kernel boundaries are the
// only grid-wide synchronisation (cheaper on this GPU than a software grid
// barrier or a fence-and-counter "last workgroup" reduction):
//   1. q = A p and the workgroup partials of p^T q   (SpMV, SELL-64 plan)
//   2. every workgroup reduces those partials to the same sigma and
//      alpha = rho / sigma (breakdown test); r = r - alpha q; quasi types
//      normalise r; partials of r^T r
//   3. every workgroup reduces those to the same rho', counts the iteration,
//      runs the FP64 residual test and forms beta; unless the solve stops
//      here, p = r + beta p
// x is needed by no step of the loop, so its updates x = x + alpha_j p_j
// may be applied XR = xr(A) iterations at a time (2 for 3-word types, else
// 1): the search directions live in a ring of XR buffers (p_k in buffer
// k % XR; with XR = 1 p is updated in place), and step 3 of every XR-th
// iteration, of the iteration that stops the solve and of one whose alpha
// step broke down adds the pending terms one after another, in iteration
// order -- the same operations on the same values as one update per
// iteration.  Chunks hold an even number of iterations, a multiple of XR,
// so each launch's buffers are fixed.  Scalars and flags an iteration
// produces are stored per iteration parity (alpha per buffer), so no
// workgroup reads what another workgroup of the same kernel writes; the
// parity and buffer of each launch are kernel arguments.
// Jacobi-preconditioned CG (opts->precond; preconditioning is future work
// in Sec. VI): the same three kernels with z = D r formed where r is (D the
// FP64 reciprocals of A's diagonal, applied as the FP64 x multi-word
// product): step 2 adds the partials of r^T z beside those of r^T r, step 3
// recomputes z from r (cheaper than storing it) for p = z + beta p and
// tests r^T r.
// After the stop every kernel only passes the stop flag on and exits, so a
// chunk of iterations is enqueued (or replayed from a captured hipGraph)
// and the host checks the flag once per chunk.  All reductions use fixed
// slots and a fixed order: the solve is run-to-run reproducible.
#include "mw_blas.hpp"

#include <cstdlib>
#include <cstring>

using namespace mwk;
using namespace mwh;

namespace {

// Workspace slot arrays hold the partials of up to this many workgroups.
constexpr int UGRID_MAX = MAX_GRID;

// r = b - q (q = A x0), p = r, partials of r^T r and b^T b.  PC (Jacobi):
// p = z = D r, partials of r^T z (to slots_rr), b^T b and r^T r (to
// slots_c).
template <int A, bool PC>
__global__ void __launch_bounds__(NT) mw_cg_init_kernel(int n, const double *__restrict__ b,
                                                        const double *__restrict__ q, double *__restrict__ r,
                                                        double *__restrict__ p, double *__restrict__ slots_rr,
                                                        double *__restrict__ slots_bb, const double *__restrict__ dinv,
                                                        double *__restrict__ slots_c)
{
    constexpr int K = words(A);
    const TileRange tr = xcd_tiles((n + NT - 1) / NT);
    Num<A> rr = zero<A>(), bb = zero<A>(), rz = zero<A>();
    for (int t = tr.first; t < tr.end; t += tr.step) {
        const long i = (long)t * NT + threadIdx.x;
        if (i >= n) continue;
        const Num<A> bi = promote<A>(b[i]);
        Num<A> ri;
        if constexpr (A == FP64) ri = promote<A>(bi.w[0] - q[i]);
        else ri = add<A>(bi, neg<A>(load<A>(q, n, i)));
        store<A>(r, n, i, ri);
        if constexpr (PC) {
            const Num<A> zi = jacobi<A>(dinv[i], ri);
            store_il<A>(p, n, i, zi);
            rz = dot_step<A>(rz, ri, zi);
        } else {
            store_il<A>(p, n, i, ri);
        }
        rr = dot_step<A>(rr, ri, ri);
        bb = dot_step<A>(bb, bi, bi);
    }
    const Num<A> s1 = block_sum<A, NT>(PC ? rz : rr);
    const Num<A> s2 = block_sum<A, NT>(bb);
    if (threadIdx.x == 0) {
        store_scalar<A>(slots_rr + (long)blockIdx.x * K, s1);
        store_scalar<A>(slots_bb + (long)blockIdx.x * K, s2);
    }
    if constexpr (PC) {
        const Num<A> s3 = block_sum<A, NT>(rr);
        if (threadIdx.x == 0) store_scalar<A>(slots_c + (long)blockIdx.x * K, s3);
    }
}

// rho0 (PC: r^T z), ||b|| and the initial flags (parity 0); the start test
// uses r^T r.
template <int A, bool PC>
__global__ void __launch_bounds__(FIN_NT) mw_cg_init_final_kernel(int nslots, const double *__restrict__ slots_rr,
                                                                  const double *__restrict__ slots_bb,
                                                                  const double *__restrict__ slots_c,
                                                                  CgState *__restrict__ st)
{
    const Num<A> rho = reduce_slots<A>(nslots, slots_rr);
    const Num<A> bb = reduce_slots<A>(nslots, slots_bb);
    Num<A> rr = rho;
    if constexpr (PC) rr = reduce_slots<A>(nslots, slots_c);
    if (threadIdx.x == 0) {
        store_scalar<A>(st->rho[0], rho);
        st->nb = sqrt(to_fp64<A>(bb));
        st->iters[0] = 0;
        st->iters_final = 0;
        st->status = MW_OK;
        const double r64 = to_fp64<A>(rr);
        int run = 1;
        if (r64 == 0.0) {
            st->rel_res = 0.0;
            run = 0;
        } else {
            st->rel_res = sqrt(r64) / st->nb;
            if (st->maxit == 0) {
                st->status = MW_NOT_CONVERGED;
                run = 0;
            }
        }
        st->run[0] = run;
        st->stopped = !run;
    }
}

// Tiles whose operands the update kernels load before their reduction of
// the previous kernel's partials, so that those loads overlap it.  Measured
// on MI355X (3D Poisson 128^3): four against two, FP64 and DW solves -2.5 %,
// QTW -1 %; TW +0.6 % (its heavier arithmetic needs the registers), so TW
// and QTWE, and the 4-word QW and QQW, keep two.
__host__ __device__ constexpr int prefetch_tiles(int a) { return a == TW || a == QTWE || words(a) == 4 ? 2 : 4; }

// Iteration step 2 (parity par; iteration k, 0-based, with k % xr(A) = kpos):
// every workgroup reduces the p^T q partials in the same fixed order, so all
// derive the same sigma and alpha = rho / sigma (stored in slot kpos);
// breakdown (sigma <= 0 or a non-finite value) stops the solve before r or
// p change.  Then r = r - alpha q, quasi types normalise r, and the
// workgroup partial of r^T r goes to slots_out.  PC (Jacobi): the partial
// of r^T z (z = D r) goes to slots_out and that of r^T r to slots_out2.
template <int A, int UNT, bool PC>
__global__ void __launch_bounds__(UNT) mw_cg_step_r_kernel(int n, int nslots_in, const double *__restrict__ slots_in,
                                                           const double *__restrict__ q, double *__restrict__ r,
                                                           double *__restrict__ slots_out, CgState *__restrict__ st,
                                                           int par, int kpos, int rev, const double *__restrict__ dinv,
                                                           double *__restrict__ slots_out2)
{
    constexpr int K = words(A);
    __shared__ Num<A> s_alpha;
    __shared__ int s_brk;
    if (!st->run[par ^ 1]) {
        if (blockIdx.x == 0 && threadIdx.x == 0) st->run[par] = 0;
        return;
    }
    // the first D tiles' operands are loaded before the reduction, so that
    // their latency overlaps it (prefetch_tiles)
    const TileWalk tw = xcd_walk((n + UNT - 1) / UNT, rev);
    constexpr int D = prefetch_tiles(A);
    Num<A> qpre[D], rpre[D];
#pragma unroll
    for (int u = 0; u < D; ++u) {
        qpre[u] = zero<A>();
        rpre[u] = zero<A>();
        const long iu = tw.count > u ? (long)tw[u] * UNT + threadIdx.x : (long)n;
        if (iu < n) {
            qpre[u] = load<A>(q, n, iu);
            rpre[u] = load<A>(r, n, iu);
        }
    }
    const Num<A> sigma = reduce_slots<A, UNT>(nslots_in, slots_in);
    if (threadIdx.x == 0) {
        const double s64 = to_fp64<A>(sigma);
        int brk = !(s64 > 0.0) || !isfinite(s64);
        Num<A> al = zero<A>();
        if (!brk) {
            al = div<A>(load_scalar<A>(st->rho[par ^ 1]), sigma);
            brk = !isfinite(to_fp64<A>(al));
        }
        s_alpha = al;
        s_brk = brk;
        if (blockIdx.x == 0) {
            st->brk[par] = brk;
            if (brk) {
                st->run[par] = 0;
                st->status = MW_BREAKDOWN;
                st->iters_final = st->iters[par ^ 1];
                st->stopped = 1;
            } else {
                store_scalar<A>(st->alpha[kpos], al);
            }
        }
    }
    __syncthreads();
    if (s_brk) return;
    const Num<A> al = s_alpha;
    // quasi types: normalise in iterations NK, 2 NK, ... (NK = 1, every
    // iteration, is Sec. IV-D; 0 never)
    const int NK = st->normalize;
    const bool norm = is_quasi(A) && NK > 0 && (st->iters[par ^ 1] + 1) % NK == 0;
    Num<A> rr = zero<A>(), rz = zero<A>();
    for (int m = 0; m < tw.count; ++m) {
        const long i = (long)tw[m] * UNT + threadIdx.x;
        if (i >= n) continue;
        Num<A> qi, rv;
        if (m < D) {
            qi = qpre[0];
            rv = rpre[0];
#pragma unroll
            for (int u = 1; u < D; ++u)
                if (m == u) {
                    qi = qpre[u];
                    rv = rpre[u];
                }
        } else {
            qi = load<A>(q, n, i);
            rv = load<A>(r, n, i);
        }
        Num<A> ri = axmy_term<A>(al, qi, rv);
        if (norm) ri = normalise<A>(ri);
        store<A>(r, n, i, ri);
        if constexpr (PC) rz = dot_step<A>(rz, ri, jacobi<A>(dinv[i], ri));
        rr = dot_step<A>(rr, ri, ri);
    }
    const Num<A> sum = block_sum<A, UNT>(PC ? rz : rr);
    if (threadIdx.x == 0) store_scalar<A>(slots_out + (long)blockIdx.x * K, sum);
    if constexpr (PC) {
        const Num<A> sum2 = block_sum<A, UNT>(rr);
        if (threadIdx.x == 0) store_scalar<A>(slots_out2 + (long)blockIdx.x * K, sum2);
    }
}

// Iteration step 3 (parity par; iteration k with k % XR = kpos, XR =
// xr(A)): every workgroup reduces the r^T r partials to the same rho',
// counts the iteration, runs the FP64 residual test and derives
// beta = rho' / rho.  pk is p_k (buffer kpos); unless the solve stops
// here, p_{k+1} = r + beta p_k goes to buffer (kpos + 1) % XR: with
// XR = 1 that is pk itself, with XR = 2 the other buffer, po, which holds
// p_{k-1}.  x takes the pending updates x = x + alpha_j p_j in iteration
// order: those of iterations k - kpos .. k when kpos = XR - 1 or the solve
// stops here, those of iterations k - kpos .. k - 1 after a breakdown of
// this iteration's alpha step.  With XR = 2 and kpos = 1 that reads
// p_{k-1} from po before the same thread stores p_{k+1} there.
// PC (Jacobi): slots_in holds the r^T z partials (rho'), slots_in2 those of
// r^T r (the test), and p_{k+1} = z + beta p_k with z = D r recomputed.
template <int A, int UNT, bool PC>
__global__ void __launch_bounds__(UNT) mw_cg_step_p_kernel(int n, int nslots_in, const double *__restrict__ slots_in,
                                                           const double *__restrict__ r, double *__restrict__ pk,
                                                           double *__restrict__ po, double *__restrict__ x,
                                                           CgState *__restrict__ st, int par, int kpos_arg, int rev,
                                                           const double *__restrict__ slots_in2,
                                                           const double *__restrict__ dinv)
{
    constexpr int XR = xr(A);
    static_assert(XR == 1 || XR == 2, "one or two search-direction buffers");
    const int kpos = XR == 1 ? 0 : kpos_arg;
    double *pn = XR == 1 ? pk : po;  // based on pk or po
    __shared__ Num<A> s_beta;
    __shared__ int s_stop;
    if (!st->run[par ^ 1]) {
        if (blockIdx.x == 0 && threadIdx.x == 0) st->run[par] = 0;
        return;
    }
    const TileWalk tw = xcd_walk((n + UNT - 1) / UNT, rev);
    if (st->brk[par]) {
        if (blockIdx.x == 0 && threadIdx.x == 0) st->run[par] = 0;
        if (XR == 1 || kpos == 0) return;
        // XR = 2, kpos = 1: iteration k - 1 is pending, its p is in po
        const Num<A> a0 = load_scalar<A>(st->alpha[0]);
        for (int m = 0; m < tw.count; ++m) {
            const long i = (long)tw[m] * UNT + threadIdx.x;
            if (i >= n) continue;
            store<A>(x, n, i, axpy_term<A>(a0, load_il<A>(po, n, i), load<A>(x, n, i)));
        }
        return;
    }
    // the first D tiles' operands are loaded before the reduction (as in
    // step r); x of the first tile where it is due
    const bool xdue = kpos == XR - 1;
    constexpr int D = prefetch_tiles(A);
    Num<A> ppre[D], rpre[D], x0 = zero<A>();
#pragma unroll
    for (int u = 0; u < D; ++u) {
        ppre[u] = zero<A>();
        rpre[u] = zero<A>();
        const long iu = tw.count > u ? (long)tw[u] * UNT + threadIdx.x : (long)n;
        if (iu < n) {
            ppre[u] = load_il<A>(pk, n, iu);
            if (u == 0 && xdue) x0 = load<A>(x, n, iu);
            rpre[u] = load<A>(r, n, iu);
        }
    }
    const Num<A> rho_new = reduce_slots<A, UNT>(nslots_in, slots_in);
    Num<A> rr_new = rho_new;
    if constexpr (PC) rr_new = reduce_slots<A, UNT>(nslots_in, slots_in2);
    if (threadIdx.x == 0) {
        const int it = st->iters[par ^ 1] + 1;
        const double rr = to_fp64<A>(rr_new);
        const bool fin = isfinite(rr) && (!PC || isfinite(to_fp64<A>(rho_new)));
        const double rel = fin ? sqrt(rr) / st->nb : rr;
        const bool conv = fin && rel < st->tol;
        const bool stop = !fin || conv || it >= st->maxit;
        Num<A> be = zero<A>();
        if (!stop) be = div<A>(rho_new, load_scalar<A>(st->rho[par ^ 1]));
        s_beta = be;
        s_stop = stop;
        if (blockIdx.x == 0) {
            st->iters[par] = it;
            store_scalar<A>(st->rho[par], rho_new);
            st->rel_res = rel;
            if (st->history) st->history[it - 1] = rel;
            st->run[par] = !stop;
            if (stop) {
                st->status = !fin ? MW_BREAKDOWN : (conv ? MW_OK : MW_NOT_CONVERGED);
                st->iters_final = it;
                st->stopped = 1;
            }
        }
    }
    __syncthreads();
    const bool stop = s_stop;
    const Num<A> be = s_beta;
    const bool xnow = stop || xdue;
    // alpha of iteration k (slot kpos) and, with XR = 2 and kpos = 1, of k - 1
    const Num<A> ak = load_scalar<A>(st->alpha[kpos]);
    const bool two = XR == 2 && kpos == 1;
    // the placement variant normalize_p: in the iterations that normalise
    // r, p_k is normalised as it enters p_{k+1} = r + beta p_k (x takes p_k
    // as the SpMV read it)
    const int NK = st->normalize;
    const bool normp = is_quasi(A) && !PC && st->normalize_p && NK > 0 && (st->iters[par ^ 1] + 1) % NK == 0;
    const Num<A> a0 = two ? load_scalar<A>(st->alpha[0]) : zero<A>();
    for (int m = 0; m < tw.count; ++m) {
        const long i = (long)tw[m] * UNT + threadIdx.x;
        if (i >= n) continue;
        Num<A> pi, rv;
        if (m < D) {
            pi = ppre[0];
            rv = rpre[0];
#pragma unroll
            for (int u = 1; u < D; ++u)
                if (m == u) {
                    pi = ppre[u];
                    rv = rpre[u];
                }
        } else {
            pi = load_il<A>(pk, n, i);
            if (!stop) rv = load<A>(r, n, i);
        }
        if (xnow) {
            Num<A> xi = (m == 0 && xdue) ? x0 : load<A>(x, n, i);
            if (two) xi = axpy_term<A>(a0, load_il<A>(po, n, i), xi);
            store<A>(x, n, i, axpy_term<A>(ak, pi, xi));
        }
        if (!stop) {
            if constexpr (PC) store_il<A>(pn, n, i, axpy_term<A>(be, pi, jacobi<A>(dinv[i], rv)));
            else store_il<A>(pn, n, i, axpy_term<A>(be, normp ? normalise<A>(pi) : pi, rv));
        }
    }
}

// ------------------------------------------------------------ host side

struct CgLayout {
    size_t r, p, q, slots_a, slots_b, slots_c, dinv, state, plan, total;
    size_t plane;  // bytes of one vector (k planes of n, 256-aligned)
};

CgLayout cg_layout(int a, int32_t n, int32_t nnz)
{
    const size_t K = (size_t)words(a);
    const size_t plane = align256(sizeof(double) * (size_t)n * (size_t)vwords(a));
    const size_t nsl = (size_t)(spmv_max_slots(n) > UGRID_MAX ? spmv_max_slots(n) : UGRID_MAX);
    const size_t slots = align256(sizeof(double) * nsl * K);
    CgLayout L;
    L.r = 0;
    L.p = L.r + plane;  // xr(a) search-direction buffers
    L.q = L.p + (size_t)xr(a) * plane;
    L.slots_a = L.q + plane;
    L.slots_b = L.slots_a + slots;
    L.slots_c = L.slots_b + slots;  // Jacobi: the r^T r partials
    L.dinv = L.slots_c + slots;     // Jacobi: d_i = fl(1 / a_ii)
    L.state = L.dinv + align256(sizeof(double) * (size_t)n);
    L.plan = L.state + align256(sizeof(CgState));
    L.total = L.plan + plan_bytes(n, nnz);
    L.plane = plane;
    return L;
}

// Host copy of the integer part of CgState (from `run` on).
struct Flags {
    int32_t run[2], iters[2], brk[2], maxit, normalize, stopped, status, iters_final, normalize_p;
};

Flags *pinned_flags()
{
    thread_local Flags *buf = nullptr;
    if (!buf && hipHostMalloc((void **)&buf, sizeof(Flags), hipHostMallocDefault) != hipSuccess) buf = nullptr;
    return buf;
}


struct EventPool {
    hipEvent_t *e = nullptr;
    int n = 0;
    EventPool() = default;
    EventPool(const EventPool &) = delete;
    EventPool &operator=(const EventPool &) = delete;
    ~EventPool() { release(); }
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
};

constexpr int NKERN = 3;  // kernels per iteration
constexpr int KCLASS[NKERN] = {MW_PROF_SPMV, MW_PROF_UPDATE_R, MW_PROF_UPDATE_P};

// Everything one chunk of iterations needs.
struct ChunkArgs {
    int arith, n, nslots_sp, nslots_up, chunk, timed_mask, unt, ugrid;
    int pc;        // Jacobi preconditioner
    long pstride;  // doubles between the search-direction buffers
    const double *dinv;
    double *slots_c;
    const mw_csr_t *M;
    const mw_spmv_plan_t *plan;
    double *r, *p, *q, *x, *slots_a, *slots_b;
    CgState *st;
};

bool same_key(const ChunkArgs &a, const ChunkArgs &b)
{
    return a.arith == b.arith && a.n == b.n && a.pc == b.pc && a.dinv == b.dinv && a.slots_c == b.slots_c &&
           a.nslots_sp == b.nslots_sp && a.nslots_up == b.nslots_up &&
           a.chunk == b.chunk && a.pstride == b.pstride && a.timed_mask == b.timed_mask && a.unt == b.unt && a.ugrid == b.ugrid && a.r == b.r && a.p == b.p && a.q == b.q &&
           a.x == b.x && a.slots_a == b.slots_a && a.slots_b == b.slots_b && a.st == b.st && a.plan && b.plan &&
           a.plan->format == b.plan->format && a.plan->nslices == b.plan->nslices && a.plan->lanes == b.plan->lanes &&
           a.plan->slice_ptr == b.plan->slice_ptr && a.plan->col == b.plan->col && a.plan->val == b.plan->val &&
           a.plan->slot_off == b.plan->slot_off && a.plan->slot_mask == b.plan->slot_mask &&
           a.M->row_ptr == b.M->row_ptr && a.M->col_idx == b.M->col_idx && a.M->val == b.M->val &&
           a.M->n == b.M->n;
}

// Enqueues one chunk (even length, a multiple of xr(A), so chunks start
// after a multiple of it: iteration j of the chunk, 0-based, has parity
// (j + 1) & 1 and uses search-direction buffer j % xr(A)).  With a mask,
// the kernels of the timed classes carry a pair of events.
template <int A, int UNT, bool PC>
void launch_steps(const ChunkArgs &c, int k, int par, int kpos, hipStream_t s, hipEvent_t e0, hipEvent_t e1)
{
    const int gu = c.nslots_up;
    // consecutive kernels walk the rows in opposite directions
    if (k == 1)
        MW_LAUNCH((mw_cg_step_r_kernel<A, UNT, PC>), dim3(gu), dim3(UNT), s, e0, e1, c.n, c.nslots_sp, c.slots_a,
                  c.q, c.r, c.slots_b, c.st, par, kpos, par ^ 1, c.dinv, c.slots_c);
    else
        MW_LAUNCH((mw_cg_step_p_kernel<A, UNT, PC>), dim3(gu), dim3(UNT), s, e0, e1, c.n, c.nslots_up, c.slots_b,
                  c.r, c.p + kpos * c.pstride, xr(A) == 1 ? nullptr : c.p + ((kpos + 1) % xr(A)) * c.pstride, c.x,
                  c.st, par, kpos, par, c.slots_c, c.dinv);
}

template <int A, int UNT>
void launch_steps_pc(const ChunkArgs &c, int k, int par, int kpos, hipStream_t s, hipEvent_t e0, hipEvent_t e1)
{
    if (c.pc) launch_steps<A, UNT, true>(c, k, par, kpos, s, e0, e1);
    else launch_steps<A, UNT, false>(c, k, par, kpos, s, e0, e1);
}

template <int A>
int enqueue_chunk(const ChunkArgs &c, EventPool *ev, hipStream_t s)
{
    for (int it = 0; it < c.chunk; ++it) {
        const int par = (it + 1) & 1;
        const int kpos = it % xr(A);
        for (int k = 0; k < NKERN; ++k) {
            const bool timed = ev && (c.timed_mask & (1 << KCLASS[k]));
            hipEvent_t e0 = timed ? ev->e[(it * NKERN + k) * 2] : nullptr;
            hipEvent_t e1 = timed ? ev->e[(it * NKERN + k) * 2 + 1] : nullptr;
            if (k == 0) {
                const int rc = spmv_launch<A>(c.M, c.plan, c.p + kpos * c.pstride, c.q, c.slots_a, &c.st->run[par ^ 1],
                                              &c.st->run[par], 1, s, nullptr, par, e0, e1, c.nslots_sp);
                if (rc) return rc;
            } else if (c.unt == 1024) {
                launch_steps_pc<A, 1024>(c, k, par, kpos, s, e0, e1);
            } else if (c.unt == 512) {
                launch_steps_pc<A, 512>(c, k, par, kpos, s, e0, e1);
            } else {
                launch_steps_pc<A, 256>(c, k, par, kpos, s, e0, e1);
            }
        }
    }
    HIP_TRY(hipGetLastError());
    return MW_OK;
}

// A captured chunk, reused by later solves whose arguments (arithmetic,
// shape, every buffer and matrix pointer) all match.
struct GraphEntry {
    bool valid = false;
    unsigned long long used = 0;
    ChunkArgs key{};
    mw_csr_t M{};
    mw_spmv_plan_t plan{};
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    void release()
    {
        if (exec) (void)hipGraphExecDestroy(exec);
        if (graph) (void)hipGraphDestroy(graph);
        exec = nullptr;
        graph = nullptr;
        valid = false;
    }
};

// Up to NGRAPH captured chunks per thread (least recently used evicted),
// so a caller alternating between a few arithmetics, matrices or
// workspaces does not capture again on every solve.
struct GraphCache {
    static constexpr int NGRAPH = 8;
    GraphEntry e[NGRAPH];
    unsigned long long tick = 0;
    GraphEntry *find(const ChunkArgs &c)
    {
        for (GraphEntry &g : e)
            if (g.valid && same_key(g.key, c)) return &g;
        return nullptr;
    }
    GraphEntry *victim()
    {
        GraphEntry *v = &e[0];
        for (GraphEntry &g : e) {
            if (!g.valid) return &g;
            if (g.used < v->used) v = &g;
        }
        return v;
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
    double *sc = (double *)(base + L.slots_c);
    double *dinv = (double *)(base + L.dinv);
    CgState *st = (CgState *)(base + L.state);
    const bool pc = opts && opts->precond == MW_PRECOND_JACOBI;
    mw_cg_prof_t *prof = opts ? opts->prof : nullptr;
    const int mask = prof ? (prof->mask ? prof->mask : 0xF) : 0;
    // events recorded by graph nodes cannot be read back: timing uses direct launches
    const bool use_graph = !(opts && opts->no_graph) && !prof;

    hipStream_t s = thread_stream<0>();
    Flags *fl = pinned_flags();
    if (!s || !fl) return hip_fail(hipErrorOutOfMemory, "stream/pinned buffer");

    EventPool ev;
    SolveEvents se;
    if (const int erc = se.start(user, s)) return erc;

    // SpMV plan: given by the caller or chosen here (plan_auto; the lanes
    // of vector rows from the launch shape)
    const mw_shape_t *xshape = opts ? opts->shape : nullptr;
    mw_spmv_plan_t own_plan;
    const mw_spmv_plan_t *plan = opts ? opts->plan : nullptr;
    if (!plan) {
        const int lanes = cg_shape(A, n, M->nnz, 1, xshape, 0).lanes;
        const int rc = plan_auto(A, M, lanes, base + L.plan, L.total - L.plan, &own_plan, s);
        if (rc) return rc;
        plan = &own_plan;
    }

    CgState h;
    memset(&h, 0, sizeof(h));
    h.tol = tol;
    h.maxit = maxit;
    h.normalize = opts ? opts->normalize : 1;
    h.normalize_p = opts ? opts->normalize_p : 0;
    h.history = opts ? opts->history : nullptr;
    HIP_TRY(hipMemcpyAsync(st, &h, sizeof(CgState), hipMemcpyHostToDevice, s));

    const CgShape sh = cg_shape(A, n, M->nnz, spmv_tiles(plan), xshape, opts ? opts->chunk : 0);
    const int chunk = sh.chunk;
    const bool sell = plan->format == MW_FMT_SELL64, vec = plan->format == MW_FMT_CSRVEC;

    // r0 = b - A x0, p0 = r0, rho0, ||b||
    int rc = spmv_launch<A>(M, plan, x, q, nullptr, nullptr, nullptr, 0, s, nullptr, 0, nullptr, nullptr,
                            sell || vec ? sh.sgrid : 0);
    if (rc) return rc;
    const int gi = persistent_grid(blocks_for(n, NT));
    if (pc) {
        launch_jacobi_dinv(M, dinv, s);
        hipLaunchKernelGGL((mw_cg_init_kernel<A, true>), dim3(gi), dim3(NT), 0, s, n, b, q, r, p, sa, sb, dinv, sc);
        hipLaunchKernelGGL((mw_cg_init_final_kernel<A, true>), dim3(1), dim3(FIN_NT), 0, s, gi, sa, sb, sc, st);
    } else {
        hipLaunchKernelGGL((mw_cg_init_kernel<A, false>), dim3(gi), dim3(NT), 0, s, n, b, q, r, p, sa, sb, dinv, sc);
        hipLaunchKernelGGL((mw_cg_init_final_kernel<A, false>), dim3(1), dim3(FIN_NT), 0, s, gi, sa, sb, sc, st);
    }
    HIP_TRY(hipGetLastError());
    HIP_TRY(hipMemcpyAsync(fl, &st->run[0], sizeof(Flags), hipMemcpyDeviceToHost, s));
    HIP_TRY(hipStreamSynchronize(s));

    ChunkArgs c{};
    c.arith = A;
    c.n = n;
    c.chunk = chunk;
    c.pc = pc;
    c.dinv = dinv;
    c.slots_c = sc;
    c.pstride = (long)(L.plane / sizeof(double));
    c.timed_mask = mask;
    c.M = M;
    c.plan = plan;
    c.r = r;
    c.p = p;
    c.q = q;
    c.x = x;
    c.slots_a = sa;
    c.slots_b = sb;
    c.st = st;
    c.unt = sh.unt;
    c.ugrid = sh.ugrid;
    c.nslots_sp = sell || vec ? sh.sgrid : blocks_for(n, NT);
    c.nslots_up = sh.ugrid;

    hipGraphExec_t exec = nullptr;
    if (!fl->stopped) {
        if (use_graph) {
            GraphCache &GC = graph_cache();
            GraphEntry *G = GC.find(c);
            if (!G) {
                G = GC.victim();
                G->release();
                HIP_TRY(hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal));
                rc = enqueue_chunk<A>(c, nullptr, s);
                hipGraph_t g = nullptr;
                const hipError_t ce = hipStreamEndCapture(s, &g);
                if (rc) return rc;
                if (ce != hipSuccess) return hip_fail(ce, "hipStreamEndCapture");
                G->graph = g;
                HIP_TRY(hipGraphInstantiate(&G->exec, g, nullptr, nullptr, 0));
                G->key = c;
                G->M = *M;
                G->plan = *plan;
                G->key.M = &G->M;
                G->key.plan = &G->plan;
                G->valid = true;
            }
            G->used = ++GC.tick;
            exec = G->exec;
        } else if (mask) {
            if ((rc = ev.init(2 * NKERN * chunk))) return rc;
        }
    }

    int iters_before = 0;
    while (!fl->stopped) {
        if (use_graph) {
            HIP_TRY(hipGraphLaunch(exec, s));
        } else {
            rc = enqueue_chunk<A>(c, mask ? &ev : nullptr, s);
            if (rc) return rc;
        }
        HIP_TRY(hipMemcpyAsync(fl, &st->run[0], sizeof(Flags), hipMemcpyDeviceToHost, s));
        HIP_TRY(hipStreamSynchronize(s));
        const int now = fl->stopped ? fl->iters_final : (fl->iters[0] > fl->iters[1] ? fl->iters[0] : fl->iters[1]);
        if (mask) {
            // iterations of this chunk that ran to completion (the one that
            // stopped the solve is left out: part of its work was skipped)
            const int done = now - iters_before - (fl->stopped ? 1 : 0);
            for (int it = 0; it < done && it < chunk; ++it)
                for (int k = 0; k < NKERN; ++k) {
                    if (!(mask & (1 << KCLASS[k]))) continue;
                    float ms = 0.f;
                    HIP_TRY(hipEventElapsedTime(&ms, ev.e[(it * NKERN + k) * 2], ev.e[(it * NKERN + k) * 2 + 1]));
                    prof->ms[KCLASS[k]] += ms;
                    prof->launches[KCLASS[k]] += 1;
                }
        }
        iters_before = now;
    }
    HIP_TRY(hipMemcpyAsync(&h, st, sizeof(CgState), hipMemcpyDeviceToHost, s));
    HIP_TRY(hipEventRecord(se.t1, s));
    HIP_TRY(hipStreamSynchronize(s));
    float ms = 0.f;
    HIP_TRY(hipEventElapsedTime(&ms, se.t0, se.t1));
    if (info) {
        info->iters = h.iters_final;
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
    if (!valid_arith(a) || n <= 0 || !size_ok(n) || !size_ok(nnz)) return 0;
    return cg_layout(a, n, nnz).total;
}

int mw_cg_plan(mw_arith_t a, const mw_csr_t *A, int32_t lanes, void *buffer, size_t bytes, mw_spmv_plan_t *plan,
               void *stream)
{
    mwh::clear_error();
    if (!valid_arith(a) || !valid_csr(A) || !plan) return MW_EINVAL;
    if (lanes != 0 && !(lanes >= 2 && lanes <= 64 && (lanes & (lanes - 1)) == 0)) return MW_EINVAL;
    MW_CSR_GUARD(A, stream);
    const int l = lanes ? lanes : cg_shape(a, A->n, A->nnz, 1, nullptr, 0).lanes;
    return plan_auto(a, A, l, buffer, bytes, plan, (hipStream_t)stream);
}

int mw_cg_solve(mw_arith_t a, const mw_csr_t *A, const double *b, double *x, double tol, int32_t maxit,
                const mw_cg_opts_t *opts, void *workspace, mw_cg_info_t *info, void *stream)
{
    mwh::clear_error();
    if (!valid_arith(a) || !valid_csr(A) || !b || !x || !workspace || !(tol >= 0.0) || maxit < 0)
        return MW_EINVAL;
    if (opts && opts->plan && (!plan_valid(opts->plan) || opts->plan->n != A->n || opts->plan->csr.row_ptr != A->row_ptr))
        return MW_EINVAL;
    if (opts && (!shape_valid(opts->shape) || opts->normalize < 0)) return MW_EINVAL;
    if (opts && (opts->normalize_p < 0 || opts->normalize_p > 1 ||
                 (opts->normalize_p && opts->precond != MW_PRECOND_NONE))) {
        set_error("mw_cg_solve: normalize_p is 0 or 1, and applies to plain CG only");
        return MW_EINVAL;
    }
    if (opts && opts->precond != MW_PRECOND_NONE && opts->precond != MW_PRECOND_JACOBI) return MW_EINVAL;
    MW_CSR_GUARD(A, stream);
    MW_DISPATCH(a, cg_a, A, b, x, tol, maxit, opts, workspace, info, (hipStream_t)stream);
}

int mw_cg_tune(mw_arith_t a, const mw_csr_t *A, const double *b, double *x, int32_t iters, void *workspace,
               mw_shape_t *best, void *stream)
{
    mwh::clear_error();
    if (!valid_arith(a) || !valid_csr(A) || !b || !x || !workspace || !best || iters < 2 || iters > 4096)
        return MW_EINVAL;
    MW_CSR_GUARD(A, stream);
    const int n = A->n;
    const CgLayout L = cg_layout(a, n, A->nnz);
    hipStream_t s = (hipStream_t)stream;
    // the plan a solve would build (plan_auto); for vector rows also half
    // and twice its lanes per row
    const CgShape cur = cg_shape(a, n, A->nnz, 1, nullptr, 0);
    mw_spmv_plan_t plans[3];
    int rc = plan_auto(a, A, cur.lanes, (char *)workspace + L.plan, L.total - L.plan, &plans[0], s);
    if (rc) return rc;
    int np = 1;
    const int lanes0 = plans[0].format == MW_FMT_CSRVEC ? plans[0].lanes : 0;
    for (int l : {lanes0 / 2, lanes0 * 2})
        if (lanes0 && l >= 2 && l <= 64 && plan_rows(A, l, &plans[np]) == MW_OK) ++np;
    const bool gridded = plans[0].format == MW_FMT_SELL64 || plans[0].format == MW_FMT_CSRVEC;
    const int sgs[] = {1024, 1280, 1536, 1792, 2048};
    const int ugs[] = {512, 1024, 2048};
    // the shape a solve would use now; kept unless a candidate is more
    // than 1 % faster (candidates differ by little; noise must not decide)
    const CgShape builtin = cg_shape(a, n, A->nnz, spmv_tiles(&plans[0]), nullptr, 0);
    int seen[48][3];
    int nseen = 0;
    double best_t = 0.0, builtin_t = 0.0;
    mw_shape_t win{};
    const size_t xbytes = sizeof(double) * (size_t)mw_words(a) * (size_t)n;
    for (int ip = 0; ip < np; ++ip) {
        const mw_spmv_plan_t &plan = plans[ip];
        const int lanes = plan.format == MW_FMT_CSRVEC ? plan.lanes : 0;
        const int tiles = spmv_tiles(&plan);
        for (int sg : sgs) {
            for (int ug : ugs) {
                mw_shape_t cand{sg, ug, 256, iters + (iters & 1), lanes, 0.0};
                const CgShape eff = cg_shape(a, n, A->nnz, tiles, &cand, 0);
                const int key[3] = {gridded ? eff.sgrid : 0, eff.ugrid, lanes};
                bool dup = false;
                for (int i = 0; i < nseen; ++i)
                    dup = dup || (seen[i][0] == key[0] && seen[i][1] == key[1] && seen[i][2] == key[2]);
                if (dup) continue;
                for (int j = 0; j < 3; ++j) seen[nseen][j] = key[j];
                ++nseen;
                mw_cg_opts_t o{};
                o.normalize = 1;
                o.plan = &plan;
                o.shape = &cand;
                double t = 0.0;
                for (int rep = 0; rep < 4; ++rep) {  // the first run captures the chunk's graph
                    HIP_TRY(hipMemsetAsync(x, 0, xbytes, s));
                    mw_cg_info_t info{};
                    rc = mw_cg_solve(a, A, b, x, 0.0, iters, &o, workspace, &info, stream);
                    if (rc < 0) return rc;
                    if (info.iters < iters) {
                        set_error("mw_cg_tune: the iterations stopped early (b = 0 or breakdown)");
                        return MW_EINVAL;
                    }
                    if (rep == 1 || (rep > 1 && info.seconds < t)) t = info.seconds;
                }
                if (ip == 0 && key[0] == (gridded ? builtin.sgrid : 0) && key[1] == builtin.ugrid) builtin_t = t;
                if (best_t == 0.0 || t < best_t) {
                    best_t = t;
                    win = cand;
                    win.spmv_grid = key[0] > 0 ? key[0] : sg;
                    win.update_grid = key[1];
                }
            }
        }
    }
    if (builtin_t > 0.0 && best_t > builtin_t / 1.01) {
        win = mw_shape_t{builtin.sgrid, builtin.ugrid, builtin.unt, 0, lanes0, 0.0};
        best_t = builtin_t;
    }
    win.us_per_iteration = 1e6 * best_t / iters;
    win.chunk = 0;  // tuned shapes leave the chunk length to the solver
    tuned_put(a, n, A->nnz, 0, win);
    *best = win;
    return MW_OK;
}

}  // extern "C"
