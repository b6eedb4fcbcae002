// mw_batch.hip -- many independent SPD systems solved together (gfx950).
//
// Each system runs exactly the CG of Alg. 1 (with Sec. IV-C/IV-D), in the
// chosen arithmetic, with its own scalars, iteration count, stopping test
// and status.  The systems are the diagonal blocks of one block-diagonal
// CSR matrix; system s owns rows sys_row_off[s] .. sys_row_off[s+1]-1.
//
// Layout: a SELL-64 copy of the matrix whose slices never straddle two
// systems (each system's rows start a new slice), so every wavefront works
// for exactly one system; slices whose rows fit diagonal slots store no
// column indices, as in the single-system plan (fill_slice).  Slices with
// very uneven rows (the longest more than VEC_PAD times the average, so
// SELL-64 would pad every row to it) are not copied: they are summed as
// vector rows straight from the caller's CSR arrays, L lanes per row
// (vec_slice_sum), so one long row costs neither padding nor a single
// lane's sequential chain.  Per-system reductions use one partial per
// slice (a wavefront shuffle tree, no workgroup barrier), summed in slice
// order by one workgroup per system.
//
// One lockstep iteration of the whole batch is five kernels (six when there
// are vector-row slices), replayed from a captured hipGraph in chunks:
//   1. q = A p over the slices of running systems; p^T q per slice (the
//      vector-row slices in a kernel of their own right after)
//   2. one workgroup per running system: sigma, alpha = rho / sigma
//   3. r = r - alpha q, quasi normalisation, r^T r per slice
//   4. one workgroup per running system: rho', FP64 test, beta; a system
//      that stops here is masked out from now on
//   5. x = x + alpha p and p = r + beta p (x only for a system that
//      stopped in step 4 of this iteration)
// Converged systems cost only a flag test per slice.  The host polls the
// number of running systems once per chunk.  All orders are fixed, so the
// batch is run-to-run reproducible.  Jacobi preconditioning (PC) follows
// the single-system solver: z = D r with d_i = fl(1 / a_ii), rho = r^T z,
// the stopping test on r^T r, p = z + beta p.
#include "mw_blas.hpp"

#include <cstdlib>
#include <cstring>
#include <vector>

using namespace mwk;
using namespace mwh;

namespace {

// What the vector-row slices read, kept in device memory so that the
// slice kernels' arguments stay small.
struct VecRows {
    const int32_t *slanes;         // ns: lanes per row of a vector-row slice, 0 = SELL-64
    const int32_t *vlist;          // the vector-row slices (any order)
    const int32_t *nvec;           // their count
    const int32_t *crp, *cci;      // the caller's CSR
    const double *cva;
};

// Device view of the batch bookkeeping (passed by value).
struct BatchDev {
    const int32_t *sys_slice_off;  // nsys + 1
    const int32_t *slice_sys;      // ns
    const int32_t *slice_row0;     // ns
    const int32_t *slice_rows;     // ns (1..64)
    const int32_t *sp;             // SELL slice offsets, ns + 1
    const int32_t *sc;             // SELL columns (-1 = padding)
    const double *sv;              // SELL values
    const int32_t *soff;           // per slot of a diagonal slice: column offset
    const uint64_t *smask;         // per slot: rows that have an entry in it
    double *rho, *alpha, *beta;    // nsys * K each
    double *nb, *rel;              // nsys each
    int32_t *active, *xdue, *iters, *status;  // nsys each
    int32_t *n_active;             // running systems
    int32_t *alist;                // slices of the systems running at the start of
                                   // the current chunk (nullptr: every slice)
    int32_t *n_alist;              // their count
    int32_t *list_pos;             // nsys: a running system's first entry in alist
    const double *dinv;            // PC: fl(1 / a_ii) per row
    const struct VecRows *vec;     // vector-row slices (device memory)
    const double *tol;             // solve parameters in device memory
    const int32_t *maxit, *normalize;
    int nsys, ns, n;
};

constexpr int BNT = NT;  // workgroup of the slice kernels: NWAVE slices

__device__ __forceinline__ TileRange slice_tiles(int ns) { return xcd_tiles((ns + NWAVE - 1) / NWAVE); }

// The slices a slice kernel walks: the running systems' list, or all.
__device__ __forceinline__ int slice_count(const BatchDev &d) { return d.alist ? *d.n_alist : d.ns; }
__device__ __forceinline__ int slice_at(const BatchDev &d, int idx) { return d.alist ? d.alist[idx] : idx; }

// ------------------------------------------------------------ plan build

// A slice takes vector rows when its longest row is more than VEC_PAD
// times its average one and has at least VEC_MIN entries.  Uniform long
// rows keep SELL-64: on a batch of 96 banded systems (81 to 401 entries
// per row, 457 k rows) vector rows measured 12-36 % slower than its
// diagonal slots, which need no column indices.
constexpr int VEC_PAD = 4;
constexpr int VEC_MIN = 9;

// Lanes per row of a vector-row slice: the smallest power of two L with
// L x per >= max(average, longest / 8) (per: 8 entries a lane for FP64
// vectors, 16 for multi-word ones), at most 64; `lanes` > 0 overrides.
__device__ __forceinline__ int vec_lanes(int lanes, int vw, int avg, int longest)
{
    if (lanes > 0) return lanes;
    const int per = vw == 1 ? 8 : 16;
    const int target = max(avg, longest / 8);
    int L = 2;
    while (L < 64 && L * per < target) L *= 2;
    return L;
}

// Per slice: its SELL-64 width (longest row), or 0 and a lane count when
// it is to be summed as vector rows; those slices are appended to vlist
// (nvec counts them; every result is stored by slice index, so their
// order does not matter).
__global__ void __launch_bounds__(BNT) mw_batch_width_kernel(BatchDev d, const int32_t *__restrict__ row_ptr,
                                                             int32_t *__restrict__ width, int32_t *__restrict__ slanes,
                                                             int32_t *__restrict__ vlist, int32_t *__restrict__ nvec,
                                                             int lanes, int vw)
{
    const int s = blockIdx.x * NWAVE + wave_id();
    const int lane = threadIdx.x & 63;
    if (s >= d.ns) return;
    const int rows = d.slice_rows[s];
    int len = 0;
    if (lane < rows) {
        const int row = d.slice_row0[s] + lane;
        len = row_ptr[row + 1] - row_ptr[row];
    }
    int longest = len, total = len;
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) {
        longest = max(longest, __shfl_xor(longest, off, 64));
        total += __shfl_xor(total, off, 64);
    }
    const int avg = total / rows;
    const bool vec = longest >= VEC_MIN && (long)rows * longest > (long)VEC_PAD * total;
    if (lane == 0) {
        width[s] = vec ? 0 : longest;
        slanes[s] = vec ? vec_lanes(lanes, vw, avg, longest) : 0;
        if (vec) vlist[atomicAdd(nvec, 1)] = s;
    }
}

__global__ void __launch_bounds__(BNT) mw_batch_fill_kernel(BatchDev d, const int32_t *__restrict__ row_ptr,
                                                            const int32_t *__restrict__ col,
                                                            const double *__restrict__ val,
                                                            const int32_t *__restrict__ slice_ptr,
                                                            int32_t *__restrict__ scol, double *__restrict__ sval,
                                                            int32_t *__restrict__ soff, uint64_t *__restrict__ smask)
{
    const int s = blockIdx.x * NWAVE + wave_id();
    const int lane = threadIdx.x & 63;
    if (s >= d.ns || d.vec->slanes[s]) return;
    const int b = slice_ptr[s];
    const int w = (slice_ptr[s + 1] - b) / 64;
    const long row = (long)d.slice_row0[s] + lane;
    int rs = 0, len = 0;
    if (lane < d.slice_rows[s]) {
        rs = row_ptr[row];
        len = row_ptr[row + 1] - rs;
    }
    (void)fill_slice(b, w, lane, row, rs, len, col, val, scol, sval, soff, smask);
}

// ------------------------------------------------------------- kernels

// Row sums of a vector-row slice (rows row0 .. row0 + rows - 1, L lanes per
// row, L a power of two): L passes of 64 / L rows; lane t of a row's group
// adds the row's entries t, t + L, ... in order from zero, then the group
// combines its L sums by a fixed halving tree -- the row order of the
// single-system vector-row plan with the same L.  Each row's sum is stored
// by its group's first lane; in CG mode (MODE 1) that lane also adds
// x_i y_i to the returned per-lane partial.  Called by the whole wavefront.
template <int A, int MODE>
__device__ __forceinline__ Num<A> vec_slice_sum(const BatchDev &d, int L, long row0, int rows, int lane,
                                                const double *__restrict__ x, double *__restrict__ y)
{
    const int32_t *__restrict__ crp = d.vec->crp;
    const int32_t *__restrict__ cci = d.vec->cci;
    const double *__restrict__ cva = d.vec->cva;
    const int lg = __builtin_ctz(L);
    const int t = lane & (L - 1);
    const int rpw = 64 >> lg;
    Num<A> part = zero<A>();
    for (int k = 0; k < L; ++k) {
        const int rl = k * rpw + (lane >> lg);
        const long row = row0 + rl;
        Num<A> acc = zero<A>();
        if (rl < rows) {
            const int re = crp[row + 1];
            for (int j = crp[row] + t; j < re; j += L) acc = row_step<A>(acc, cva[j], load_v<A, MODE>(x, d.n, cci[j]));
        }
        for (int off = L >> 1; off > 0; off >>= 1) {
            const Num<A> o = shfl_down<A>(acc, off);
            if (t < off) acc = add<A>(acc, o);
        }
        if (t == 0 && rl < rows) {
            store<A>(y, d.n, row, acc);
            if constexpr (MODE == 1) part = dot_step<A>(part, load_v<A, MODE>(x, d.n, row), acc);
        }
    }
    return part;
}

// y = A x over the slices; MODE 1 (CG) skips stopped systems and leaves
// the slice partial of p^T q in slots[s].
template <int A, int MODE>
__global__ void __launch_bounds__(BNT) mw_batch_spmv_kernel(BatchDev d, const double *__restrict__ x,
                                                            double *__restrict__ y, double *__restrict__ slots)
{
    constexpr int K = words(A);
    const int lane = threadIdx.x & 63, wave = wave_id();
    const int nl = slice_count(d);
    const TileRange tr = slice_tiles(nl);
    for (int t = tr.first; t < tr.end; t += tr.step) {
        const int idx = t * NWAVE + wave;
        if (idx >= nl) continue;
        const int s = slice_at(d, idx);
        if constexpr (MODE == 1) {
            if (!d.active[d.slice_sys[s]]) continue;
        }
        const int b = d.sp[s];
        const int w = (d.sp[s + 1] - b) >> 6;
        // a vector-row slice stores nothing in the SELL-64 copy (w = 0):
        // mw_batch_vec_spmv_kernel sums it
        if (w == 0 && d.vec->slanes[s]) continue;
        const bool valid = lane < d.slice_rows[s];
        const long row = (long)d.slice_row0[s] + lane;
        Num<A> acc, xc = zero<A>();
        if (slice_is_diag(b, w, d.smask)) {
            if (valid) xc = load_v<A, MODE>(x, d.n, row);
            Num<A> xe = zero<A>();
            if constexpr (neighbour_moves<A>()) {
                const long re = lane == 0 ? row - 1 : row + 1;
                if ((lane == 0 || lane == 63) && re >= 0 && re < d.n) xe = load_v<A, MODE>(x, d.n, re);
            }
            acc = dia_row_sum<A, MODE, false>(b, w, lane, row, d.soff + (b >> 6), d.smask + (b >> 6), d.sv, x, d.n, xc,
                                              xe, nullptr);
        } else {
            acc = sell_row_sum<A, MODE>(b, w, lane, d.sc, d.sv, x, d.n);
            if (MODE == 1 && valid) xc = load_il<A>(x, d.n, row);
        }
        if (valid) store<A>(y, d.n, row, acc);
        if constexpr (MODE == 1) {
            Num<A> c = zero<A>();
            if (valid) c = dot_step<A>(c, xc, acc);
            c = wave_sum<A>(c);
            if (lane == 0) store_scalar<A>(slots + (long)s * K, c);
        }
    }
}

// The vector-row slices (vlist), one wavefront each, as the SELL kernel's
// MODE for the others: y and, in CG mode, the slice partial of p^T q.
template <int A, int MODE>
__global__ void __launch_bounds__(BNT) mw_batch_vec_spmv_kernel(BatchDev d, const double *__restrict__ x,
                                                                double *__restrict__ y, double *__restrict__ slots)
{
    constexpr int K = words(A);
    const int lane = threadIdx.x & 63;
    const int nv = *d.vec->nvec;
    const int step = gridDim.x * NWAVE;
    for (int idx = blockIdx.x * NWAVE + wave_id(); idx < nv; idx += step) {
        const int s = d.vec->vlist[idx];
        if constexpr (MODE == 1) {
            if (!d.active[d.slice_sys[s]]) continue;
        }
        const Num<A> part = vec_slice_sum<A, MODE>(d, d.vec->slanes[s], d.slice_row0[s], d.slice_rows[s], lane, x, y);
        if constexpr (MODE == 1) {
            const Num<A> c = wave_sum<A>(part);
            if (lane == 0) store_scalar<A>(slots + (long)s * K, c);
        }
    }
}

// r = b - q, p = r, slice partials of r^T r and b^T b.  PC: p = z = D r,
// slots_rr takes the partials of r^T z and slots_c those of r^T r.
template <int A, bool PC>
__global__ void __launch_bounds__(BNT) mw_batch_init_kernel(BatchDev d, const double *__restrict__ b,
                                                            const double *__restrict__ q, double *__restrict__ r,
                                                            double *__restrict__ p, double *__restrict__ slots_rr,
                                                            double *__restrict__ slots_bb, double *__restrict__ slots_c)
{
    constexpr int K = words(A);
    const int lane = threadIdx.x & 63, wave = wave_id();
    const int nl = slice_count(d);
    const TileRange tr = slice_tiles(nl);
    for (int t = tr.first; t < tr.end; t += tr.step) {
        const int idx = t * NWAVE + wave;
        if (idx >= nl) continue;
        const int s = slice_at(d, idx);
        Num<A> rr = zero<A>(), bb = zero<A>(), rz = zero<A>();
        if (lane < d.slice_rows[s]) {
            const long i = (long)d.slice_row0[s] + lane;
            const Num<A> bi = promote<A>(b[i]);
            Num<A> ri;
            if constexpr (A == FP64) ri = promote<A>(bi.w[0] - q[i]);
            else ri = add<A>(bi, neg<A>(load<A>(q, d.n, i)));
            store<A>(r, d.n, i, ri);
            if constexpr (PC) {
                const Num<A> zi = jacobi<A>(d.dinv[i], ri);
                store_il<A>(p, d.n, i, zi);
                rz = dot_step<A>(rz, ri, zi);
            } else {
                store_il<A>(p, d.n, i, ri);
            }
            rr = dot_step<A>(rr, ri, ri);
            bb = dot_step<A>(bb, bi, bi);
        }
        rr = wave_sum<A>(rr);
        bb = wave_sum<A>(bb);
        if constexpr (PC) rz = wave_sum<A>(rz);
        if (lane == 0) {
            store_scalar<A>(slots_rr + (long)s * K, PC ? rz : rr);
            store_scalar<A>(slots_bb + (long)s * K, bb);
            if constexpr (PC) store_scalar<A>(slots_c + (long)s * K, rr);
        }
    }
}

// Sum of a system's slice partials, slice order, by one workgroup.
template <int A>
__device__ __forceinline__ Num<A> system_sum(const BatchDev &d, int sys, const double *__restrict__ slots)
{
    constexpr int K = words(A);
    const int s0 = d.sys_slice_off[sys], s1 = d.sys_slice_off[sys + 1];
    return reduce_slots<A, BNT>(s1 - s0, slots + (long)s0 * K);
}

template <int A, bool PC>
__global__ void __launch_bounds__(BNT) mw_batch_init_final_kernel(BatchDev d, const double *__restrict__ slots_rr,
                                                                  const double *__restrict__ slots_bb,
                                                                  const double *__restrict__ slots_c)
{
    constexpr int K = words(A);
    const int sys = blockIdx.x;
    const Num<A> rho = system_sum<A>(d, sys, slots_rr);
    const Num<A> bb = system_sum<A>(d, sys, slots_bb);
    Num<A> rr = rho;
    if constexpr (PC) rr = system_sum<A>(d, sys, slots_c);
    if (threadIdx.x == 0) {
        store_scalar<A>(d.rho + (long)sys * K, rho);
        d.nb[sys] = sqrt(to_fp64<A>(bb));
        d.iters[sys] = 0;
        d.xdue[sys] = 0;
        const double r64 = to_fp64<A>(rr);
        int run = 1, status = MW_OK;
        if (r64 == 0.0) {
            d.rel[sys] = 0.0;
            run = 0;
        } else {
            d.rel[sys] = sqrt(r64) / d.nb[sys];
            if (*d.maxit == 0) {
                status = MW_NOT_CONVERGED;
                run = 0;
            }
        }
        d.status[sys] = status;
        d.active[sys] = run;
        if (run) atomicAdd(d.n_active, 1);
    }
}

// alpha per running system; a stopped system drops its pending x flag.
template <int A>
__global__ void __launch_bounds__(BNT) mw_batch_alpha_kernel(BatchDev d, const double *__restrict__ slots)
{
    constexpr int K = words(A);
    const int sys = blockIdx.x;
    if (!d.active[sys]) {
        if (threadIdx.x == 0) d.xdue[sys] = 0;
        return;
    }
    const Num<A> sigma = system_sum<A>(d, sys, slots);
    if (threadIdx.x == 0) {
        const double s64 = to_fp64<A>(sigma);
        bool brk = !(s64 > 0.0) || !isfinite(s64);
        Num<A> al = zero<A>();
        if (!brk) {
            al = div<A>(load_scalar<A>(d.rho + (long)sys * K), sigma);
            brk = !isfinite(to_fp64<A>(al));
        }
        if (brk) {
            d.status[sys] = MW_BREAKDOWN;
            d.active[sys] = 0;
            atomicSub(d.n_active, 1);
        } else {
            store_scalar<A>(d.alpha + (long)sys * K, al);
        }
    }
}

// r = r - alpha q (quasi types normalise it), slice partials of r^T r
// (PC: of r^T z to slots, of r^T r to slots_c).
template <int A, bool PC>
__global__ void __launch_bounds__(BNT) mw_batch_step_r_kernel(BatchDev d, const double *__restrict__ q,
                                                              double *__restrict__ r, double *__restrict__ slots,
                                                              double *__restrict__ slots_c)
{
    constexpr int K = words(A);
    const int lane = threadIdx.x & 63, wave = wave_id();
    // quasi types: normalise in iterations NK, 2 NK, ... of each system
    const int NK = *d.normalize;
    const int nl = slice_count(d);
    const TileRange tr = slice_tiles(nl);
    for (int t = tr.first; t < tr.end; t += tr.step) {
        const int idx = t * NWAVE + wave;
        if (idx >= nl) continue;
        const int s = slice_at(d, idx);
        const int sys = d.slice_sys[s];
        if (!d.active[sys]) continue;
        const bool norm = is_quasi(A) && NK > 0 && (d.iters[sys] + 1) % NK == 0;
        const Num<A> al = load_scalar<A>(d.alpha + (long)sys * K);
        Num<A> rr = zero<A>(), rz = zero<A>();
        if (lane < d.slice_rows[s]) {
            const long i = (long)d.slice_row0[s] + lane;
            Num<A> ri = axmy_term<A>(al, load<A>(q, d.n, i), load<A>(r, d.n, i));
            if (norm) ri = normalise<A>(ri);
            store<A>(r, d.n, i, ri);
            if constexpr (PC) rz = dot_step<A>(rz, ri, jacobi<A>(d.dinv[i], ri));
            rr = dot_step<A>(rr, ri, ri);
        }
        rr = wave_sum<A>(rr);
        if constexpr (PC) rz = wave_sum<A>(rz);
        if (lane == 0) {
            store_scalar<A>(slots + (long)s * K, PC ? rz : rr);
            if constexpr (PC) store_scalar<A>(slots_c + (long)s * K, rr);
        }
    }
}

// rho', the FP64 test (on r^T r) and beta per running system.
template <int A, bool PC>
__global__ void __launch_bounds__(BNT) mw_batch_beta_kernel(BatchDev d, const double *__restrict__ slots,
                                                            const double *__restrict__ slots_c)
{
    constexpr int K = words(A);
    const int sys = blockIdx.x;
    if (!d.active[sys]) return;
    const Num<A> rho_new = system_sum<A>(d, sys, slots);
    Num<A> rr_new = rho_new;
    if constexpr (PC) rr_new = system_sum<A>(d, sys, slots_c);
    if (threadIdx.x == 0) {
        const int it = d.iters[sys] + 1;
        d.iters[sys] = it;
        const double rr = to_fp64<A>(rr_new);
        const bool fin = isfinite(rr) && (!PC || isfinite(to_fp64<A>(rho_new)));
        const double rel = fin ? sqrt(rr) / d.nb[sys] : rr;
        const bool conv = fin && rel < *d.tol;
        if (fin) d.rel[sys] = rel;
        if (!fin || conv || it >= *d.maxit) {
            d.status[sys] = !fin ? MW_BREAKDOWN : (conv ? MW_OK : MW_NOT_CONVERGED);
            d.active[sys] = 0;
            d.xdue[sys] = 1;
            atomicSub(d.n_active, 1);
        } else {
            store_scalar<A>(d.beta + (long)sys * K, div<A>(rho_new, load_scalar<A>(d.rho + (long)sys * K)));
            store_scalar<A>(d.rho + (long)sys * K, rho_new);
        }
    }
}

// x = x + alpha p; p = r + beta p (PC: z + beta p, z = D r).
template <int A, bool PC>
__global__ void __launch_bounds__(BNT) mw_batch_step_p_kernel(BatchDev d, const double *__restrict__ r,
                                                              double *__restrict__ p, double *__restrict__ x)
{
    constexpr int K = words(A);
    const int lane = threadIdx.x & 63, wave = wave_id();
    const int nl = slice_count(d);
    const TileRange tr = slice_tiles(nl);
    for (int t = tr.first; t < tr.end; t += tr.step) {
        const int idx = t * NWAVE + wave;
        if (idx >= nl) continue;
        const int s = slice_at(d, idx);
        const int sys = d.slice_sys[s];
        const bool run = d.active[sys];
        if (!run && !d.xdue[sys]) continue;
        if (lane >= d.slice_rows[s]) continue;
        const long i = (long)d.slice_row0[s] + lane;
        const Num<A> al = load_scalar<A>(d.alpha + (long)sys * K);
        const Num<A> pi = load_il<A>(p, d.n, i);
        store<A>(x, d.n, i, axpy_term<A>(al, pi, load<A>(x, d.n, i)));
        if (run) {
            const Num<A> be = load_scalar<A>(d.beta + (long)sys * K);
            const Num<A> ri = load<A>(r, d.n, i);
            if constexpr (PC) store_il<A>(p, d.n, i, axpy_term<A>(be, pi, jacobi<A>(d.dinv[i], ri)));
            else store_il<A>(p, d.n, i, axpy_term<A>(be, pi, ri));
        }
    }
}

// The running systems' slices, rebuilt at the start of every chunk so the
// slice kernels of a batch's tail walk only those.  Every per-slice result
// is stored by slice index, so the list order does not change results; it
// is kept ascending so that the workgroups of an XCD, which take
// consecutive list entries, work on one or two systems at a time and
// their gathers of p stay in that XCD's L2 (with the list in arbitrary
// 64-slice runs, the QTW batch SpMV fetched 1.6x its algorithmic bytes).
// Step 1, one workgroup: each running system's first list position (an
// exclusive scan of the running systems' slice counts in system order)
// and the list length.
__global__ void __launch_bounds__(BNT) mw_batch_list_scan_kernel(BatchDev d)
{
    __shared__ int part[BNT];
    const int t = threadIdx.x;
    const int per = (d.nsys + BNT - 1) / BNT;
    const int s0 = t * per, s1 = min(s0 + per, d.nsys);
    int sum = 0;
    for (int s = s0; s < s1; ++s)
        if (d.active[s]) sum += d.sys_slice_off[s + 1] - d.sys_slice_off[s];
    part[t] = sum;
    __syncthreads();
    if (t == 0) {
        int acc = 0;
        for (int u = 0; u < BNT; ++u) {
            const int v = part[u];
            part[u] = acc;
            acc += v;
        }
        *d.n_alist = acc;
    }
    __syncthreads();
    int pos = part[t];
    for (int s = s0; s < s1; ++s) {
        d.list_pos[s] = pos;
        if (d.active[s]) pos += d.sys_slice_off[s + 1] - d.sys_slice_off[s];
    }
}

// Step 2, one workgroup per system: a running system's slices, in order.
__global__ void __launch_bounds__(BNT) mw_batch_list_fill_kernel(BatchDev d)
{
    const int sys = blockIdx.x;
    if (!d.active[sys]) return;
    const int first = d.sys_slice_off[sys], cnt = d.sys_slice_off[sys + 1] - first, pos = d.list_pos[sys];
    for (int k = threadIdx.x; k < cnt; k += BNT) d.alist[pos + k] = first + k;
}

// ------------------------------------------------------------ host side

struct BatchLayout {
    size_t r, p, q, slots_a, slots_b, slots_c, dinv, sys_slice_off, slice_sys, slice_row0, slice_rows, dscal, iscal, params, width,
        slice_ptr, total, alist, n_alist, list_pos, slanes, vlist, vecrows, soff, smask, col, val, bytes;
    long long ns_max, cap;
};

BatchLayout batch_layout(int a, int32_t nsys, int32_t n, int32_t nnz)
{
    const size_t K = (size_t)words(a), KV = (size_t)vwords(a);  // scalar / vector words
    BatchLayout L;
    L.ns_max = ((long long)n + 63) / 64 + nsys;
    L.cap = (long long)nnz + (long long)nnz / 4 + 64 * L.ns_max;
    size_t o = 0;
    auto take = [&](size_t bytes) {
        const size_t at = o;
        o += align256(bytes);
        return at;
    };
    L.r = take(sizeof(double) * KV * n);
    L.p = take(sizeof(double) * KV * n);
    L.q = take(sizeof(double) * KV * n);
    L.slots_a = take(sizeof(double) * K * L.ns_max);
    L.slots_b = take(sizeof(double) * K * L.ns_max);
    L.slots_c = take(sizeof(double) * K * L.ns_max);
    L.dinv = take(sizeof(double) * n);
    L.sys_slice_off = take(sizeof(int32_t) * (nsys + 1));
    L.slice_sys = take(sizeof(int32_t) * L.ns_max);
    L.slice_row0 = take(sizeof(int32_t) * L.ns_max);
    L.slice_rows = take(sizeof(int32_t) * L.ns_max);
    L.dscal = take(sizeof(double) * (3 * K + 2) * nsys);
    L.iscal = take(sizeof(int32_t) * (4 * nsys + 1));
    L.params = take(64);
    L.width = take(sizeof(int32_t) * L.ns_max);
    L.slice_ptr = take(sizeof(int32_t) * (L.ns_max + 1));
    L.total = take(2 * sizeof(long long));  // stored entries; vector-row slices
    L.alist = take(sizeof(int32_t) * L.ns_max);
    L.n_alist = take(sizeof(int32_t));
    L.list_pos = take(sizeof(int32_t) * nsys);
    L.slanes = take(sizeof(int32_t) * L.ns_max);
    L.vlist = take(sizeof(int32_t) * L.ns_max);
    L.vecrows = take(sizeof(VecRows));
    L.soff = take(sizeof(int32_t) * (L.cap / 64 + 8));
    L.smask = take(sizeof(uint64_t) * (L.cap / 64 + 8));
    L.col = take(sizeof(int32_t) * L.cap);
    L.val = take(sizeof(double) * L.cap);
    L.bytes = o;
    return L;
}

struct BatchParams {
    double tol;
    int32_t maxit, normalize;
};

// Vector-row slices of the calling thread's last batched solve (read by
// the tuner to decide whether lanes per row is worth sweeping).
thread_local int g_last_vec_slices = 0;

int32_t *pinned_count()
{
    thread_local int32_t *buf = nullptr;
    if (!buf && hipHostMalloc((void **)&buf, 64, hipHostMallocDefault) != hipSuccess) buf = nullptr;
    return buf;
}

// What a captured chunk depends on: the sizes that place the workspace's
// arrays (batch_layout: n, nnz and nsys move the slice copy's offsets) and
// every pointer its kernels take, the BatchDev fields included.
struct BatchKey {
    int arith, nsys, ns, n, nnz, chunk, grid, pc, vgrid;
    static constexpr int NPTR = 17;
    const void *ptrs[NPTR];
    bool operator==(const BatchKey &o) const
    {
        if (arith != o.arith || nsys != o.nsys || ns != o.ns || n != o.n || nnz != o.nnz || chunk != o.chunk ||
            grid != o.grid || pc != o.pc || vgrid != o.vgrid)
            return false;
        for (int i = 0; i < NPTR; ++i)
            if (ptrs[i] != o.ptrs[i]) return false;
        return true;
    }
};

struct BatchGraph {
    bool valid = false;
    BatchKey key{};
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

// Heap-allocated and never freed (no HIP call during process teardown).
BatchGraph &batch_graph()
{
    thread_local BatchGraph *g = new BatchGraph();
    return *g;
}

template <int A, bool PC>
int enqueue_batch_chunk(const BatchDev &d, int chunk, int g, int vg, double *r, double *p, double *q, double *x,
                        double *sa, double *sb, double *sc, hipStream_t s)
{
    hipLaunchKernelGGL(mw_batch_list_scan_kernel, dim3(1), dim3(BNT), 0, s, d);
    hipLaunchKernelGGL(mw_batch_list_fill_kernel, dim3(d.nsys), dim3(BNT), 0, s, d);
    for (int it = 0; it < chunk; ++it) {
        hipLaunchKernelGGL((mw_batch_spmv_kernel<A, 1>), dim3(g), dim3(BNT), 0, s, d, p, q, sa);
        if (vg > 0) hipLaunchKernelGGL((mw_batch_vec_spmv_kernel<A, 1>), dim3(vg), dim3(BNT), 0, s, d, p, q, sa);
        hipLaunchKernelGGL((mw_batch_alpha_kernel<A>), dim3(d.nsys), dim3(BNT), 0, s, d, sa);
        hipLaunchKernelGGL((mw_batch_step_r_kernel<A, PC>), dim3(g), dim3(BNT), 0, s, d, q, r, sb, sc);
        hipLaunchKernelGGL((mw_batch_beta_kernel<A, PC>), dim3(d.nsys), dim3(BNT), 0, s, d, sb, sc);
        hipLaunchKernelGGL((mw_batch_step_p_kernel<A, PC>), dim3(g), dim3(BNT), 0, s, d, r, p, x);
    }
    HIP_TRY(hipGetLastError());
    return MW_OK;
}

template <int A>
int enqueue_batch_chunk_pc(bool pc, const BatchDev &d, int chunk, int g, int vg, double *r, double *p, double *q,
                           double *x, double *sa, double *sb, double *sc, hipStream_t s)
{
    return pc ? enqueue_batch_chunk<A, true>(d, chunk, g, vg, r, p, q, x, sa, sb, sc, s)
              : enqueue_batch_chunk<A, false>(d, chunk, g, vg, r, p, q, x, sa, sb, sc, s);
}

template <int A>
int batched_a(int32_t nsys, const int32_t *off, const mw_csr_t *M, const double *b, double *x, double tol,
              int32_t maxit, const mw_cg_opts_t *opts, void *ws, int32_t *iters_out, int32_t *status_out,
              double *rel_out, mw_cg_info_t *info, hipStream_t user)
{
    constexpr int K = words(A);
    const int n = M->n;
    const BatchLayout L = batch_layout(A, nsys, n, M->nnz);
    char *base = (char *)ws;
    const bool use_graph = !(opts && opts->no_graph);
    const bool pc = opts && opts->precond == MW_PRECOND_JACOBI;

    // slices: each system starts a new 64-row slice
    std::vector<int32_t> h_sso(nsys + 1), h_sys, h_row0, h_rows;
    h_sys.reserve(L.ns_max);
    h_row0.reserve(L.ns_max);
    h_rows.reserve(L.ns_max);
    for (int s = 0; s < nsys; ++s) {
        h_sso[s] = (int32_t)h_sys.size();
        for (int r0 = off[s]; r0 < off[s + 1]; r0 += 64) {
            h_sys.push_back(s);
            h_row0.push_back(r0);
            h_rows.push_back(off[s + 1] - r0 < 64 ? off[s + 1] - r0 : 64);
        }
    }
    h_sso[nsys] = (int32_t)h_sys.size();
    const int ns = (int)h_sys.size();
    const BatchShape bsh = batch_shape(A, n, M->nnz, nsys, ns, opts ? opts->shape : nullptr, opts ? opts->chunk : 0);
    const int chunk = bsh.chunk;

    hipStream_t s = thread_stream<1>();
    int32_t *hcount = pinned_count();
    if (!s || !hcount) return hip_fail(hipErrorOutOfMemory, "stream/pinned buffer");
    SolveEvents se;
    if (const int erc = se.start(user, s)) return erc;

    BatchDev d{};
    d.sys_slice_off = (int32_t *)(base + L.sys_slice_off);
    d.slice_sys = (int32_t *)(base + L.slice_sys);
    d.slice_row0 = (int32_t *)(base + L.slice_row0);
    d.slice_rows = (int32_t *)(base + L.slice_rows);
    d.sp = (int32_t *)(base + L.slice_ptr);
    d.sc = (int32_t *)(base + L.col);
    d.sv = (double *)(base + L.val);
    d.alist = nullptr;  // set for the iteration chunks, after the set-up kernels
    d.n_alist = (int32_t *)(base + L.n_alist);
    d.list_pos = (int32_t *)(base + L.list_pos);
    int32_t *slanes = (int32_t *)(base + L.slanes);
    int32_t *vlist = (int32_t *)(base + L.vlist);
    VecRows *vecrows = (VecRows *)(base + L.vecrows);
    d.vec = vecrows;
    d.soff = (int32_t *)(base + L.soff);
    d.smask = (uint64_t *)(base + L.smask);
    double *dscal = (double *)(base + L.dscal);
    d.rho = dscal;
    d.alpha = d.rho + (size_t)K * nsys;
    d.beta = d.alpha + (size_t)K * nsys;
    d.nb = d.beta + (size_t)K * nsys;
    d.rel = d.nb + nsys;
    int32_t *iscal = (int32_t *)(base + L.iscal);
    d.active = iscal;
    d.xdue = iscal + nsys;
    d.iters = iscal + 2 * nsys;
    d.status = iscal + 3 * nsys;
    d.n_active = iscal + 4 * nsys;
    BatchParams *prm = (BatchParams *)(base + L.params);
    d.tol = &prm->tol;
    d.maxit = &prm->maxit;
    d.normalize = &prm->normalize;
    d.dinv = (const double *)(base + L.dinv);
    d.nsys = nsys;
    d.ns = ns;
    d.n = n;
    double *r = (double *)(base + L.r);
    double *p = (double *)(base + L.p);
    double *q = (double *)(base + L.q);
    double *sa = (double *)(base + L.slots_a);
    double *sb = (double *)(base + L.slots_b);
    double *sc = (double *)(base + L.slots_c);
    int32_t *width = (int32_t *)(base + L.width);
    long long *total = (long long *)(base + L.total);

    const BatchParams hp{tol, maxit, opts ? opts->normalize : 1};
    HIP_TRY(hipMemcpyAsync(prm, &hp, sizeof(hp), hipMemcpyHostToDevice, s));
    HIP_TRY(hipMemcpyAsync((void *)d.sys_slice_off, h_sso.data(), sizeof(int32_t) * (nsys + 1),
                           hipMemcpyHostToDevice, s));
    if (ns > 0) {
        HIP_TRY(hipMemcpyAsync((void *)d.slice_sys, h_sys.data(), sizeof(int32_t) * ns, hipMemcpyHostToDevice, s));
        HIP_TRY(hipMemcpyAsync((void *)d.slice_row0, h_row0.data(), sizeof(int32_t) * ns, hipMemcpyHostToDevice, s));
        HIP_TRY(hipMemcpyAsync((void *)d.slice_rows, h_rows.data(), sizeof(int32_t) * ns, hipMemcpyHostToDevice, s));
    }
    // system-aligned SELL-64 plan
    const int nbw = blocks_for(ns > 0 ? ns : 1, NWAVE);
    int32_t *nvec = (int32_t *)(total + 1);
    // (the record is read by the kernels below, on this stream; the host
    // copy lives until the synchronisation after the scan)
    const VecRows h_vec{slanes, vlist, nvec, M->row_ptr, M->col_idx, M->val};
    HIP_TRY(hipMemsetAsync(nvec, 0, sizeof(int32_t), s));
    HIP_TRY(hipMemcpyAsync(vecrows, &h_vec, sizeof(VecRows), hipMemcpyHostToDevice, s));
    hipLaunchKernelGGL(mw_batch_width_kernel, dim3(nbw), dim3(BNT), 0, s, d, M->row_ptr, width, slanes, vlist, nvec,
                       bsh.lanes, vwords(A));
    HIP_TRY(hipGetLastError());
    int rc = launch_sell_scan(ns, width, (int32_t *)d.sp, total, s);
    if (rc) return rc;
    HIP_TRY(hipMemcpyAsync(hcount, total, 2 * sizeof(long long), hipMemcpyDeviceToHost, s));
    HIP_TRY(hipStreamSynchronize(s));  // also retires the host-array uploads above
    const long long stored = *(long long *)hcount;
    g_last_vec_slices = *(int32_t *)((long long *)hcount + 1);
    // grid of the vector-row slice kernel: one wavefront per slice, at most
    // a persistent grid's worth (0: no such slices, no launch)
    const int vg = g_last_vec_slices > 0 ? persistent_grid(blocks_for(g_last_vec_slices, NWAVE)) : 0;
    if (stored > L.cap || stored > 0x7fffffffLL) {
        set_error("batched solve: SELL-64 padding exceeds the workspace (rows of very uneven length)");
        return MW_EINVAL;
    }
    hipLaunchKernelGGL(mw_batch_fill_kernel, dim3(nbw), dim3(BNT), 0, s, d, M->row_ptr, M->col_idx, M->val, d.sp,
                       (int32_t *)d.sc, (double *)d.sv, (int32_t *)d.soff, (uint64_t *)d.smask);
    HIP_TRY(hipGetLastError());

    // r0 = b - A x0, p0 = r0, per-system rho0, ||b||, flags
    const int g = bsh.grid;
    HIP_TRY(hipMemsetAsync(d.n_active, 0, sizeof(int32_t), s));
    hipLaunchKernelGGL((mw_batch_spmv_kernel<A, 0>), dim3(g), dim3(BNT), 0, s, d, x, q, sa);
    if (vg > 0) hipLaunchKernelGGL((mw_batch_vec_spmv_kernel<A, 0>), dim3(vg), dim3(BNT), 0, s, d, x, q, sa);
    if (pc) {
        launch_jacobi_dinv(M, (double *)d.dinv, s);
        hipLaunchKernelGGL((mw_batch_init_kernel<A, true>), dim3(g), dim3(BNT), 0, s, d, b, q, r, p, sa, sb, sc);
        hipLaunchKernelGGL((mw_batch_init_final_kernel<A, true>), dim3(nsys), dim3(BNT), 0, s, d, sa, sb, sc);
    } else {
        hipLaunchKernelGGL((mw_batch_init_kernel<A, false>), dim3(g), dim3(BNT), 0, s, d, b, q, r, p, sa, sb, sc);
        hipLaunchKernelGGL((mw_batch_init_final_kernel<A, false>), dim3(nsys), dim3(BNT), 0, s, d, sa, sb, sc);
    }
    HIP_TRY(hipGetLastError());
    HIP_TRY(hipMemcpyAsync(hcount, d.n_active, sizeof(int32_t), hipMemcpyDeviceToHost, s));
    HIP_TRY(hipStreamSynchronize(s));

    d.alist = (int32_t *)(base + L.alist);
    int chunks = 0;
    if (*hcount > 0 && use_graph) {
        BatchGraph &G = batch_graph();
        BatchKey key{A, nsys, ns, n, M->nnz, chunk, g, pc ? 1 : 0, vg,
                     {r, p, q, x, sa, sb, sc, base, d.sp, d.sc, d.sv, d.soff, d.smask, d.dinv, M->row_ptr, M->col_idx,
                      M->val}};
        if (!(G.valid && G.key == key)) {
            G.release();
            HIP_TRY(hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal));
            rc = enqueue_batch_chunk_pc<A>(pc, d, chunk, g, vg, r, p, q, x, sa, sb, sc, s);
            hipGraph_t gr = nullptr;
            const hipError_t ce = hipStreamEndCapture(s, &gr);
            if (rc) return rc;
            if (ce != hipSuccess) return hip_fail(ce, "hipStreamEndCapture");
            G.graph = gr;
            HIP_TRY(hipGraphInstantiate(&G.exec, gr, nullptr, nullptr, 0));
            G.key = key;
            G.valid = true;
        }
    }
    while (*hcount > 0) {
        if (use_graph) {
            HIP_TRY(hipGraphLaunch(batch_graph().exec, s));
        } else {
            rc = enqueue_batch_chunk_pc<A>(pc, d, chunk, g, vg, r, p, q, x, sa, sb, sc, s);
            if (rc) return rc;
        }
        ++chunks;
        HIP_TRY(hipMemcpyAsync(hcount, d.n_active, sizeof(int32_t), hipMemcpyDeviceToHost, s));
        HIP_TRY(hipStreamSynchronize(s));
    }
    // (a system that stops in step 4 gets its last x update in step 5 of the
    // same iteration; step 2 of the next iteration clears its pending flag)
    if (iters_out) HIP_TRY(hipMemcpyAsync(iters_out, d.iters, sizeof(int32_t) * nsys, hipMemcpyDeviceToDevice, s));
    if (status_out) HIP_TRY(hipMemcpyAsync(status_out, d.status, sizeof(int32_t) * nsys, hipMemcpyDeviceToDevice, s));
    if (rel_out) HIP_TRY(hipMemcpyAsync(rel_out, d.rel, sizeof(double) * nsys, hipMemcpyDeviceToDevice, s));
    std::vector<int32_t> hi(2 * (size_t)nsys);
    HIP_TRY(hipMemcpyAsync(hi.data(), d.iters, sizeof(int32_t) * 2 * nsys, hipMemcpyDeviceToHost, s));
    HIP_TRY(hipEventRecord(se.t1, s));
    HIP_TRY(hipStreamSynchronize(s));
    float ms = 0.f;
    HIP_TRY(hipEventElapsedTime(&ms, se.t0, se.t1));
    int worst = MW_OK, maxit_seen = 0;
    for (int i = 0; i < nsys; ++i) {
        if (hi[i] > maxit_seen) maxit_seen = hi[i];
        if (hi[nsys + i] > worst) worst = hi[nsys + i];
    }
    if (info) {
        info->iters = maxit_seen;
        info->status = worst;
        info->rel_res = 0.0;
        info->seconds = ms * 1e-3;
    }
    (void)chunks;
    return worst;
}

}  // namespace

// ================================================================== C ABI

extern "C" {

size_t mw_cg_batched_workspace_bytes(mw_arith_t a, int32_t nsys, int32_t n, int32_t nnz)
{
    if (!valid_arith(a) || nsys <= 0 || n <= 0 || !size_ok(n) || !size_ok(nnz)) return 0;
    return batch_layout(a, nsys, n, nnz).bytes;
}

}  // extern "C"

namespace {

bool batched_args_ok(int a, int32_t nsys, const int32_t *sys_row_off, const mw_csr_t *A, const double *b,
                     const double *x, const void *workspace)
{
    if (!valid_arith(a) || nsys <= 0 || !sys_row_off || !valid_csr(A) || !b || !x || !workspace) return false;
    if (sys_row_off[0] != 0 || sys_row_off[nsys] != A->n) return false;
    for (int s = 0; s < nsys; ++s)
        if (sys_row_off[s + 1] < sys_row_off[s]) return false;
    return true;
}

}  // namespace

extern "C" {

int mw_cg_solve_batched(mw_arith_t a, int32_t nsys, const int32_t *sys_row_off, const mw_csr_t *A, const double *b,
                        double *x, double tol, int32_t maxit, const mw_cg_opts_t *opts, void *workspace,
                        int32_t *iters, int32_t *status, double *rel_res, mw_cg_info_t *info, void *stream)
{
    mwh::clear_error();
    if (!batched_args_ok(a, nsys, sys_row_off, A, b, x, workspace) || !(tol >= 0.0) || maxit < 0) return MW_EINVAL;
    if (opts && (!shape_valid(opts->shape) || opts->normalize < 0 || opts->normalize_p != 0 ||
                 (opts->precond != MW_PRECOND_NONE && opts->precond != MW_PRECOND_JACOBI)))
        return MW_EINVAL;
    MW_CSR_GUARD(A, stream);
    MW_DISPATCH(a, batched_a, nsys, sys_row_off, A, b, x, tol, maxit, opts, workspace, iters, status, rel_res, info,
                (hipStream_t)stream);
}

int mw_cg_batched_tune(mw_arith_t a, int32_t nsys, const int32_t *sys_row_off, const mw_csr_t *A,
                       const double *b, double *x, int32_t iters, void *workspace, mw_shape_t *best, void *stream)
{
    mwh::clear_error();
    if (!best || iters < 2 || iters > 4096 || !batched_args_ok(a, nsys, sys_row_off, A, b, x, workspace))
        return MW_EINVAL;
    const int grids[] = {256, 512, 1024, 1536, 2048};
    const size_t xbytes = sizeof(double) * (size_t)mw_words(a) * (size_t)A->n;
    hipStream_t s = (hipStream_t)stream;
    double best_t = 0.0;
    mw_shape_t win{};
    // the time of `iters` lockstep iterations with shape `cand` (best of the
    // runs after the one that captures the chunk's graph)
    auto run = [&](mw_shape_t cand, double *out) -> int {
        mw_cg_opts_t o{};
        o.normalize = 1;
        o.shape = &cand;
        double t = 0.0;
        for (int rep = 0; rep < 3; ++rep) {
            HIP_TRY(hipMemsetAsync(x, 0, xbytes, s));
            mw_cg_info_t info{};
            const int rc = mw_cg_solve_batched(a, nsys, sys_row_off, A, b, x, 0.0, iters, &o, workspace, nullptr,
                                               nullptr, nullptr, &info, stream);
            if (rc < 0) return rc;
            if (info.iters < iters) {
                set_error("mw_cg_batched_tune: the iterations stopped early (b = 0 or breakdown)");
                return MW_EINVAL;
            }
            if (rep == 1 || (rep > 1 && info.seconds < t)) t = info.seconds;
        }
        *out = t;
        if (best_t == 0.0 || t < best_t) {
            best_t = t;
            win = cand;
        }
        return MW_OK;
    };
    int last = -1;
    int ns = 0;
    for (int k = 0; k < nsys; ++k) ns += (sys_row_off[k + 1] - sys_row_off[k] + 63) / 64;
    const int need = persistent_grid(blocks_for(ns > 0 ? ns : 1, NWAVE));
    int vec_slices = 0;
    for (int g : grids) {
        double t = 0.0;
        if (const int rc = run(mw_shape_t{g, 0, 0, iters, 0, 0.0}, &t)) return rc;
        vec_slices = g_last_vec_slices;
        // larger grids clamp to the slices' own count: stop once they do
        if (g >= need || g == last) break;
        last = g;
    }
    // lanes per row of the vector-row slices (rows per wavefront = 64 /
    // lanes), on the best grid, when the batch has such slices
    if (vec_slices > 0) {
        const int g = win.spmv_grid;
        for (int l = 2; l <= 64; l *= 2) {
            double t = 0.0;
            if (const int rc = run(mw_shape_t{g, 0, 0, iters, l, 0.0}, &t)) return rc;
        }
    }
    win.us_per_iteration = 1e6 * best_t / iters;
    win.chunk = 0;
    tuned_put(a, A->n, A->nnz, nsys, win);
    *best = win;
    return MW_OK;
}

}  // extern "C"
