// mw_blas.hpp -- internal interface between the BLAS/SpMV and CG parts of
// libmwcg.
#pragma once

#include "mw_common.hpp"

namespace mwk {

// Device-resident state of one CG solve.  Values an iteration produces are
// kept per iteration parity (index i & 1 for iteration i, parity 0 holding
// the initial values): iteration i reads only the other parity's entries,
// which the previous iteration wrote before a kernel boundary, so no
// workgroup ever reads an entry another workgroup of the same kernel
// writes.
// Search-direction buffers of the CG solver: x takes the updates
// alpha_j p_j of xr(a) consecutive iterations in one pass, so one read and
// write of x serves xr(a) iterations at the cost of a second p buffer.
// For 3- and 4-word types that pays (measured on MI355X, 3D Poisson 128^3:
// QTW solve -2 %); for 1- and 2-word types the solver's working set (matrix
// and four vectors) just fits the 256 MB Infinity Cache and a second p
// buffer costs more than x's traffic (DW +11 %), so they keep one.
__host__ __device__ constexpr int xr(int a) { return vwords(a) >= 3 ? 2 : 1; }
constexpr int XR_MAX = 2;
constexpr int KMAX = 4;  // words of the widest arithmetic

struct CgState {
    double rho[2][KMAX];         // r^T r after the iteration of each parity
    double alpha[XR_MAX][KMAX];  // alpha of iteration k (0-based) in slot k % xr
    double nb;           // ||b||_2
    double tol;
    double rel_res;      // relative residual at the stop (or the last test)
    double *history;     // optional per-iteration relative residuals
    int32_t run[2];      // the iteration of this parity left the solve running
    int32_t iters[2];    // iteration count after the iteration of this parity
    int32_t brk[2];      // the alpha step of this parity broke down
    int32_t maxit;
    int32_t normalize;
    int32_t stopped;     // set once, when the solve stops (polled by the host)
    int32_t status;      // final status (valid once stopped)
    int32_t iters_final; // final iteration count (valid once stopped)
    int32_t normalize_p; // quasi types: p normalised with r (a placement variant)
};
// Loads of the matrix stream in the planned SpMV.  For 3- and 4-word vectors
// the CG working set (four vectors of 24 or 32 bytes per row) competes with the
// matrix stream for the 256 MB Infinity Cache; the matrix entries are used
// once per SpMV, so they are loaded non-temporally there.  For 1- and
// 2-word vectors plain loads measured faster.
template <int A, typename T>
__device__ __forceinline__ T load_matrix(const T *p)
{
    if constexpr (vwords(A) >= 3) return __builtin_nontemporal_load(p);
    else return *p;
}

// Sum of one row of a SELL-64 slice of width w starting at entry b, for
// lane l.  Inside a slice the entries are stored in pairs: entries 2m and
// 2m + 1 of lane l at b + 128 m + 2 l (+1), so one 16-byte load brings
// two values (8 bytes two columns); an odd last entry at b + 128 (w/2) + l.
// Every wavefront load is contiguous.  The entries are added in order
// j = 0, 1, ..., from zero; padding (col < 0) is skipped.  x is in word
// planes (XL = 0) or in the gather layout of load_il (XL = 1).
typedef int ivec2 __attribute__((ext_vector_type(2)));

template <int A, int XL>
__device__ __forceinline__ Num<A> sell_row_sum(int b, int w, int lane, const int32_t *__restrict__ sc,
                                               const double *__restrict__ sv, const double *__restrict__ x, long n)
{
    Num<A> acc = zero<A>();
    const int wp = w >> 1;
    for (int m = 0; m < wp; ++m) {
        const int z = b + 128 * m + 2 * lane;
        const dvec2 a = load_matrix<A>((const dvec2 *)(sv + z));
        const ivec2 c = load_matrix<A>((const ivec2 *)(sc + z));
        const Num<A> x0 = load_v<A, XL>(x, n, c.x < 0 ? 0 : c.x);
        const Num<A> x1 = load_v<A, XL>(x, n, c.y < 0 ? 0 : c.y);
        if (c.x >= 0) acc = row_step<A>(acc, a.x, x0);
        if (c.y >= 0) acc = row_step<A>(acc, a.y, x1);
    }
    if (w & 1) {
        const int z = b + 128 * wp + lane;
        const double a0 = load_matrix<A>(sv + z);
        const int c0 = load_matrix<A>(sc + z);
        const Num<A> x0 = load_v<A, XL>(x, n, c0 < 0 ? 0 : c0);
        if (c0 >= 0) acc = row_step<A>(acc, a0, x0);
    }
    return acc;
}

// Whether diagonal slices take the +-1 offsets from the neighbouring lane
// (DPP moves, see dia_x) instead of gathering them.  It pays for QTW, whose
// SpMV is bound by its gather traffic (measured on MI355X: 48.4 -> 44.5 us
// on 3D Poisson 128^3); FP64/DW/QDW gain nothing and TW, bound by its
// arithmetic, loses to the extra moves.
template <int A>
constexpr bool neighbour_moves() { return A == QTW; }

// The x window of a diagonal-slot slice: when every slot offset of a slice
// lies in [-WIN, WIN], the wavefront stages rows 64 s - WIN .. 64 s + 63 + WIN
// of x in its own LDS region (two coalesced loads per lane: its row, which
// the slice needs anyway, and one halo row), and every slot reads its
// operand from there instead of gathering it through the vector memory
// path.  Same values, same order: the row sums are bit-identical either
// way.  Slices with fewer than WIN_MIN_W slots (the 7-point stencils) keep
// the gathers: their two +-1 slots do not repay the halo load.  FP64 vectors
// (FP64 and the mixed types) keep them too: its 8-byte gathers are cheap, and with the window its SpMV on
// the 27-slot banded matrix measured 7 % slower (multi-word: DW 14 %, QTW
// 30 % faster).
constexpr int WIN = 32;
constexpr int WIN_ROWS = 64 + 2 * WIN;
constexpr int WIN_MIN_W = 5;

template <int A>
constexpr bool dia_window() { return vwords(A) > 1; }

// Whether all w slot offsets of a diagonal slice lie in [-WIN, WIN]
// (wave-uniform: scalar loads).  The slots follow the rows' CSR order, so
// their offsets need not be sorted; the loop stops at the first one
// outside.
__device__ __forceinline__ bool offsets_in_window(const int32_t *__restrict__ so, int w)
{
    for (int j = 0; j < w; ++j) {
        const int o = so[j];
        if (o < -WIN || o > WIN) return false;
    }
    return true;
}

// Orders a wavefront's own LDS accesses: LDS instructions of one wavefront
// execute in issue order, so only the compiler must not move the window's
// stores and loads across this point.
__device__ __forceinline__ void wave_lds_order()
{
    __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
    __builtin_amdgcn_wave_barrier();
}

// Stages the window of the slice whose first row is row - lane: lane l
// stores its x[row] (xc) at window index WIN + l and one halo row, lanes
// below WIN the row WIN above (index l), the others the row WIN below
// (index l + 2 WIN); rows outside [0, n) are stored as zero (no entry ever
// reads them).  wv: the wavefront's K * WIN_ROWS doubles of LDS, in the
// gather layout of WIN_ROWS elements.
template <int A, int XL>
__device__ __forceinline__ void stage_window(double *wv, int lane, long row, Num<A> xc,
                                             const double *__restrict__ x, long n)
{
    const long hr = lane < WIN ? row - WIN : row + WIN;
    const Num<A> xh = (hr >= 0 && hr < n) ? load_v<A, XL>(x, n, hr) : zero<A>();
    wave_lds_order();  // the previous slice's window reads come first
    store_il<A>(wv, WIN_ROWS, WIN + lane, xc);
    store_il<A>(wv, WIN_ROWS, lane < WIN ? lane : lane + 2 * WIN, xh);
    wave_lds_order();
}

// x[row + o] for a lane of a diagonal-slot slice whose slot has column
// offset o (wave-uniform); need: the lane has an entry in the slot.  xc is
// x[row] (0 for rows past n).  Offset 0 is xc itself.  With the window
// (W, wv staged by stage_window) every offset is read from LDS.  Else, with
// neighbour_moves, offsets +-1 are xc moved from the neighbouring lane and
// xe is the value one row beyond the slice's edge lane (lane 0:
// x[row - 1], lane 63: x[row + 1]), and any other offset is a gather.
// Called by the whole wavefront (the moves need every lane).
template <int A, int XL, bool W>
__device__ __forceinline__ Num<A> dia_x(int o, bool need, long row, Num<A> xc, Num<A> xe,
                                        const double *__restrict__ x, long n, const double *wv, int lane)
{
    if (o == 0) return xc;
    if constexpr (W) {
        return load_il<A>(wv, WIN_ROWS, WIN + lane + o);
    } else {
        if constexpr (neighbour_moves<A>()) {
            if (o == 1) return wave_shift1<1, A>(xc, xe);
            if (o == -1) return wave_shift1<-1, A>(xc, xe);
        }
        Num<A> v = zero<A>();
        if (need) v = load_v<A, XL>(x, n, row + o);
        return v;
    }
}

// Sum of one row of a diagonal-slot slice (same value positions as
// sell_row_sum): slot j holds, for every lane whose bit is set in
// smask[j], the entry in column row + soff[j]; other lanes hold 0 there
// and skip the slot.  A lane's entries occupy its set slots in CSR order,
// so the row is summed in CSR order from zero, as in sell_row_sum.
// soff / smask point at the slice's first slot (wave-uniform: scalar
// loads); the gathers need no column loads.  xc, xe: see dia_x.
template <int A, int XL, bool W>
__device__ __forceinline__ Num<A> dia_row_sum(int b, int w, int lane, long row, const int32_t *__restrict__ soff,
                                              const uint64_t *__restrict__ smask, const double *__restrict__ sv,
                                              const double *__restrict__ x, long n, Num<A> xc,
                                              Num<A> xe, const double *wv)
{
    Num<A> acc = zero<A>();
    const int wp = w >> 1;
    for (int m = 0; m < wp; ++m) {
        const int z = b + 128 * m + 2 * lane;
        const dvec2 a = load_matrix<A>((const dvec2 *)(sv + z));
        const bool p0 = (smask[2 * m] >> lane) & 1, p1 = (smask[2 * m + 1] >> lane) & 1;
        const Num<A> x0 = dia_x<A, XL, W>(soff[2 * m], p0, row, xc, xe, x, n, wv, lane);
        const Num<A> x1 = dia_x<A, XL, W>(soff[2 * m + 1], p1, row, xc, xe, x, n, wv, lane);
        if (p0) acc = row_step<A>(acc, a.x, x0);
        if (p1) acc = row_step<A>(acc, a.y, x1);
    }
    if (w & 1) {
        const int z = b + 128 * wp + lane;
        const double a0 = load_matrix<A>(sv + z);
        const bool p0 = (smask[w - 1] >> lane) & 1;
        const Num<A> x0 = dia_x<A, XL, W>(soff[w - 1], p0, row, xc, xe, x, n, wv, lane);
        if (p0) acc = row_step<A>(acc, a0, x0);
    }
    return acc;
}

// A slice starting at b with width w uses diagonal slots when its first
// slot mask is nonzero (wave-uniform).
__device__ __forceinline__ bool slice_is_diag(int b, int w, const uint64_t *__restrict__ smask)
{
    return w > 0 && smask[b >> 6] != 0;
}

// Position of entry j of lane l in a slice of width w starting at b.
__device__ __forceinline__ int sell_pos(int b, int w, int j, int lane)
{
    const int wp = w >> 1;
    return (j < 2 * wp) ? b + 128 * (j >> 1) + 2 * lane + (j & 1) : b + 128 * wp + lane;
}

// Scatters one slice (rows given per lane: first entry rs, length len; 0
// for lanes without a row) starting at entry b with width w.  First the
// diagonal-slot assignment is tried: slot j takes, from every lane whose
// next unplaced entry has the smallest column offset (column - row) among
// all lanes' next entries, that entry (each lane keeps its CSR order).
// When that places every entry within w slots, the slice keeps the values
// so placed plus one offset and lane mask per slot (slots from b / 64);
// otherwise it is rewritten with explicit columns and zero slot masks.
// Called by a whole wavefront; returns whether the slice is diagonal.
__device__ __forceinline__ bool fill_slice(int b, int w, int lane, long row, int rs, int len,
                                           const int32_t *__restrict__ col, const double *__restrict__ val,
                                           int32_t *__restrict__ scol, double *__restrict__ sval,
                                           int32_t *__restrict__ soff, uint64_t *__restrict__ smask)
{
    const int sl = b >> 6;
    int k = 0;  // this lane's entries placed so far
    // the lane's next FW entries (k .. k + FW - 1), loaded ahead so that a
    // slot does not wait for the load of the entry it places
    constexpr int FW = 4;
    int c[FW];
    double v[FW];
#pragma unroll
    for (int d = 0; d < FW; ++d) {
        c[d] = d < len ? col[rs + d] : 0;
        v[d] = d < len ? val[rs + d] : 0.0;
    }
    // values of a slot pair are stored together (one 16-byte store per
    // lane at the pair's position), the odd last slot alone
    double pend = 0.0;
    for (int j = 0; j < w; ++j) {
        const int cand = k < len ? (int)(c[0] - row) : 0x7fffffff;
        int m = cand;
#pragma unroll
        for (int off = 32; off > 0; off >>= 1) m = min(m, __shfl_xor(m, off, 64));
        const bool has = k < len && cand == m;
        const uint64_t mask = __ballot(has);
        const double vj = has ? v[0] : 0.0;
        if (j >= 2 * (w >> 1)) sval[sell_pos(b, w, j, lane)] = vj;
        else if (j & 1) *(dvec2 *)(sval + sell_pos(b, w, j - 1, lane)) = dvec2{pend, vj};
        else pend = vj;
        if (lane == 0) {
            soff[sl + j] = m;
            smask[sl + j] = mask;
        }
        if (has) {
#pragma unroll
            for (int d = 0; d + 1 < FW; ++d) {
                c[d] = c[d + 1];
                v[d] = v[d + 1];
            }
            const int nk = k + FW;
            c[FW - 1] = nk < len ? col[rs + nk] : 0;
            v[FW - 1] = nk < len ? val[rs + nk] : 0.0;
            ++k;
        }
    }
    if (__ballot(k != len) == 0) return w > 0;
    for (int j = 0; j < w; ++j) {
        const int pos = sell_pos(b, w, j, lane);
        if (j < len) {
            sval[pos] = val[rs + j];
            scol[pos] = col[rs + j];
        } else {
            sval[pos] = 0.0;
            scol[pos] = -1;
        }
        if (lane == 0) smask[sl + j] = 0;
    }
    return false;
}

// Sum over the 64 lanes of a wavefront (shuffle tree, offsets 32 .. 1);
// valid in lane 0.
template <int A>
__device__ __forceinline__ Num<A> wave_sum(Num<A> v)
{
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v = add<A>(v, shfl_down<A>(v, off));
    return v;
}

// z_i = d_i r_i, the Jacobi step of the preconditioned solvers: the FP64
// reciprocal of a_ii times the multi-word residual (FP64, and the mixed
// types, whose z is an FP64 vector: one rounded product).
template <int A>
__device__ __forceinline__ Num<A> jacobi(double d, const Num<A> &r)
{
    if constexpr (A == FP64 || is_mixed(A)) return promote<A>(d * r.w[0]);
    else return dxmul<A>(d, r);
}

}  // namespace mwk

namespace mwh {

// Exclusive scan of 64 * width[0..ns) into slice_ptr[0..ns], 64-bit total
// into *total (one workgroup).
int launch_sell_scan(int ns, const int32_t *width, int32_t *slice_ptr, long long *total, hipStream_t s);


// Bytes of a SpMV plan buffer for an n x n matrix with nnz entries.
size_t plan_bytes(int32_t n, int32_t nnz);

// Builds a plan (SELL-64, or the CSR fallback) in `buffer`; synchronises s.
int plan_build(const mw_csr_t *A, void *buffer, size_t bytes, mw_spmv_plan_t *plan, hipStream_t s);

// The CSR check of mw_csr_check (synchronises s), and whether every entry
// point that reads a matrix runs it first (MW_CHECK_CSR=1 in the
// environment, read once).
int csr_check(const mw_csr_t *A, hipStream_t s);
bool csr_check_on();
#define MW_CSR_GUARD(A, s)                                              \
    do {                                                                \
        if (mwh::csr_check_on()) {                                      \
            const int rc_ = mwh::csr_check((A), (hipStream_t)(s));      \
            if (rc_) return rc_;                                        \
        }                                                               \
    } while (0)

// dinv[i] = fl(1 / a_ii) for every row of A (the Jacobi preconditioner;
// see launch_jacobi_dinv in mw_blas.hip).
void launch_jacobi_dinv(const mw_csr_t *A, double *dinv, hipStream_t s);

// Most reduction slots any CG-mode SpMV launch writes for n rows.
int spmv_max_slots(int32_t n);

// A plan's fields are consistent with its format (for plans a caller
// hands in: a known format, SELL arrays present, lanes a power of two).
bool plan_valid(const mw_spmv_plan_t *plan);
// Vector-row plans (MW_FMT_CSRVEC): fill `plan` with `lanes` lanes per row
// (0: about eight entries per lane for the average row).
int plan_rows(const mw_csr_t *A, int lanes, mw_spmv_plan_t *plan);
// Whether a solve in arithmetic a takes vector rows for A on its row
// count and length alone (too few 64-row slices to fill the GPU), and the
// lanes per row it then takes (`lanes` > 0: that many).
bool rows_by_size(int n, int nnz);
int rows_lanes(int a, int n, int nnz, int lanes);
// The plan a solve builds for itself: vector rows when rows_by_size, or
// when SELL-64 would pad too much (irregular rows, the CSR fallback) and
// rows average 16 entries or more; else SELL-64 (or the CSR fallback) in
// `buffer`.  Synchronises s unless vector rows are chosen by size.
int plan_auto(int a, const mw_csr_t *A, int lanes, void *buffer, size_t bytes, mw_spmv_plan_t *plan,
              hipStream_t s);
// Workgroup tiles of a plan's SpMV (SELL-64: four slices; vector rows:
// 4 * 64 / lanes rows); a persistent grid larger than this idles.
int spmv_tiles(const mw_spmv_plan_t *plan);

// y = A x.  plan == nullptr or plan->format == MW_FMT_CSR: CSR kernel on M
// (one workgroup per NT rows); else the SELL-64 kernel on `grid`
// workgroups (0: the built-in shape, cg_shape).  mode 1 (CG): x is p, y is
// q, the workgroup partials of p^T q go to `slots` (their count to
// *nslots); the launch does nothing but pass the stop on (*run_cur = 0)
// when *run_prev is 0.  rev: walk the tiles backwards (see xcd_walk).
// ev0/ev1: optional events that time the kernel (MW_LAUNCH).
template <int A>
int spmv_launch(const mw_csr_t *M, const mw_spmv_plan_t *plan, const double *x, double *y, double *slots,
                const int32_t *run_prev, int32_t *run_cur, int mode, hipStream_t s, int *nslots = nullptr,
                int rev = 0, hipEvent_t ev0 = nullptr, hipEvent_t ev1 = nullptr, int grid = 0);

// Launch shapes (mw_tune.hip).  Precedence: the fields an explicit shape
// sets, then a tuned shape of the same (arith, n, nnz[, nsys]), then the
// MW_SGRID / MW_UGRID / MW_UNT environment overrides, then the built-in
// shape.
struct CgShape {
    int sgrid;  // workgroups of the SpMV (SELL-64 or vector rows)
    int unt;    // threads per update workgroup (256, 512, 1024)
    int ugrid;  // workgroups of the update kernels
    int chunk;  // iterations per chunk (even)
    int lanes;  // lanes per row of a vector-row plan the solver builds (0: its rule)
};
struct BatchShape {
    int grid;   // workgroups of the slice kernels
    int chunk;  // iterations per chunk
    int lanes;  // lanes per row of the vector-row slices (0: each slice's rule)
};
CgShape cg_shape(int a, int n, int nnz, int tiles, const mw_shape_t *explicit_shape, int opts_chunk);
BatchShape batch_shape(int a, int n, int nnz, int nsys, int ns, const mw_shape_t *explicit_shape, int opts_chunk);
void tuned_put(int a, int n, int nnz, int nsys, const mw_shape_t &s);
bool tuned_get(int a, int n, int nnz, int nsys, mw_shape_t *s);
bool shape_valid(const mw_shape_t *s);

}  // namespace mwh
