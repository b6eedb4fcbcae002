// mw_tune.hip -- launch shapes of the solvers: the built-in shapes, the
// environment overrides, the per-process table the tuners fill (and its
// copy in a file, MW_TUNE_CACHE), and their precedence (explicit > tuned >
// environment > built-in).  The tuners themselves run the solvers and live
// beside them (mw_cg.hip, mw_batch.hip).
#include "mw_blas.hpp"

#include <unistd.h>

#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <mutex>
#include <string>

using namespace mwk;
using namespace mwh;

namespace {

struct TunedEntry {
    int a, n, nnz, nsys;
    mw_shape_t s;
};

constexpr int TABLE_SIZE = 64;  // distinct matrix sizes remembered; oldest replaced

std::mutex g_mu;
TunedEntry g_tab[TABLE_SIZE];
int g_used = 0, g_next = 0;

int env_int(const char *name)
{
    const char *e = getenv(name);
    return e ? atoi(e) : 0;
}

bool in_range(int v, int lo, int hi) { return v <= 0 || (v >= lo && v <= hi); }

void put_locked(int a, int n, int nnz, int nsys, const mw_shape_t &s)
{
    for (int i = 0; i < g_used; ++i) {
        TunedEntry &e = g_tab[i];
        if (e.a == a && e.n == n && e.nnz == nnz && e.nsys == nsys) {
            e.s = s;
            return;
        }
    }
    g_tab[g_next] = TunedEntry{a, n, nnz, nsys, s};
    g_next = (g_next + 1) % TABLE_SIZE;
    if (g_used < TABLE_SIZE) ++g_used;
}

// ---- the table's file (MW_TUNE_CACHE): one JSON object per line, keyed by
// the device (architecture name / compute units) and (arith, n, nnz, nsys).
// Read into the table at the first lookup; every tuner result rewrites the
// file (a temporary file renamed over it), keeping the lines of other
// devices and sizes.  A file that cannot be read or written is skipped.

constexpr int DEV_LEN = 96;
bool g_loaded = false;

const char *cache_path()
{
    const char *p = getenv("MW_TUNE_CACHE");
    return p && *p ? p : nullptr;
}

bool device_key(char *out)
{
    int dev = 0;
    hipDeviceProp_t p;
    if (hipGetDevice(&dev) != hipSuccess || hipGetDeviceProperties(&p, dev) != hipSuccess) {
        (void)hipGetLastError();
        return false;
    }
    std::string arch(p.gcnArchName);
    arch = arch.substr(0, arch.find(':'));
    snprintf(out, DEV_LEN, "%s/%d", arch.c_str(), p.multiProcessorCount);
    return true;
}

struct CacheLine {
    char dev[DEV_LEN];
    int a, n, nnz, nsys;
    mw_shape_t s;
};

bool parse_line(const char *line, CacheLine *c)
{
    *c = CacheLine{};
    const int got = sscanf(line,
                           "{\"device\": \"%95[^\"]\", \"arith\": %d, \"n\": %d, \"nnz\": %d, \"nsys\": %d, "
                           "\"spmv_grid\": %d, \"update_grid\": %d, \"update_threads\": %d, \"chunk\": %d, "
                           "\"lanes\": %d, \"us_per_iteration\": %lf}",
                           c->dev, &c->a, &c->n, &c->nnz, &c->nsys, &c->s.spmv_grid, &c->s.update_grid,
                           &c->s.update_threads, &c->s.chunk, &c->s.lanes, &c->s.us_per_iteration);
    return got == 11 && valid_arith(c->a) && c->n > 0 && c->nnz >= 0 && c->nsys >= 0 && shape_valid(&c->s);
}

void format_line(char *out, size_t len, const CacheLine &c)
{
    snprintf(out, len,
             "{\"device\": \"%s\", \"arith\": %d, \"n\": %d, \"nnz\": %d, \"nsys\": %d, \"spmv_grid\": %d, "
             "\"update_grid\": %d, \"update_threads\": %d, \"chunk\": %d, \"lanes\": %d, "
             "\"us_per_iteration\": %.6f}\n",
             c.dev, c.a, c.n, c.nnz, c.nsys, c.s.spmv_grid, c.s.update_grid, c.s.update_threads, c.s.chunk,
             c.s.lanes, c.s.us_per_iteration);
}

void load_locked()
{
    if (g_loaded) return;
    g_loaded = true;
    const char *path = cache_path();
    char dev[DEV_LEN];
    if (!path || !device_key(dev)) return;
    FILE *f = fopen(path, "r");
    if (!f) return;
    char line[512];
    CacheLine c;
    while (fgets(line, sizeof(line), f))
        if (parse_line(line, &c) && strcmp(c.dev, dev) == 0) put_locked(c.a, c.n, c.nnz, c.nsys, c.s);
    fclose(f);
}

void save_locked(int a, int n, int nnz, int nsys, const mw_shape_t &s)
{
    const char *path = cache_path();
    CacheLine me{};
    if (!path || !device_key(me.dev)) return;
    me.a = a;
    me.n = n;
    me.nnz = nnz;
    me.nsys = nsys;
    me.s = s;
    std::string text;
    char line[512];
    if (FILE *f = fopen(path, "r")) {
        CacheLine c;
        while (fgets(line, sizeof(line), f))
            if (parse_line(line, &c) && !(strcmp(c.dev, me.dev) == 0 && c.a == a && c.n == n && c.nnz == nnz &&
                                          c.nsys == nsys)) {
                format_line(line, sizeof(line), c);
                text += line;
            }
        fclose(f);
    }
    format_line(line, sizeof(line), me);
    text += line;
    const std::string tmp = std::string(path) + ".tmp" + std::to_string((long)getpid());
    FILE *f = fopen(tmp.c_str(), "w");
    if (!f) return;
    const bool ok = fwrite(text.data(), 1, text.size(), f) == text.size();
    if (fclose(f) != 0 || !ok || rename(tmp.c_str(), path) != 0) remove(tmp.c_str());
}

}  // namespace

namespace mwh {

void tuned_put(int a, int n, int nnz, int nsys, const mw_shape_t &s)
{
    std::lock_guard<std::mutex> lk(g_mu);
    load_locked();
    put_locked(a, n, nnz, nsys, s);
    save_locked(a, n, nnz, nsys, s);
}

bool tuned_get(int a, int n, int nnz, int nsys, mw_shape_t *s)
{
    std::lock_guard<std::mutex> lk(g_mu);
    load_locked();
    for (int i = 0; i < g_used; ++i) {
        const TunedEntry &e = g_tab[i];
        if (e.a == a && e.n == n && e.nnz == nnz && e.nsys == nsys) {
            *s = e.s;
            return true;
        }
    }
    return false;
}

bool shape_valid(const mw_shape_t *s)
{
    if (!s) return true;
    const int t = s->update_threads;
    return in_range(s->spmv_grid, 8, MAX_GRID) && in_range(s->update_grid, 8, MAX_GRID) &&
           (t <= 0 || t == 256 || t == 512 || t == 1024) && in_range(s->chunk, 1, 4096) &&
           (s->lanes <= 0 || (s->lanes >= 2 && s->lanes <= 64 && (s->lanes & (s->lanes - 1)) == 0));
}

// The fields set in `over` replace those of `base`.
static mw_shape_t overlay(mw_shape_t base, const mw_shape_t *over)
{
    if (!over) return base;
    if (over->spmv_grid > 0) base.spmv_grid = over->spmv_grid;
    if (over->update_grid > 0) base.update_grid = over->update_grid;
    if (over->update_threads > 0) base.update_threads = over->update_threads;
    if (over->chunk > 0) base.chunk = over->chunk;
    if (over->lanes > 0) base.lanes = over->lanes;
    return base;
}

CgShape cg_shape(int a, int n, int nnz, int tiles, const mw_shape_t *explicit_shape, int opts_chunk)
{
    mw_shape_t s{};
    (void)tuned_get(a, n, nnz, 0, &s);
    s = overlay(s, explicit_shape);
    CgShape r;
    // SpMV: QTW runs best with six resident wavefronts per SIMD (1536
    // workgroups of four), the other arithmetics with eight (2048), swept
    // on MI355X for 3D Poisson 128^3 over 512 .. 2048.
    int cap = s.spmv_grid;
    if (cap <= 0) {
        cap = (a == MW_QTW) ? 1536 : MAX_GRID;
        const int e = env_int("MW_SGRID");
        if (e >= 8 && e <= MAX_GRID) cap = e;
    }
    const int g = persistent_grid(tiles);
    r.sgrid = g < cap ? g : cap;
    // vector updates: 256 threads, at most 1024 workgroups (best of the
    // swept 256/512/1024-thread, 256 .. 2048-workgroup shapes on MI355X)
    r.unt = s.update_threads;
    if (r.unt <= 0) {
        r.unt = 256;
        const int e = env_int("MW_UNT");
        if (e == 256 || e == 512 || e == 1024) r.unt = e;
    }
    int ucap = s.update_grid;
    if (ucap <= 0) {
        ucap = 1024;
        const int e = env_int("MW_UGRID");
        if (e >= 8 && e <= MAX_GRID) ucap = e;
    }
    const int ub = blocks_for(n, r.unt);
    r.ugrid = ub < ucap ? ub : ucap;
    r.chunk = opts_chunk > 0 ? opts_chunk : (s.chunk > 0 ? s.chunk : 32);
    // even (a multiple of xr(a) <= 2): the parity pattern and the
    // search-direction buffers repeat per chunk
    r.chunk += r.chunk & 1;
    r.lanes = s.lanes;
    return r;
}

BatchShape batch_shape(int a, int n, int nnz, int nsys, int ns, const mw_shape_t *explicit_shape, int opts_chunk)
{
    mw_shape_t s{};
    (void)tuned_get(a, n, nnz, nsys, &s);
    s = overlay(s, explicit_shape);
    BatchShape r;
    const int g = persistent_grid(blocks_for(ns > 0 ? ns : 1, NWAVE));
    r.grid = (s.spmv_grid > 0 && s.spmv_grid < g) ? s.spmv_grid : g;
    r.chunk = opts_chunk > 0 ? opts_chunk : (s.chunk > 0 ? s.chunk : 16);
    r.lanes = s.lanes;
    return r;
}

}  // namespace mwh

extern "C" {

int mw_cg_shape(mw_arith_t a, int32_t n, int32_t nnz, int32_t nsys, mw_shape_t *shape)
{
    mwh::clear_error();
    if (!valid_arith(a) || n <= 0 || !size_ok(n) || !size_ok(nnz) || nsys < 0 || !shape) return MW_EINVAL;
    mw_shape_t t{};
    const bool tuned = tuned_get(a, n, nnz, nsys, &t);
    *shape = mw_shape_t{};
    if (nsys == 0) {
        // the plan format by size alone (plan_auto); irregular rows are not
        // seen from n and nnz
        const bool vec = rows_by_size(n, nnz);
        const int lanes = vec ? rows_lanes(a, n, nnz, cg_shape(a, n, nnz, 1, nullptr, 0).lanes) : 0;
        const long rpt = vec ? (long)NWAVE * (64 / lanes) : 64L * NWAVE;
        const CgShape c = cg_shape(a, n, nnz, (int)((n + rpt - 1) / rpt), nullptr, 0);
        shape->spmv_grid = c.sgrid;
        shape->update_grid = c.ugrid;
        shape->update_threads = c.unt;
        shape->chunk = c.chunk;
        shape->lanes = lanes;
    } else {
        shape->spmv_grid = tuned ? t.spmv_grid : 0;
        shape->chunk = tuned && t.chunk > 0 ? t.chunk : 16;
        shape->lanes = tuned ? t.lanes : 0;
    }
    shape->us_per_iteration = tuned ? t.us_per_iteration : 0.0;
    return tuned ? 1 : 0;
}

}  // extern "C"
