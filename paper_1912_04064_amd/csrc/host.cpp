// host.cpp -- C-ABI implementation and host runtime of the SDMD PIC library.
//
// A context holds up to max_runs independent runs in a device run table.
// Runs of the same dimensionality, precision and patch class share one
// launch per phase, so a step is three launches per class whatever the
// number of runs:
//   push  (one workgroup per segment slot of every run)  -- particles phase
//   yee   (one workgroup per region tile of every run)   -- transfer (i),
//         current filter, Maxwell (or J only, followed by the spectral
//         launches of each spectral run)
//   post  (ghost chunks + leaver insertion)              -- Sync
// and every `relayout_every` steps a re-layout check (three launches that
// exit at once unless some patch overflowed).  Runs of 2 and 8 steps (E/B
// buffer parity 0 then 1, repeated) and a whole re-layout period with its
// check are captured once in hipGraphs and replayed.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <array>
#include <chrono>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <map>
#include <mutex>
#include <string>
#include <tuple>
#include <vector>

#include "launch.h"
#include "sdmd_dev.h"
#include "sdmd_pic.h"

using namespace sdmd;

namespace {

thread_local std::string g_init_error;

struct DevBuf {
    void *p = nullptr;
    size_t bytes = 0;
};

struct Run {
    bool active = false;
    int dims = 2, prec = PIC_FP64, pc = 8, px = 0;
    int ytx = 64;          // field-kernel tile width along x
    bool split = false;
    int ncell = 0;
    int total_ghosts = 0;
    int64_t steps = 0;     // steps taken (issued, capped at target)
    int64_t issued = 0;    // steps enqueued since admission
    int64_t target = 0;    // max_steps (0 = unlimited)
    int par0 = 0;          // E/B buffer holding the state at admission
    double *gauss0 = nullptr;   // div_h E - rho of the initial state, per node
    size_t bytes = 0;
    RunDev rd{};
    std::vector<DevBuf> bufs;
};

struct PushClass {
    int dims, pc, px;
    bool split;
    std::vector<int2> h;
    int2 *d = nullptr;
    size_t cap = 0;
};

struct FieldClass {
    int dims;
    bool split;
    int tx;      // Yee tile x extent
    bool filt;   // runs with the binomial current filter
    int solver;  // PIC_SOLVER_*
    std::vector<int4> hy, hp;
    std::vector<int> slots;
    int4 *dy = nullptr, *dp = nullptr;
    int *dslots = nullptr;
    size_t capy = 0, capp = 0, caps = 0;
    int count_gx = 1, move_gx = 1, commit_gx = 1;
};

}  // namespace

struct pic_ctx {
    pic_runtime rt{};
    hipStream_t stream = nullptr;
    hipStream_t cap_stream = nullptr;
    int device = -1;          // the device current at pic_init
    bool det = false;         // deterministic mode (pic_runtime.deterministic)
    int max_runs = 0;
    std::vector<Run> runs;
    RunDev *d_runs = nullptr;
    int *d_slot1 = nullptr;   // one slot, for single-run re-layouts
    std::vector<PushClass> pcls;
    std::vector<FieldClass> fcls;
    std::vector<DevBuf> own;   // context-level buffers
    int par = 0;
    int64_t step = 0;
    int relayout_every = 16;
    bool use_graph = true;
    hipGraphExec_t g2 = nullptr;      // two steps
    hipGraphExec_t g8 = nullptr;      // eight steps
    hipGraphExec_t gK = nullptr;      // relayout_every steps and the re-layout check after them
    hipGraphExec_t grel = nullptr;    // re-layout check
    bool graphs_valid = false;
    size_t bytes = 0;        // device bytes held now
    size_t peak_bytes = 0;   // the most held since pic_init
    std::string err;
    double t_ms[4] = {0, 0, 0, 0};
    double t_push_kernel_ms = 0.0;   // the particle kernels' own duration per step (last pic_time_phases)
};

// ------------------------------------------------------------------ errors
static int set_err(pic_ctx *c, int code, const char *fmt, ...)
{
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    if (c)
        c->err = buf;
    else
        g_init_error = buf;
    return code;
}

#define HIPCHK(ctx, expr)                                                                                  \
    do {                                                                                                   \
        hipError_t e_ = (expr);                                                                            \
        if (e_ != hipSuccess) return set_err(ctx, PIC_E_DEVICE, "%s: %s", #expr, hipGetErrorString(e_));   \
    } while (0)

// ------------------------------------------------------------------ static scratch
// Device scratch of pic_diag_noalloc: one array per GPU in this library's
// code object, held until the process ends.  Host code never uses the
// array's name as an address (in host code it is only a stand-in for the
// symbol): the device address is looked up once per device, at pic_init
// with that device current, and every use goes through that address.
// All calls on one GPU share the array.
constexpr size_t STATIC_SCRATCH_BYTES = (size_t)64 << 20;
static __device__ __align__(256) char scratch[STATIC_SCRATCH_BYTES];

constexpr int MAX_DEVICES = 64;
static std::mutex g_scratch_mu;
static void *g_scratch_ptr[MAX_DEVICES];
static hipError_t g_scratch_err[MAX_DEVICES];
static bool g_scratch_done[MAX_DEVICES];

static void resolve_static_scratch(int dev)
{
    if (dev < 0 || dev >= MAX_DEVICES) return;
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (g_scratch_done[dev]) return;
    void *p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    g_scratch_ptr[dev] = e == hipSuccess ? p : nullptr;
    g_scratch_err[dev] = e;
    g_scratch_done[dev] = true;
}

static void *static_scratch(int dev)
{
    if (dev < 0 || dev >= MAX_DEVICES) return nullptr;
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    return g_scratch_done[dev] ? g_scratch_ptr[dev] : nullptr;
}

static const char *static_scratch_error(int dev)
{
    if (dev < 0 || dev >= MAX_DEVICES) return "device index out of range";
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (!g_scratch_done[dev]) return "not looked up: no context was created on this device";
    return hipGetErrorString(g_scratch_err[dev]);
}

// ------------------------------------------------------------------ memory
// Every device allocation of a context goes through dev_alloc, rounded to
// 256 bytes.  With an HBM budget set, an allocation that would take the
// context's total above it fails (the caller reports PIC_E_NOMEM), so the
// context never holds more than its budget.
static size_t alloc_size(size_t bytes) { return bytes == 0 ? 256 : ((bytes + 255) & ~(size_t)255); }

static void *dev_alloc(pic_ctx *c, size_t bytes)
{
    bytes = alloc_size(bytes);
    if (c->rt.hbm_budget && c->bytes + bytes > c->rt.hbm_budget) return nullptr;
    void *p = nullptr;
    if (c->rt.alloc) {
        p = c->rt.alloc(bytes, c->rt.stream, c->rt.user);
    } else if (hipMalloc(&p, bytes) != hipSuccess) {
        p = nullptr;
    }
    if (p) {
        c->bytes += bytes;
        c->peak_bytes = std::max(c->peak_bytes, c->bytes);
    }
    return p;
}

static void dev_free(pic_ctx *c, DevBuf &b)
{
    if (!b.p) return;
    if (c->rt.free)
        c->rt.free(b.p, b.bytes, c->rt.stream, c->rt.user);
    else
        hipFree(b.p);
    c->bytes -= b.bytes;
    b.p = nullptr;
    b.bytes = 0;
}

static void *run_alloc(pic_ctx *c, Run &r, size_t bytes)
{
    const size_t b = alloc_size(bytes);
    void *p = dev_alloc(c, b);
    if (p) r.bufs.push_back({p, b});
    return p;
}

// Short-lived device buffers of one call (staging, partial sums), released
// when the call returns, on every path.
struct Scratch {
    pic_ctx *c;
    std::vector<DevBuf> bufs;
    explicit Scratch(pic_ctx *ctx) : c(ctx) {}
    Scratch(const Scratch &) = delete;
    Scratch &operator=(const Scratch &) = delete;
    void *get(size_t bytes)
    {
        void *p = dev_alloc(c, bytes);
        if (p) bufs.push_back({p, alloc_size(bytes)});
        return p;
    }
    ~Scratch()
    {
        for (auto &b : bufs) dev_free(c, b);
    }
};

// ------------------------------------------------------------------ layout
struct Layout {
    int dims, pc;
    bool split;
    int n[3], P[3], np[3], nreg[3], rs[3], ra[3], TA[3];
    int n_patch, n_regions, tsz, ghosts;
    int seg_cap, seg_max;
    long long rsize;
    long long n_total, cap_total;
    size_t tile_esz;   // bytes per tile value: FP32 / FP64, 8 in the deterministic mode
    size_t resident;   // device bytes the run holds between calls
    size_t bytes;      // resident + the most any call takes on top (set-up
                       // staging, read-out scratch, the run's item lists)
};

static int patch_class(int dims, const int P[3])
{
    int m = std::max(P[0], P[1]);
    if (dims == 3) m = std::max(m, P[2]);
    if (m <= 8) return 8;
    if (m <= 16) return 16;
    return 32;
}

static size_t align256(size_t b) { return (b + 255) & ~(size_t)255; }

// live particles per segment a re-layout aims at: 8 chunks of the 2D
// workgroup width (256); 4 chunks of the 3D one (1024).  In 3D a segment
// also costs a window load of 6 x 11^3 nodes and a 3 x 13^3 tile that the
// field kernel gathers, so segments are larger (measured on the 3D
// cylinder input: 2048 -> 4096 cuts the step by 15 %, 8192 is slower
// again).
constexpr int SEG_CAP_2D = 2048;
constexpr int SEG_CAP_3D = 4096;

// exact patch edge with a compiled fast path of the particle kernel, or 0
static int fast_patch(const Layout &L)
{
    const bool square = L.P[0] == L.P[1] && (L.dims == 2 || L.P[2] == L.P[0]);
    if (!square) return 0;
    const int p = L.P[0];
    if (L.dims == 2) {
        if (p == 8 || p == 16 || (p == 32 && L.split)) return p;
        return 0;
    }
    return p == 8 ? 8 : 0;
}

// validate a config (patch already chosen) and derive the layout
static int make_layout(const pic_config *cfg, const int P[3], bool det, Layout &L, std::string &why)
{
    char buf[256];
    auto fail = [&](const char *m) {
        why = m;
        return PIC_E_CONFIG;
    };
    const int dims = cfg->dims;
    if (dims != 2 && dims != 3) return fail("dims must be 2 or 3");
    if (cfg->shape_order != 2) return fail("shape_order must be 2 (quadratic shapes, Esirkepov 5-point frame)");
    if (cfg->precision != PIC_FP64 && cfg->precision != PIC_FP32_SPLIT) return fail("unknown precision");
    if (!(cfg->m > 0)) return fail("mass must be positive");
    double inv2 = 0.0;
    for (int a = 0; a < dims; ++a) {
        if (cfg->bc[a] != PIC_BC_PERIODIC) return fail("only periodic boundaries are supported");
        if (cfg->n_cells[a] < 1) return fail("n_cells must be >= 1");
        if (!(cfg->d[a] > 0)) return fail("cell sizes must be positive");
        inv2 += 1.0 / (cfg->d[a] * cfg->d[a]);
    }
    if (dims == 2 && cfg->n_cells[2] != 1) return fail("n_cells[2] must be 1 in 2D");
    if (cfg->field_solver != PIC_SOLVER_YEE && cfg->field_solver != PIC_SOLVER_PSATD) return fail("unknown field solver");
    if (cfg->field_solver == PIC_SOLVER_YEE) {
        if (!(cfg->dt > 0) || !(cfg->dt < 1.0 / std::sqrt(inv2)))
            return fail("dt must satisfy 0 < dt < 1/sqrt(sum 1/d^2)");
    } else {
        double dmin = cfg->d[0];
        for (int a = 1; a < dims; ++a) dmin = std::min(dmin, cfg->d[a]);
        if (!(cfg->dt > 0) || !(cfg->dt < dmin)) return fail("spectral solver: dt must satisfy 0 < dt < min d");
        for (int a = 0; a < dims; ++a) {
            const int n = cfg->n_cells[a];
            if (n > 2048 || (n & (n - 1)) != 0) return fail("spectral solver: n_cells must be powers of two <= 2048");
            if (cfg->n_regions[a] != 1) return fail("spectral solver: one region");
        }
    }
    if (cfg->filter_passes < 0 || cfg->filter_passes > (dims == 2 ? 4 : 2))
        return fail("filter_passes must be 0..4 in 2D, 0..2 in 3D");
    if (cfg->seg_cap != 0 && (cfg->seg_cap < 256 || cfg->seg_cap > 65536))
        return fail("seg_cap must be 0 or in [256, 65536]");
    if (cfg->field_tile_x != 0) {
        const int t = cfg->field_tile_x;
        const bool ok = dims == 2 ? (t == 8 || t == 16 || t == 32 || t == 64)
                                  : (cfg->filter_passes > 0 ? t == 8 : (t == 8 || t == 16 || t == 32));
        if (!ok) return fail("field_tile_x must be 0 or a compiled width (2D: 8, 16, 32, 64; 3D: 8, 16, 32; 3D with "
                             "the filter: 8)");
    }
    const int pmax = dims == 2 ? 32 : 8;
    L.dims = dims;
    L.split = cfg->precision == PIC_FP32_SPLIT;
    long long ncell = 1;
    for (int a = 0; a < 3; ++a) {
        if (a >= dims) {
            L.n[a] = 1;
            L.P[a] = 1;
            L.np[a] = 1;
            L.nreg[a] = 1;
            L.rs[a] = 1;
            L.ra[a] = 1;
            L.TA[a] = 1;
            continue;
        }
        L.n[a] = cfg->n_cells[a];
        L.P[a] = P[a];
        if (P[a] < 4) return fail("patch size must be >= 4 cells per axis (a patch holds the interpolation support)");
        if (P[a] > pmax) {
            snprintf(buf, sizeof buf, "patch size must be <= %d cells per axis in %dD", pmax, dims);
            why = buf;
            return PIC_E_CONFIG;
        }
        if (L.n[a] % P[a]) return fail("patch size must divide n_cells");
        L.np[a] = L.n[a] / P[a];
        const int nr = cfg->n_regions[a] < 1 ? 1 : cfg->n_regions[a];
        if (L.np[a] % nr) return fail("regions must be made of whole patches and all of equal shape");
        L.nreg[a] = nr;
        L.rs[a] = L.n[a] / nr;
        L.ra[a] = L.rs[a] + 2 * GH;
        L.TA[a] = P[a] + 5;
        ncell *= L.n[a];
    }
    if (ncell > (1LL << 31) - 1) return fail("grid too large");
    L.pc = patch_class(dims, L.P);
    L.n_patch = L.np[0] * L.np[1] * L.np[2];
    L.n_regions = L.nreg[0] * L.nreg[1] * L.nreg[2];
    L.rsize = (long long)L.ra[0] * L.ra[1] * L.ra[2];
    L.tsz = L.TA[0] * L.TA[1] * L.TA[2];
    const int G2 = 2 * GH;
    if (dims == 2)
        L.ghosts = G2 * L.ra[0] + G2 * L.rs[1];
    else
        L.ghosts = G2 * L.ra[0] * L.ra[1] + L.rs[2] * G2 * L.ra[0] + L.rs[2] * L.rs[1] * G2;
    L.n_total = cfg->particles ? cfg->particles->n : 0;
    if (L.n_total < 0) return fail("negative particle count");
    // segments: a re-layout splits a patch into ceil(count / seg_cap)
    // segments, so at most n_patch + N / seg_cap of them exist
    L.seg_cap = cfg->seg_cap > 0 ? cfg->seg_cap : (dims == 3 ? SEG_CAP_3D : SEG_CAP_2D);
    L.seg_max = (int)(L.n_patch + (L.n_total + L.seg_cap - 1) / L.seg_cap + 16);
    L.cap_total = L.n_total + L.n_total / 2 + 32LL * L.seg_max + 1024;
    if (L.cap_total > (1LL << 31) - 1) return fail("too many particles for one run");
    // bytes
    const size_t rsz = L.split ? 4 : 8;
    L.tile_esz = det ? 8 : rsz;
    const bool ids = cfg->track_ids != 0;
    const size_t per = dims * rsz + (L.split ? 2 : 0) + 3 * rsz + rsz + (ids ? 4 : 0);
    size_t b = 0;
    b += align256((size_t)L.n_regions * F_NCOMP * L.rsize * 8);
    b += align256((size_t)L.seg_max * 3 * L.tsz * L.tile_esz);
    b += 7 * align256((size_t)(L.n_patch + 1) * 4) + 7 * align256((size_t)(L.seg_max + 1) * 4);
    b += 2 * (size_t)L.cap_total * per + align256((size_t)L.cap_total * 4);
    b += 2 * (size_t)std::max<long long>(L.n_total, 1) * (per + 4);
    if (cfg->field_solver == PIC_SOLVER_PSATD) b += align256((size_t)SPEC_ARRAYS * ncell * 16) + align256((size_t)SPEC_TW_LEN * 16);
    b += align256((size_t)ncell * 8);   // initial Gauss residual
    b += 64 * 256;   // per-array rounding and the control block
    L.resident = b;
    // transient device memory, the largest of: the set-up staging (fields,
    // then FP64 particles and ids, then the charge density of the initial
    // Gauss residual, one after the other), and the read-out scratch of
    // pic_fields, pic_diag (partial sums, residual, charge density) and
    // pic_particles (FP64 arrays, ids, patches, segment offsets)
    const size_t nt = (size_t)std::max<long long>(L.n_total, 1);
    const size_t nb = (size_t)std::max<long long>(1, std::min<long long>(1024, (ncell + BLOCK - 1) / BLOCK));
    const size_t cell8 = align256((size_t)ncell * 8);
    size_t tr = std::max({align256((size_t)3 * ncell * 8), 7 * align256(nt * 8) + align256(nt * 4), cell8});
    tr = std::max(tr, align256(std::max(2 * nb, (size_t)L.seg_max + 1) * 8) + align256((size_t)ncell * 8 + 2 * nb * 8) +
                          cell8);
    tr = std::max(tr, 7 * align256(nt * 8) + 2 * align256(nt * 4) + align256(((size_t)L.seg_max + 1) * 4));
    // item lists of the run's launches (kept at up to twice their size):
    // particle items per segment slot; field items per region tile (a tile
    // covers at least 64 nodes, or a whole smaller region); post items per
    // 256 ghost nodes (fewer than 2 per node) and per segment
    const size_t yee_items = (size_t)ncell / 64 + (size_t)L.n_regions;
    const size_t post_items = (size_t)ncell / 128 + (size_t)L.n_regions + (size_t)L.seg_max + 64;
    const size_t items = 2 * ((size_t)(L.seg_max + 8) * 8 + (yee_items + post_items) * 16);
    L.bytes = b + tr + align256(items) + 4096;
    return PIC_OK;
}

// default patch shape when the caller leaves it to the library: the
// measured choice for 2D is 16 cells (8 for small grids); 3D uses 8
static void default_patch(const pic_config *cfg, int P[3])
{
    const int dims = cfg->dims;
    for (int a = 0; a < 3; ++a) P[a] = 1;
    const int cands2[] = {16, 8, 32, 12, 10, 4};
    const int cands3[] = {8, 4, 6};
    for (int a = 0; a < dims; ++a) {
        const int nr = cfg->n_regions[a] < 1 ? 1 : cfg->n_regions[a];
        const int *c = dims == 2 ? cands2 : cands3;
        const int nc = dims == 2 ? 6 : 3;
        P[a] = 0;
        for (int i = 0; i < nc; ++i)
            if (cfg->n_cells[a] % (c[i] * nr) == 0) {
                P[a] = c[i];
                break;
            }
    }
}

// ------------------------------------------------------------------ run setup
static void free_run(pic_ctx *c, Run &r)
{
    for (auto &b : r.bufs) dev_free(c, b);
    r.bufs.clear();
    r.active = false;
}

static void make_store(pic_ctx *c, Run &r, Store &s, long long n, bool split, int dims, bool ids, bool &ok)
{
    const size_t rsz = split ? 4 : 8;
    const size_t nn = (size_t)std::max<long long>(n, 1);
    for (int a = 0; a < 3; ++a) s.pos[a] = a < dims ? run_alloc(c, r, nn * rsz) : nullptr;
    s.cell = split ? (uint16_t *)run_alloc(c, r, nn * 2) : nullptr;
    for (int a = 0; a < 3; ++a) s.u[a] = run_alloc(c, r, nn * rsz);
    s.w = run_alloc(c, r, nn * rsz);
    s.id = ids ? (uint32_t *)run_alloc(c, r, nn * 4) : nullptr;
    for (int a = 0; a < dims; ++a) ok = ok && s.pos[a];
    ok = ok && s.u[0] && s.u[1] && s.u[2] && s.w && (!split || s.cell) && (!ids || s.id);
}

static int upload_rd(pic_ctx *c, int slot)
{
    HIPCHK(c, hipMemcpyAsync(c->d_runs + slot, &c->runs[slot].rd, sizeof(RunDev), hipMemcpyHostToDevice, c->stream));
    return PIC_OK;
}

static Ctl read_ctl(pic_ctx *c, int slot, hipError_t &e)
{
    Ctl ctl;
    memset(&ctl, 0, sizeof ctl);
    e = hipMemcpy(&ctl, c->runs[slot].rd.ctl, sizeof ctl, hipMemcpyDeviceToHost);
    ctl.nspill = std::max(0, std::min(ctl.nspill, c->runs[slot].rd.n_total));
    return ctl;
}

static int check_run_err(pic_ctx *c, int slot, int *flags_out = nullptr)
{
    Ctl ctl;
    HIPCHK(c, hipMemcpyAsync(&ctl, c->runs[slot].rd.ctl, sizeof ctl, hipMemcpyDeviceToHost, c->stream));
    HIPCHK(c, hipStreamSynchronize(c->stream));
    if (flags_out) *flags_out = ctl.err;
    if (ctl.err & ERR_RANGE) return set_err(c, PIC_E_CONFIG, "run %d: particle position outside [0, L)", slot);
    if (ctl.err & ERR_NONFINITE) return set_err(c, PIC_E_NUMERIC, "run %d: non-finite particle value", slot);
    if (ctl.err & ERR_MOVE) return set_err(c, PIC_E_NUMERIC, "run %d: a particle moved a cell or more in one step", slot);
    if (ctl.err & ERR_CAPACITY) return set_err(c, PIC_E_OVERFLOW, "run %d: particle store capacity exceeded", slot);
    return PIC_OK;
}

// host copy of a run's segment table (diagnostics and export only)
struct SegView {
    int nseg = 0;
    std::vector<int> sseg, scnt, spat;
};

static int read_segments(pic_ctx *c, int slot, const Ctl &ctl, SegView &v)
{
    const RunDev &d = c->runs[slot].rd;
    v.nseg = std::max(0, std::min(ctl.nseg, d.seg_max));
    v.sseg.assign(v.nseg + 1, 0);
    v.scnt.assign(std::max(v.nseg, 1), 0);
    v.spat.assign(std::max(v.nseg, 1), 0);
    HIPCHK(c, hipMemcpy(v.sseg.data(), d.sseg, (v.nseg + 1) * 4, hipMemcpyDeviceToHost));
    if (v.nseg > 0) {
        HIPCHK(c, hipMemcpy(v.scnt.data(), d.scnt, v.nseg * 4, hipMemcpyDeviceToHost));
        HIPCHK(c, hipMemcpy(v.spat.data(), d.spat, v.nseg * 4, hipMemcpyDeviceToHost));
    }
    return PIC_OK;
}

static int relayout_one(pic_ctx *c, int slot, int force)
{
    Run &r = c->runs[slot];
    HIPCHK(c, hipMemcpyAsync(c->d_slot1, &slot, sizeof(int), hipMemcpyHostToDevice, c->stream));
    const int nsb = std::max(1, std::min(1024, (int)(r.rd.n_total / (BLOCK * 64))));
    const int mgx = move_chunk_blocks(r.rd.n_patch, r.rd.n_total) + nsb;
    int cb = (int)std::min<long long>(64, std::max<long long>(1, (r.rd.seg_max + BLOCK) / BLOCK));
    HIPCHK(c, launch_relayout(r.dims, r.split, c->d_runs, c->d_slot1, 1, nsb, mgx, cb, force, c->stream));
    return PIC_OK;
}

// ------------------------------------------------------------------ autotuner
// Square patch edges the particle kernel has compiled paths for
static std::vector<int> patch_candidates(const pic_config *cfg)
{
    std::vector<int> out;
    const int c2[] = {8, 16, 32}, c3[] = {4, 8};
    const int *cs = cfg->dims == 2 ? c2 : c3;
    const int nc = cfg->dims == 2 ? 3 : 2;
    for (int i = 0; i < nc; ++i) {
        bool ok = true;
        for (int a = 0; a < cfg->dims; ++a) {
            const int nr = cfg->n_regions[a] < 1 ? 1 : cfg->n_regions[a];
            if (cfg->n_cells[a] % (cs[i] * nr)) ok = false;
        }
        if (ok) out.push_back(cs[i]);
    }
    return out;
}

static bool auto_patch(const pic_config *cfg)
{
    return cfg->patch[0] == 0 && cfg->patch[1] == 0 && (cfg->dims == 2 || cfg->patch[2] == 0);
}

// segment capacities the autotuner tries (the first is the default)
static std::vector<int> cap_candidates(int dims)
{
    return dims == 2 ? std::vector<int>{SEG_CAP_2D, 1024, 4096} : std::vector<int>{SEG_CAP_3D, 2048, 8192};
}

// field tile widths the autotuner tries: the compiled widths no wider than
// the region (at least 8), the default first
static std::vector<int> tile_candidates(const pic_config *cfg)
{
    const bool filt = cfg->filter_passes > 0;
    const int nr = cfg->n_regions[0] < 1 ? 1 : cfg->n_regions[0];
    const int rs0 = cfg->n_cells[0] / nr;
    std::vector<int> out{yee_tile_x(cfg->dims, rs0, filt)};
    if (cfg->dims == 3 && filt) return out;
    const int top = cfg->dims == 2 ? 64 : 32;
    for (int t = top; t >= 8; t /= 2)
        if (t != out[0] && (t <= rs0 || t == 8)) out.push_back(t);
    return out;
}

struct Tuned {
    int patch, seg_cap, tile_x;
};
using TuneKey = std::tuple<int, int, int, int, int, int, int, int, int, int, int>;
static std::map<TuneKey, Tuned> g_tune_cache;
static std::mutex g_tune_mu;

// Milliseconds of 4 steps (after 2 warm-up steps) of `tc` in a scratch
// context beside c, on the caller's stream; 1e30 if it cannot be set up
// (for instance because the remaining HBM budget is too small).
static float trial_ms(pic_ctx *c, const pic_config &tc)
{
    pic_runtime trt = c->rt;
    trt.flags |= PIC_RT_NO_GRAPH;
    trt.max_runs = 1;
    // the scratch context lives beside this one: it may use what this
    // context's budget leaves, and its peak counts here
    trt.hbm_budget = c->rt.hbm_budget ? (c->rt.hbm_budget > c->bytes ? c->rt.hbm_budget - c->bytes : 1) : 0;
    pic_ctx *t = nullptr;
    if (pic_init(&tc, 1, &trt, &t) != PIC_OK) return 1e30f;
    c->peak_bytes = std::max(c->peak_bytes, c->bytes + t->peak_bytes);
    float ms = 1e30f;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    if (hipEventCreate(&e0) == hipSuccess && hipEventCreate(&e1) == hipSuccess && pic_step(t, 2) == PIC_OK &&
        hipEventRecord(e0, t->stream) == hipSuccess && pic_step(t, 4) == PIC_OK &&
        hipEventRecord(e1, t->stream) == hipSuccess && hipEventSynchronize(e1) == hipSuccess) {
        if (hipEventElapsedTime(&ms, e0, e1) != hipSuccess) ms = 1e30f;
    }
    if (e0) hipEventDestroy(e0);
    if (e1) hipEventDestroy(e1);
    c->peak_bytes = std::max(c->peak_bytes, c->bytes + t->peak_bytes);
    pic_free(t);
    return ms;
}

// The autotuner (patch = 0 on every axis): a staged search, each stage
// keeping the fastest of its trials -- the square patch edge with the
// default segment capacity and field tile, then the segment capacity with
// that patch, then the field tile width.  Results are cached per grid,
// precision, density class, region layout, filter and solver.
static Tuned autotune(pic_ctx *c, const pic_config *cfg)
{
    std::vector<int> cand = patch_candidates(cfg);
    if (cand.empty()) {
        int P[3];
        default_patch(cfg, P);
        return Tuned{P[0], 0, 0};
    }
    const long long n = cfg->particles ? cfg->particles->n : 0;
    long long ncell = 1;
    for (int a = 0; a < cfg->dims; ++a) ncell *= cfg->n_cells[a];
    const int ppcb = (int)std::lround(std::log2(std::max(1.0, (double)n / (double)ncell)));
    const TuneKey key{cfg->dims,          cfg->n_cells[0],   cfg->n_cells[1],     cfg->dims == 3 ? cfg->n_cells[2] : 1,
                      cfg->precision,     ppcb,              cfg->n_regions[0],   cfg->n_regions[1],
                      cfg->n_regions[2],  cfg->filter_passes, cfg->field_solver};
    {
        std::lock_guard<std::mutex> lk(g_tune_mu);
        auto it = g_tune_cache.find(key);
        if (it != g_tune_cache.end()) return it->second;
    }
    pic_config tc = *cfg;
    tc.max_steps = 0;
    auto set_patch = [&](int p) {
        tc.patch[0] = tc.patch[1] = p;
        tc.patch[2] = cfg->dims == 3 ? p : 1;
    };
    Tuned best{cand[0], cfg->seg_cap, cfg->field_tile_x};
    float best_ms = 1e30f;
    // stage 1: the patch edge (with one candidate, the baseline for the
    // later stages)
    tc.seg_cap = cfg->seg_cap;
    tc.field_tile_x = cfg->field_tile_x;
    const bool later = cfg->seg_cap == 0 || cfg->field_tile_x == 0;
    if (cand.size() > 1 || later)
        for (int p : cand) {
            set_patch(p);
            const float ms = trial_ms(c, tc);
            if (ms < best_ms) {
                best_ms = ms;
                best.patch = p;
            }
        }
    set_patch(best.patch);
    // stage 2: the segment capacity (unless the caller fixed it)
    if (cfg->seg_cap == 0) {
        const std::vector<int> caps = cap_candidates(cfg->dims);
        best.seg_cap = caps[0];
        for (size_t i = 1; i < caps.size(); ++i) {
            tc.seg_cap = caps[i];
            const float ms = trial_ms(c, tc);
            if (ms < best_ms) {
                best_ms = ms;
                best.seg_cap = caps[i];
            }
        }
        tc.seg_cap = best.seg_cap;
    }
    // stage 3: the field tile width (unless the caller fixed it)
    if (cfg->field_tile_x == 0) {
        const std::vector<int> txs = tile_candidates(cfg);
        best.tile_x = txs[0];
        for (size_t i = 1; i < txs.size(); ++i) {
            tc.field_tile_x = txs[i];
            const float ms = trial_ms(c, tc);
            if (ms < best_ms) {
                best_ms = ms;
                best.tile_x = txs[i];
            }
        }
    }
    std::lock_guard<std::mutex> lk(g_tune_mu);
    g_tune_cache[key] = best;
    return best;
}

static int gauss_field(pic_ctx *c, int slot, double *g);

// The largest power of two 2^e with unit * count * 2^e <= 2^62 and
// unit * 2^e <= 2^50: `count` contributions of magnitude at most `unit`,
// each rounded to a multiple of 2^-e, then sum without leaving the signed
// 64-bit range, and each scaled contribution stays inside the exact range
// of the rounding in to_fixed (|v| < 2^51).
static double fixed_scale(double unit, double count)
{
    if (!(unit > 0) || !std::isfinite(unit)) return 1.0;
    const double lim = std::min(std::ldexp(1.0, 62) / (unit * std::max(count, 1.0)), std::ldexp(1.0, 50) / unit);
    const int e = std::max(-1000, std::min(1000, (int)std::floor(std::log2(lim))));
    return std::ldexp(1.0, e);
}

// Fixed-point scales of the deterministic mode.  A node receives at most
// one contribution per particle and component per step.  A current
// contribution is q w times a sum of shape-factor differences of modulus at
// most 1, times d/dt (Jx, Jy, Jz in 3D) or v_z with |v_z| < 1 (Jz in 2D);
// a charge contribution is q w times shape factors of at most 1.  So |q| w_max
// max(1, d/dt) and |q| w_max bound them, and N of them still fit.  Scales
// depend only on the run's configuration and particle weights, so a run
// alone, in a batch, re-decomposed or resumed from its exported state sums
// with the same quantum.
static void fixed_point_scales(const pic_config *cfg, const Layout &L, RunDev &d)
{
    // the weights as the particle store keeps them (FP32 in the split form),
    // so that a run re-created from its exported particles gets the same scale
    double wmax = 0.0;
    if (cfg->particles && cfg->particles->w)
        for (long long i = 0; i < L.n_total; ++i) {
            const double w = cfg->particles->w[i];
            wmax = std::max(wmax, std::fabs(L.split ? (double)(float)w : w));
        }
    const double uq = std::fabs(cfg->q) * wmax;
    double dmax = 1.0;
    for (int a = 0; a < L.dims; ++a) dmax = std::max(dmax, d.d[a] / cfg->dt);
    const double n = (double)std::max<long long>(L.n_total, 1);
    d.junit = uq * dmax;
    d.jscale = fixed_scale(uq * dmax, n);
    d.jscale_inv = 1.0 / d.jscale;
    d.rscale = fixed_scale(uq, n);
    d.rscale_inv = 1.0 / d.rscale;
}

static int setup_run(pic_ctx *c, int slot, const pic_config *cfg_in)
{
    Run &r = c->runs[slot];
    pic_config tuned = *cfg_in;
    if (auto_patch(cfg_in)) {
        const Tuned t = autotune(c, cfg_in);
        tuned.patch[0] = tuned.patch[1] = t.patch;
        tuned.patch[2] = cfg_in->dims == 3 ? t.patch : 1;
        tuned.seg_cap = t.seg_cap;
        tuned.field_tile_x = t.tile_x;
    }
    const pic_config *cfg = &tuned;
    int P[3] = {cfg->patch[0], cfg->patch[1], cfg->patch[2]};
    Layout L;
    std::string why;
    int rc = make_layout(cfg, P, c->det, L, why);
    if (rc) return set_err(c, rc, "%s", why.c_str());
    if (c->rt.hbm_budget && c->bytes + L.bytes > c->rt.hbm_budget)
        return set_err(c, PIC_E_NOMEM, "HBM budget exceeded (%zu + %zu > %zu)", c->bytes, L.bytes, c->rt.hbm_budget);

    r = Run();
    r.dims = L.dims;
    r.split = L.split;
    r.prec = cfg->precision;
    r.pc = L.pc;
    r.px = fast_patch(L);
    r.ytx = cfg->field_tile_x > 0 ? cfg->field_tile_x : yee_tile_x(L.dims, L.rs[0], cfg->filter_passes > 0);
    r.ncell = L.n[0] * L.n[1] * L.n[2];
    r.total_ghosts = L.ghosts * L.n_regions;
    RunDev &d = r.rd;
    memset(&d, 0, sizeof d);
    d.dims = L.dims;
    d.prec = cfg->precision;
    d.filter = cfg->filter_passes;
    d.solver = cfg->field_solver;
    d.det = c->det ? 1 : 0;
    for (int a = 0; a < 3; ++a) {
        d.n[a] = L.n[a];
        d.P[a] = L.P[a];
        d.np[a] = L.np[a];
        d.nreg[a] = L.nreg[a];
        d.rs[a] = L.rs[a];
        d.ra[a] = L.ra[a];
        d.TA[a] = L.TA[a];
        d.d[a] = a < L.dims ? cfg->d[a] : 1.0;
        d.L[a] = d.n[a] * d.d[a];
    }
    d.n_patch = L.n_patch;
    d.n_regions = L.n_regions;
    d.rsize = L.rsize;
    d.tsz = L.tsz;
    d.cap_total = (int)L.cap_total;
    d.seg_max = L.seg_max;
    d.seg_cap = L.seg_cap;
    d.n_total = (int)L.n_total;
    d.ins_blocks = std::max(1, std::min(64, (int)(L.n_total / 65536)));
    d.ins_segs = 4;
    d.ghosts = L.ghosts;
    d.dt = cfg->dt;
    d.q = cfg->q;
    d.m = cfg->m;
    d.qmh = 0.5 * cfg->q / cfg->m * cfg->dt;
    d.f_qmh = (float)d.qmh;
    d.f_q = (float)cfg->q;
    for (int a = 0; a < 3; ++a) {
        d.f_dtd[a] = (float)(cfg->dt / d.d[a]);
        d.f_cj[a] = (float)(-cfg->q * d.d[a] / cfg->dt);
    }
    fixed_point_scales(cfg, L, d);
    const size_t rsz = L.split ? 4 : 8;
    const bool ids = cfg->track_ids != 0;
    bool ok = true;
    d.fld = (double *)run_alloc(c, r, (size_t)L.n_regions * F_NCOMP * L.rsize * 8);
    d.tiles = run_alloc(c, r, (size_t)L.seg_max * 3 * L.tsz * L.tile_esz);
    const size_t pb = (size_t)(L.n_patch + 1) * 4, sb = (size_t)(L.seg_max + 1) * 4;
    d.pseg = (int *)run_alloc(c, r, pb);
    d.pseg2 = (int *)run_alloc(c, r, pb);
    d.tot = (int *)run_alloc(c, r, pb);
    d.preg = (int *)run_alloc(c, r, pb);
    d.fill = (int *)run_alloc(c, r, pb);
    d.cpre = (int *)run_alloc(c, r, pb);
    d.spcnt = (int *)run_alloc(c, r, pb);
    d.sseg = (int *)run_alloc(c, r, sb);
    d.scnt = (int *)run_alloc(c, r, sb);
    d.spat = (int *)run_alloc(c, r, sb);
    d.sseg2 = (int *)run_alloc(c, r, sb);
    d.scnt2 = (int *)run_alloc(c, r, sb);
    d.spat2 = (int *)run_alloc(c, r, sb);
    d.ctl = (Ctl *)run_alloc(c, r, sizeof(Ctl));
    ok = d.fld && d.tiles && d.pseg && d.pseg2 && d.tot && d.preg && d.fill && d.cpre && d.spcnt && d.sseg && d.scnt && d.spat &&
         d.sseg2 && d.scnt2 && d.spat2 && d.ctl;
    make_store(c, r, d.st, L.cap_total, L.split, L.dims, ids, ok);
    make_store(c, r, d.lv, L.cap_total, L.split, L.dims, ids, ok);
    make_store(c, r, d.sp, L.n_total, L.split, L.dims, ids, ok);
    make_store(c, r, d.lo, L.n_total, L.split, L.dims, ids, ok);
    d.lpatch = (int *)run_alloc(c, r, (size_t)L.cap_total * 4);
    d.spatch = (int *)run_alloc(c, r, (size_t)std::max<long long>(L.n_total, 1) * 4);
    d.lopatch = (int *)run_alloc(c, r, (size_t)std::max<long long>(L.n_total, 1) * 4);
    d.nlv = (int *)run_alloc(c, r, sb);
    d.tflag = (int *)run_alloc(c, r, sb);
    ok = ok && d.lpatch && d.spatch && d.lopatch && d.nlv && d.tflag;
    d.spec = nullptr;
    d.spec_tw = nullptr;
    if (d.solver == PIC_SOLVER_PSATD) {
        d.spec = (double2 *)run_alloc(c, r, (size_t)SPEC_ARRAYS * r.ncell * 16);
        d.spec_tw = (double2 *)run_alloc(c, r, (size_t)SPEC_TW_LEN * 16);
        ok = ok && d.spec && d.spec_tw;
    }
    r.gauss0 = (double *)run_alloc(c, r, (size_t)r.ncell * 8);
    ok = ok && r.gauss0;
    r.bytes = 0;
    for (auto &b : r.bufs) r.bytes += b.bytes;
    if (!ok) {
        free_run(c, r);
        return set_err(c, PIC_E_NOMEM, "device allocation failed");
    }
    r.active = true;
    hipStream_t s = c->stream;
    HIPCHK(c, hipMemsetAsync(d.fld, 0, (size_t)L.n_regions * F_NCOMP * L.rsize * 8, s));
    HIPCHK(c, hipMemsetAsync(d.tiles, 0, (size_t)L.seg_max * 3 * L.tsz * L.tile_esz, s));
    HIPCHK(c, hipMemsetAsync(d.pseg, 0, pb, s));
    HIPCHK(c, hipMemsetAsync(d.spcnt, 0, pb, s));
    HIPCHK(c, hipMemsetAsync(d.sseg, 0, sb, s));
    HIPCHK(c, hipMemsetAsync(d.scnt, 0, sb, s));
    HIPCHK(c, hipMemsetAsync(d.nlv, 0, sb, s));
    HIPCHK(c, hipMemsetAsync(d.tflag, 0, sb, s));
    HIPCHK(c, hipMemsetAsync(d.ctl, 0, sizeof(Ctl), s));
    if (d.spec_tw) HIPCHK(c, launch_spec_twiddles(d.spec_tw, s));
    {
        Ctl init;
        memset(&init, 0, sizeof init);
        init.remaining[0] = init.remaining[1] =
            cfg->max_steps > 0 ? (int)std::min<int64_t>(cfg->max_steps, (1LL << 30)) : -1;
        HIPCHK(c, hipMemcpyAsync(d.ctl, &init, sizeof init, hipMemcpyHostToDevice, s));
        HIPCHK(c, hipStreamSynchronize(s));
    }
    r.target = cfg->max_steps > 0 ? cfg->max_steps : 0;
    r.par0 = c->par;
    if ((rc = upload_rd(c, slot))) return rc;

    // fields
    const int par = c->par;
    const int ncell = r.ncell;
    if (cfg->fields) {
        const pic_fields_in *f = cfg->fields;
        if (!f->E || !f->B || (f->kind != 0 && f->kind != 1)) return set_err(c, PIC_E_INVAL, "fields: E and B required, kind 0 or 1");
        Scratch tmp(c);
        double *stg = (double *)tmp.get((size_t)3 * ncell * 8);
        if (!stg) return set_err(c, PIC_E_NOMEM, "staging allocation failed");
        auto up = [&](const double *src, int c0) -> int {
            HIPCHK(c, hipMemcpyAsync(stg, src, (size_t)3 * ncell * 8, hipMemcpyHostToDevice, s));
            HIPCHK(c, launch_scatter_fields(c->d_runs, slot, ncell, stg, c0, s));
            HIPCHK(c, hipStreamSynchronize(s));
            return PIC_OK;
        };
        if ((rc = up(f->E, f_E(par)))) return rc;
        if (r.rd.solver == PIC_SOLVER_PSATD) {
            // E and B at the same time: B^n = B^0 (kind 0) or Bm^n (kind 1)
            const double *Bn = (f->kind == 1 && f->Bm) ? f->Bm : f->B;
            if ((rc = up(Bn, f_B(par)))) return rc;
            if ((rc = up(Bn, F_BM))) return rc;
        } else {
            if ((rc = up(f->B, f_B(par)))) return rc;
            if (f->kind == 1) {
                if ((rc = up(f->Bm ? f->Bm : f->B, F_BM))) return rc;
            }
        }
        HIPCHK(c, launch_ghosts(c->d_runs, slot, r.total_ghosts, f_E(par), 3, s));
        HIPCHK(c, launch_ghosts(c->d_runs, slot, r.total_ghosts, f_B(par), 3, s));
        if (f->kind == 0 && r.rd.solver != PIC_SOLVER_PSATD) HIPCHK(c, launch_half_faraday(c->d_runs, slot, ncell, par, s));
        HIPCHK(c, launch_ghosts(c->d_runs, slot, r.total_ghosts, f_B(par), 3, s));
        HIPCHK(c, launch_ghosts(c->d_runs, slot, r.total_ghosts, F_BM, 3, s));
    }

    // particles: FP64 staging -> spill store -> forced re-layout (binning)
    const long long n = L.n_total;
    if (n > 0) {
        const pic_particles_in *p = cfg->particles;
        if (!p->x || !p->y || (L.dims == 3 && !p->z) || !p->ux || !p->uy || !p->uz || !p->w)
            return set_err(c, PIC_E_INVAL, "particles: x, y, (z), ux, uy, uz, w required");
        const int nar = 7;
        Scratch tmp(c);
        const double *src[7] = {p->x, p->y, L.dims == 3 ? p->z : p->x, p->ux, p->uy, p->uz, p->w};
        double *dp[7];
        for (int i = 0; i < nar; ++i) {
            dp[i] = (double *)tmp.get((size_t)n * 8);
            if (!dp[i]) return set_err(c, PIC_E_NOMEM, "staging allocation failed");
            HIPCHK(c, hipMemcpyAsync(dp[i], src[i], (size_t)n * 8, hipMemcpyHostToDevice, s));
        }
        uint32_t *did = nullptr;
        if (p->id) {
            did = (uint32_t *)tmp.get((size_t)n * 4);
            if (!did) return set_err(c, PIC_E_NOMEM, "staging allocation failed");
            HIPCHK(c, hipMemcpyAsync(did, p->id, (size_t)n * 4, hipMemcpyHostToDevice, s));
        }
        HIPCHK(c, launch_convert(L.dims, L.split, c->d_runs, slot, (int)n, dp[0], dp[1], dp[2], dp[3], dp[4], dp[5],
                                 dp[6], did, s));
        HIPCHK(c, hipStreamSynchronize(s));
    }
    // binning: the first re-layout gathers the particles into their patch
    // segments, the second spreads each segment's storage order (see the
    // permutation in the re-layout kernel)
    if ((rc = relayout_one(c, slot, 1))) return rc;
    if ((rc = relayout_one(c, slot, 1))) return rc;
    if ((rc = check_run_err(c, slot))) {
        free_run(c, r);
        return rc;
    }
    r.steps = 0;
    if ((rc = gauss_field(c, slot, r.gauss0))) return rc;
    return PIC_OK;
}

// ------------------------------------------------------------------ classes
template <class V>
static int upload_vec(pic_ctx *c, const std::vector<V> &h, V *&d, size_t &cap)
{
    // grow to twice the size; shrink when a quarter is left in use, so the
    // lists of retired runs do not stay allocated
    if (h.size() > cap || !d || (cap > 64 && h.size() * 4 < cap)) {
        for (auto it = c->own.begin(); it != c->own.end(); ++it)
            if (it->p == d) {
                dev_free(c, *it);
                c->own.erase(it);
                break;
            }
        cap = std::max<size_t>(h.size(), 1) * 2;
        d = (V *)dev_alloc(c, cap * sizeof(V));
        if (!d) return set_err(c, PIC_E_NOMEM, "item list allocation failed");
        c->own.push_back({(void *)d, align256(cap * sizeof(V))});
    }
    if (!h.empty()) HIPCHK(c, hipMemcpyAsync(d, h.data(), h.size() * sizeof(V), hipMemcpyHostToDevice, c->stream));
    return PIC_OK;
}

static int rebuild_items(pic_ctx *c)
{
    for (auto &pc : c->pcls) pc.h.clear();
    for (auto &fc : c->fcls) {
        fc.hy.clear();
        fc.hp.clear();
        fc.slots.clear();
        fc.count_gx = 1;
        fc.move_gx = 1;
        fc.commit_gx = 1;
    }
    for (int slot = 0; slot < (int)c->runs.size(); ++slot) {
        Run &r = c->runs[slot];
        if (!r.active) continue;
        PushClass *pc = nullptr;
        for (auto &x : c->pcls)
            if (x.dims == r.dims && x.split == r.split && x.pc == r.pc && x.px == r.px) pc = &x;
        if (!pc) {
            c->pcls.push_back(PushClass{r.dims, r.pc, r.px, r.split});
            pc = &c->pcls.back();
        }
        const bool filt = r.rd.filter > 0;
        const int ytx = r.ytx;
        FieldClass *fc = nullptr;
        for (auto &x : c->fcls)
            if (x.dims == r.dims && x.split == r.split && x.tx == ytx && x.filt == filt && x.solver == r.rd.solver)
                fc = &x;
        if (!fc) {
            c->fcls.push_back(FieldClass{r.dims, r.split, ytx, filt, r.rd.solver});
            fc = &c->fcls.back();
        }
        const RunDev &d = r.rd;
        // push items: the run's block of (run, l) items, l = 0 .. seg_max
        // rounded up to a multiple of 8, starting at a multiple of 8 so that
        // item l runs on XCD l % 8; the kernel maps l to a segment from the
        // live segment count (see push_kernel)
        const int npad = (d.seg_max + 7) / 8 * 8;
        for (int l = 0; l < npad; ++l) pc->h.push_back(make_int2(slot, l));
        // yee items
        int shape[3];
        yee_tile_shape(r.dims, ytx, shape);
        const int tx = shape[0], ty = shape[1], tz = shape[2];
        const int ntiles = ((d.rs[0] + tx - 1) / tx) * ((d.rs[1] + ty - 1) / ty) * ((d.rs[2] + tz - 1) / tz);
        bool first = true;
        for (int reg = 0; reg < d.n_regions; ++reg)
            for (int t = 0; t < ntiles; ++t) {
                fc->hy.push_back(make_int4(slot, reg, t, first ? 1 : 0));
                first = false;
            }
        // post items
        for (int g = 0; g < r.total_ghosts; g += BLOCK) fc->hp.push_back(make_int4(slot, 0, g, 0));
        for (int sg = 0; sg < d.seg_max; sg += d.ins_segs) fc->hp.push_back(make_int4(slot, 1, sg, d.ins_segs));
        for (int b = 0; b < d.ins_blocks; ++b) fc->hp.push_back(make_int4(slot, 2, b, d.ins_blocks));
        fc->slots.push_back(slot);
        const int nsb = std::max(1, std::min(1024, (int)(d.n_total / (BLOCK * 64))));
        fc->count_gx = std::max(fc->count_gx, nsb);
        fc->move_gx = std::max(fc->move_gx, move_chunk_blocks(d.n_patch, d.n_total) + nsb);
        fc->commit_gx = std::max(fc->commit_gx, std::min(64, std::max(1, (d.seg_max + BLOCK) / BLOCK)));
    }
    int rc;
    for (auto &pc : c->pcls)
        if ((rc = upload_vec(c, pc.h, pc.d, pc.cap))) return rc;
    for (auto &fc : c->fcls) {
        if ((rc = upload_vec(c, fc.hy, fc.dy, fc.capy))) return rc;
        if ((rc = upload_vec(c, fc.hp, fc.dp, fc.capp))) return rc;
        if ((rc = upload_vec(c, fc.slots, fc.dslots, fc.caps))) return rc;
    }
    c->graphs_valid = false;
    return PIC_OK;
}

// ------------------------------------------------------------------ stepping
// ev0 / ev1 (may be null): recorded at the start of the first particle
// kernel and at the end of the last one
static hipError_t enqueue_push(pic_ctx *c, int par, hipStream_t s, hipEvent_t ev0 = nullptr,
                               hipEvent_t ev1 = nullptr)
{
    const size_t nc = c->pcls.size();
    for (size_t k = 0; k < nc; ++k) {
        auto &pc = c->pcls[k];
        hipError_t e = launch_push(pc.dims, pc.split, pc.px, pc.pc, c->det, c->d_runs, pc.d, (int)pc.h.size(), par, s,
                                   k == 0 ? ev0 : nullptr, k + 1 == nc ? ev1 : nullptr);
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}

static hipError_t enqueue_yee(pic_ctx *c, int par, hipStream_t s)
{
    for (auto &fc : c->fcls) {
        hipError_t e =
            launch_yee(fc.dims, fc.split, fc.tx, fc.filt, c->det, c->d_runs, fc.dy, (int)fc.hy.size(), par, s);
        if (e != hipSuccess) return e;
        if (fc.solver == PIC_SOLVER_PSATD)
            for (int slot : fc.slots) {
                e = launch_spectral(c->d_runs, slot, c->runs[slot].rd.dims, c->runs[slot].rd.n, par, s);
                if (e != hipSuccess) return e;
            }
    }
    return hipSuccess;
}

static hipError_t enqueue_post(pic_ctx *c, int par, hipStream_t s)
{
    for (auto &fc : c->fcls) {
        hipError_t e = launch_post(fc.dims, fc.split, c->d_runs, fc.dp, (int)fc.hp.size(), 1 - par, s);
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}

static hipError_t enqueue_step(pic_ctx *c, int par, hipStream_t s)
{
    hipError_t e = enqueue_push(c, par, s);
    if (e == hipSuccess) e = enqueue_yee(c, par, s);
    if (e == hipSuccess) e = enqueue_post(c, par, s);
    return e;
}

static hipError_t enqueue_relayout(pic_ctx *c, hipStream_t s)
{
    for (auto &fc : c->fcls) {
        if (fc.slots.empty()) continue;
        hipError_t e = launch_relayout(fc.dims, fc.split, c->d_runs, fc.dslots, (int)fc.slots.size(), fc.count_gx,
                                       fc.move_gx, fc.commit_gx, 0, s);
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}

static void drop_graphs(pic_ctx *c)
{
    for (hipGraphExec_t *g : {&c->g2, &c->g8, &c->gK, &c->grel}) {
        if (*g) hipGraphExecDestroy(*g);
        *g = nullptr;
    }
    c->graphs_valid = false;
}

static int build_graphs(pic_ctx *c)
{
    drop_graphs(c);
    if (!c->use_graph) return PIC_OK;
    // Each graph launch costs the GPU a gap of several microseconds, so the
    // common stretches of steps are captured whole: 2 and 8 steps, and a
    // full re-layout period with its check.  Steps come in pairs (E/B
    // buffer parity 0 then 1).
    const int K = c->relayout_every;
    for (int k = 0; k < 4; ++k) {
        hipGraph_t g = nullptr;
        const int nsteps = k == 0 ? 2 : (k == 1 ? 0 : (k == 2 ? 8 : K));
        HIPCHK(c, hipStreamBeginCapture(c->cap_stream, hipStreamCaptureModeThreadLocal));
        hipError_t e = hipSuccess;
        for (int i = 0; i < nsteps && e == hipSuccess; ++i) e = enqueue_step(c, i & 1, c->cap_stream);
        if (e == hipSuccess && (k == 1 || k == 3)) e = enqueue_relayout(c, c->cap_stream);
        hipError_t e2 = hipStreamEndCapture(c->cap_stream, &g);
        if (e != hipSuccess || e2 != hipSuccess) {
            if (g) hipGraphDestroy(g);
            return set_err(c, PIC_E_DEVICE, "graph capture failed: %s",
                           hipGetErrorString(e != hipSuccess ? e : e2));
        }
        hipGraphExec_t ex = nullptr;
        hipError_t e3 = hipGraphInstantiate(&ex, g, nullptr, nullptr, 0);
        hipGraphDestroy(g);
        if (e3 != hipSuccess) return set_err(c, PIC_E_DEVICE, "graph instantiate failed: %s", hipGetErrorString(e3));
        (k == 0 ? c->g2 : (k == 1 ? c->grel : (k == 2 ? c->g8 : c->gK))) = ex;
    }
    c->graphs_valid = true;
    return PIC_OK;
}

static bool any_active(pic_ctx *c)
{
    for (auto &r : c->runs)
        if (r.active) return true;
    return false;
}

static int run_par(const Run &r) { return r.par0 ^ (int)(r.steps & 1); }

// div_h E - rho of a run's current state into g (device, ncell doubles)
static int gauss_field(pic_ctx *c, int slot, double *g)
{
    Run &r = c->runs[slot];
    Scratch tmp(c);
    double *rho = (double *)tmp.get((size_t)r.ncell * 8);
    if (!rho) return set_err(c, PIC_E_NOMEM, "staging allocation failed");
    hipError_t e;
    Ctl ctl = read_ctl(c, slot, e);
    if (e == hipSuccess)
        e = launch_rho(r.dims, r.split, r.rd.det, c->d_runs, slot, r.rd.seg_max, ctl.nspill, r.ncell, rho, c->stream);
    if (e == hipSuccess) e = launch_gauss(c->d_runs, slot, r.ncell, run_par(r), rho, g, c->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
    if (e != hipSuccess) return set_err(c, PIC_E_DEVICE, "Gauss residual: %s", hipGetErrorString(e));
    return PIC_OK;
}


static void advance(pic_ctx *c, int nsteps)
{
    for (auto &r : c->runs)
        if (r.active) {
            r.issued += nsteps;
            r.steps = r.target > 0 ? std::min(r.issued, r.target) : r.issued;
        }
    c->step += nsteps;
    if (nsteps & 1) c->par ^= 1;
}

// ------------------------------------------------------------------ ABI
extern "C" {

const char *pic_strerror(int code)
{
    switch (code) {
    case PIC_OK: return "ok";
    case PIC_E_INVAL: return "invalid argument";
    case PIC_E_CONFIG: return "invalid configuration";
    case PIC_E_NOMEM: return "out of device memory or over the HBM budget";
    case PIC_E_DEVICE: return "HIP runtime error";
    case PIC_E_NUMERIC: return "numerical error (non-finite value or a move of a cell or more in one step)";
    case PIC_E_CAPACITY: return "no free run slot";
    case PIC_E_STATE: return "call not valid in the current state";
    case PIC_E_OVERFLOW: return "a particle store of the run overflowed";
    default: return "unknown error";
    }
}

const char *pic_last_error(pic_ctx *ctx) { return ctx ? ctx->err.c_str() : g_init_error.c_str(); }

int pic_mem_bytes(const pic_config *cfg, size_t *bytes)
{
    if (!cfg || !bytes) return set_err(nullptr, PIC_E_INVAL, "null argument");
    std::vector<std::array<int, 3>> shapes;
    if (auto_patch(cfg)) {
        for (int p : patch_candidates(cfg)) shapes.push_back({p, p, cfg->dims == 3 ? p : 1});
        if (shapes.empty()) {
            int P[3];
            default_patch(cfg, P);
            shapes.push_back({P[0], P[1], P[2]});
        }
    } else {
        shapes.push_back({cfg->patch[0], cfg->patch[1], cfg->patch[2]});
    }
    // with the autotuner, the worst of the patch edges and segment
    // capacities it may choose (smaller segments: more tiles)
    std::vector<int> caps{cfg->seg_cap};
    if (auto_patch(cfg) && cfg->seg_cap == 0) caps = cap_candidates(cfg->dims);
    size_t worst = 0;
    for (auto &sh : shapes)
        for (int cap : caps) {
            pic_config tc = *cfg;
            tc.seg_cap = cap;
            Layout L;
            std::string why;
            int rc = make_layout(&tc, sh.data(), true, L, why);
            if (rc) return set_err(nullptr, rc, "%s", why.c_str());
            worst = std::max(worst, L.bytes);
        }
    *bytes = worst;
    return PIC_OK;
}

void pic_free(pic_ctx *ctx)
{
    if (!ctx) return;
    hipStreamSynchronize(ctx->stream);
    drop_graphs(ctx);
    for (auto &r : ctx->runs) free_run(ctx, r);
    for (auto &b : ctx->own) dev_free(ctx, b);
    if (ctx->cap_stream) hipStreamDestroy(ctx->cap_stream);
    delete ctx;
}

int pic_init(const pic_config *cfgs, int32_t n_runs, const pic_runtime *rt, pic_ctx **out)
{
    g_init_error.clear();
    if (!out || n_runs < 0 || (n_runs > 0 && !cfgs)) return set_err(nullptr, PIC_E_INVAL, "null argument");
    *out = nullptr;
    int ndev = 0;
    if (hipGetDeviceCount(&ndev) != hipSuccess || ndev < 1) return set_err(nullptr, PIC_E_DEVICE, "no HIP device");
    // validate every config before touching the device
    for (int i = 0; i < n_runs; ++i) {
        int P[3] = {cfgs[i].patch[0], cfgs[i].patch[1], cfgs[i].patch[2]};
        if (auto_patch(&cfgs[i])) {
            std::vector<int> cand = patch_candidates(&cfgs[i]);
            if (cand.empty())
                default_patch(&cfgs[i], P);
            else
                P[0] = P[1] = P[2] = cand[0];
            if (cfgs[i].dims == 2) P[2] = 1;
        }
        Layout L;
        std::string why;
        int rc = make_layout(&cfgs[i], P, rt && rt->deterministic, L, why);
        if (rc) return set_err(nullptr, rc, "run %d: %s", i, why.c_str());
    }
    pic_ctx *c = new pic_ctx();
    if (rt) c->rt = *rt;
    if (hipGetDevice(&c->device) != hipSuccess) c->device = -1;
    c->det = c->rt.deterministic != 0;
    resolve_static_scratch(c->device);
    c->stream = (hipStream_t)c->rt.stream;
    c->max_runs = c->rt.max_runs > 0 ? std::max(c->rt.max_runs, n_runs) : std::max(n_runs, 1);
    c->use_graph = !(c->rt.flags & PIC_RT_NO_GRAPH);
    c->runs.resize(c->max_runs);
    if (hipStreamCreateWithFlags(&c->cap_stream, hipStreamNonBlocking) != hipSuccess) {
        delete c;
        return set_err(nullptr, PIC_E_DEVICE, "stream creation failed");
    }
    c->d_runs = (RunDev *)dev_alloc(c, sizeof(RunDev) * c->max_runs);
    c->d_slot1 = (int *)dev_alloc(c, 256);
    if (!c->d_runs || !c->d_slot1) {
        pic_free(c);
        return set_err(nullptr, PIC_E_NOMEM, "device allocation failed");
    }
    c->own.push_back({c->d_runs, align256(sizeof(RunDev) * c->max_runs)});
    c->own.push_back({c->d_slot1, 256});
    for (int i = 0; i < n_runs; ++i) {
        int rc = setup_run(c, i, &cfgs[i]);
        if (rc) {
            g_init_error = "run " + std::to_string(i) + ": " + c->err;
            pic_free(c);
            return rc;
        }
    }
    int rc = rebuild_items(c);
    if (rc) {
        g_init_error = c->err;
        pic_free(c);
        return rc;
    }
    if (hipStreamSynchronize(c->stream) != hipSuccess) {
        pic_free(c);
        return set_err(nullptr, PIC_E_DEVICE, "synchronisation failed");
    }
    *out = c;
    return PIC_OK;
}

int pic_step(pic_ctx *c, int32_t n_steps)
{
    if (!c || n_steps < 0) return set_err(c, PIC_E_INVAL, "bad argument");
    if (!any_active(c) || n_steps == 0) return PIC_OK;
    if (c->use_graph && !c->graphs_valid) {
        int rc = build_graphs(c);
        if (rc) return rc;
    }
    int left = n_steps;
    while (left > 0) {
        const int K = c->relayout_every;
        const int to_check = K - (int)(c->step % K);
        if (c->use_graph && c->gK && c->par == 0 && to_check == K && left >= K) {
            HIPCHK(c, hipGraphLaunch(c->gK, c->stream));   // a whole period and its check
            advance(c, K);
            left -= K;
            continue;
        }
        if (c->use_graph && c->g8 && c->par == 0 && left >= 8 && to_check >= 8) {
            HIPCHK(c, hipGraphLaunch(c->g8, c->stream));
            advance(c, 8);
            left -= 8;
        } else if (c->use_graph && c->g2 && c->par == 0 && left >= 2 && to_check >= 2) {
            HIPCHK(c, hipGraphLaunch(c->g2, c->stream));
            advance(c, 2);
            left -= 2;
        } else {
            HIPCHK(c, enqueue_step(c, c->par, c->stream));
            advance(c, 1);
            left -= 1;
        }
        if (c->step % K == 0) {
            if (c->use_graph && c->grel)
                HIPCHK(c, hipGraphLaunch(c->grel, c->stream));
            else
                HIPCHK(c, enqueue_relayout(c, c->stream));
        }
    }
    return PIC_OK;
}

int pic_run_steps(pic_ctx *c, int32_t run, int64_t *steps)
{
    if (!c || !steps || run < 0 || run >= (int)c->runs.size() || !c->runs[run].active)
        return set_err(c, PIC_E_INVAL, "bad run");
    *steps = c->runs[run].steps;
    return PIC_OK;
}

int pic_time_phases(pic_ctx *c, int32_t n_steps)
{
    if (!c || n_steps < 1) return PIC_E_INVAL;
    if (!any_active(c)) return PIC_OK;
    // n steps enqueued phase by phase with an event between phases and one
    // synchronisation at the end: the kernels run back to back as in a
    // normal step (the host stays ahead of the device), and the stream
    // waits ~200 us first while the host enqueues the opening steps, so
    // each interval holds its kernels only
    // phase events (4 per step and one more) and the particle kernel's own
    // start / end events (2 per step)
    std::vector<hipEvent_t> ev(6 * (size_t)n_steps + 1);
    const size_t kbase = 4 * (size_t)n_steps + 1;
    size_t made = 0;
    int rc = PIC_OK;
    for (; made < ev.size(); ++made)
        if (hipEventCreate(&ev[made]) != hipSuccess) break;
    auto fail_dev = [&](hipError_t e) { return set_err(c, PIC_E_DEVICE, "HIP: %s", hipGetErrorString(e)); };
    hipError_t e = made == ev.size() ? hipSuccess : hipErrorOutOfMemory;
    if (e == hipSuccess) e = launch_gate(200, c->stream);
    if (e == hipSuccess) e = hipEventRecord(ev[0], c->stream);
    for (int k = 0; k < n_steps && e == hipSuccess; ++k) {
        hipEvent_t *q = &ev[4 * (size_t)k];
        e = enqueue_push(c, c->par, c->stream, ev[kbase + 2 * (size_t)k], ev[kbase + 2 * (size_t)k + 1]);
        if (e == hipSuccess) e = hipEventRecord(q[1], c->stream);
        if (e == hipSuccess) e = enqueue_yee(c, c->par, c->stream);
        if (e == hipSuccess) e = hipEventRecord(q[2], c->stream);
        if (e == hipSuccess) e = enqueue_post(c, c->par, c->stream);
        if (e == hipSuccess) e = hipEventRecord(q[3], c->stream);
        if (e != hipSuccess) break;
        advance(c, 1);
        if (c->step % c->relayout_every == 0) e = enqueue_relayout(c, c->stream);
        if (e == hipSuccess) e = hipEventRecord(q[4], c->stream);
    }
    if (e == hipSuccess) e = hipEventSynchronize(ev[4 * (size_t)n_steps]);
    if (e == hipSuccess) {
        double sum[4] = {0, 0, 0, 0}, kern = 0.0;
        for (int k = 0; k < n_steps; ++k) {
            for (int i = 0; i < 4; ++i) {
                float ms = 0;
                hipEventElapsedTime(&ms, ev[4 * (size_t)k + i], ev[4 * (size_t)k + i + 1]);
                sum[i] += ms;
            }
            float ms = 0;
            hipEventElapsedTime(&ms, ev[kbase + 2 * (size_t)k], ev[kbase + 2 * (size_t)k + 1]);
            kern += ms;
        }
        for (int i = 0; i < 4; ++i) c->t_ms[i] = sum[i] / n_steps;
        c->t_push_kernel_ms = kern / n_steps;
    } else {
        rc = fail_dev(e);
    }
    for (size_t i = 0; i < made; ++i) hipEventDestroy(ev[i]);
    return rc;
}

static int field_comp(int bit, int par)
{
    if (bit < 3) return f_E(par) + bit;
    if (bit < 6) return F_BM + (bit - 3);
    if (bit < 9) return f_B(par) + (bit - 6);
    if (bit < 12) return F_J + (bit - 9);
    return -1;
}

int pic_fields(pic_ctx *c, int32_t run, uint32_t mask, double *dst, size_t dst_len, int32_t dst_on_device)
{
    if (!c || run < 0 || run >= (int)c->runs.size() || !c->runs[run].active || (!dst && mask))
        return set_err(c, PIC_E_INVAL, "bad argument");
    Run &r = c->runs[run];
    const size_t nc = (size_t)r.ncell;
    int ncomp = 0;
    for (int b = 0; b < 13; ++b)
        if (mask & (1u << b)) ++ncomp;
    if ((size_t)ncomp * nc > dst_len) return set_err(c, PIC_E_INVAL, "dst too small: need %zu", (size_t)ncomp * nc);
    HIPCHK(c, hipStreamSynchronize(c->stream));
    Scratch scr(c);
    double *tmp = (double *)scr.get(nc * 8);
    if (!tmp) return set_err(c, PIC_E_NOMEM, "staging allocation failed");
    size_t o = 0;
    int rc = PIC_OK;
    for (int b = 0; b < 13 && rc == PIC_OK; ++b) {
        if (!(mask & (1u << b))) continue;
        hipError_t e;
        if (b < 12) {
            e = launch_assemble(c->d_runs, run, r.ncell, field_comp(b, run_par(r)), tmp, c->stream);
        } else {
            Ctl ctl = read_ctl(c, run, e);
            if (e == hipSuccess)
                e = launch_rho(r.dims, r.split, r.rd.det, c->d_runs, run, r.rd.seg_max, ctl.nspill, r.ncell, tmp,
                               c->stream);
        }
        if (e == hipSuccess)
            e = hipMemcpyAsync(dst + o, tmp, nc * 8, dst_on_device ? hipMemcpyDeviceToDevice : hipMemcpyDeviceToHost,
                               c->stream);
        if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
        if (e != hipSuccess) rc = set_err(c, PIC_E_DEVICE, "field readout: %s", hipGetErrorString(e));
        o += nc;
    }
    if (rc) return rc;
    return check_run_err(c, run);
}

}  // extern "C"

// Device scratch of one diagnostics call: partial sums (max(2 nb, nk)
// doubles), the Gauss residual per node plus its block maxima (ncell + 2 nb
// doubles), the charge density (ncell doubles).
struct DiagScratch {
    double *part, *gb, *rho;
};

static void diag_sizes(const Run &r, int &nb, int &nk)
{
    nb = std::max(1, std::min(1024, (r.ncell + BLOCK - 1) / BLOCK));
    nk = r.rd.seg_max + 1;
}

static size_t diag_scratch_bytes(const Run &r, size_t off[3])
{
    int nb, nk;
    diag_sizes(r, nb, nk);
    off[0] = 0;
    off[1] = align256((size_t)std::max(2 * nb, nk) * 8);
    off[2] = off[1] + align256((size_t)r.ncell * 8 + (size_t)2 * nb * 8);
    return off[2] + align256((size_t)r.ncell * 8);
}

static int diag_impl(pic_ctx *c, int32_t run, pic_diag_t *out, const DiagScratch &ds);

extern "C" {

int pic_diag(pic_ctx *c, int32_t run, pic_diag_t *out)
{
    if (!c || !out || run < 0 || run >= (int)c->runs.size() || !c->runs[run].active)
        return set_err(c, PIC_E_INVAL, "bad argument");
    int nb, nk;
    diag_sizes(c->runs[run], nb, nk);
    Scratch scr(c);
    DiagScratch ds;
    ds.part = (double *)scr.get((size_t)std::max(2 * nb, nk) * 8);
    ds.gb = ds.part ? (double *)scr.get((size_t)c->runs[run].ncell * 8 + (size_t)2 * nb * 8) : nullptr;
    ds.rho = ds.gb ? (double *)scr.get((size_t)c->runs[run].ncell * 8) : nullptr;
    if (!ds.part || !ds.gb || !ds.rho) return set_err(c, PIC_E_NOMEM, "staging allocation failed");
    return diag_impl(c, run, out, ds);
}

int pic_diag_noalloc(pic_ctx *c, int32_t run, pic_diag_t *out)
{
    if (!c || !out || run < 0 || run >= (int)c->runs.size() || !c->runs[run].active)
        return set_err(c, PIC_E_INVAL, "bad argument");
    char *base = (char *)static_scratch(c->device);
    if (!base)
        return set_err(c, PIC_E_DEVICE, "pic_diag_noalloc: static scratch of device %d unavailable (%s)", c->device,
                       static_scratch_error(c->device));
    size_t off[3];
    const size_t need = diag_scratch_bytes(c->runs[run], off);
    if (need > STATIC_SCRATCH_BYTES)
        return set_err(c, PIC_E_NOMEM,
                       "pic_diag_noalloc: run %d needs %zu bytes of scratch; the static scratch holds %zu "
                       "(grids up to about 4.1 million cells)",
                       run, need, STATIC_SCRATCH_BYTES);
    DiagScratch ds{(double *)(base + off[0]), (double *)(base + off[1]), (double *)(base + off[2])};
    return diag_impl(c, run, out, ds);
}

}  // extern "C"

static int diag_impl(pic_ctx *c, int32_t run, pic_diag_t *out, const DiagScratch &ds)
{
    Run &r = c->runs[run];
    const RunDev &d = r.rd;
    memset(out, 0, sizeof *out);
    HIPCHK(c, hipStreamSynchronize(c->stream));
    hipError_t ce;
    Ctl ctl = read_ctl(c, run, ce);
    HIPCHK(c, ce);
    SegView sv;
    int rc0 = read_segments(c, run, ctl, sv);
    if (rc0) return rc0;
    std::vector<long long> per(d.n_patch, 0);
    std::vector<int> sp(ctl.nspill);
    if (ctl.nspill > 0) HIPCHK(c, hipMemcpy(sp.data(), d.spatch, sp.size() * 4, hipMemcpyDeviceToHost));
    long long n = 0;
    for (int k = 0; k < sv.nseg; ++k) {
        const int q = sv.spat[k];
        const long long l = std::min(sv.scnt[k], sv.sseg[k + 1] - sv.sseg[k]);
        if (q >= 0 && q < d.n_patch) per[q] += l;
        n += l;
    }
    for (int q : sp)
        if (q >= 0 && q < d.n_patch) per[q]++;
    n += ctl.nspill;
    out->step = r.steps;
    out->t = r.steps * d.dt;
    out->n_particles = n;
    if (d.n_patch > 0) {
        out->patch_min = *std::min_element(per.begin(), per.end());
        out->patch_max = *std::max_element(per.begin(), per.end());
        out->patch_mean = (double)n / d.n_patch;
    }
    const double dV = d.d[0] * d.d[1] * (d.dims == 3 ? d.d[2] : 1.0);
    int nb, nk;
    diag_sizes(r, nb, nk);
    double *part = ds.part;
    std::vector<double> h(std::max(2 * nb, nk));
    HIPCHK(c, launch_field_energy(c->d_runs, run, r.ncell, run_par(r), part, nb, c->stream));
    HIPCHK(c, hipMemcpyAsync(h.data(), part, 2 * nb * 8, hipMemcpyDeviceToHost, c->stream));
    HIPCHK(c, hipStreamSynchronize(c->stream));
    double ue = 0, ub = 0;
    for (int i = 0; i < nb; ++i) {
        ue += h[2 * i];
        ub += h[2 * i + 1];
    }
    HIPCHK(c, launch_kinetic(r.dims, r.split, c->d_runs, run, d.seg_max, ctl.nspill, part, c->stream));
    HIPCHK(c, hipMemcpyAsync(h.data(), part, (size_t)nk * 8, hipMemcpyDeviceToHost, c->stream));
    HIPCHK(c, hipStreamSynchronize(c->stream));
    double k = 0;
    for (int i = 0; i < nk; ++i) k += h[i];
    out->U_E = 0.5 * ue * dV;
    out->U_B = 0.5 * ub * dV;
    out->K = k * dV;
    for (int i = 0; i < 4; ++i) out->t_ms[i] = c->t_ms[i];
    out->t_push_kernel_ms = c->t_push_kernel_ms;
    {
        // Gauss-law residual against the initial state
        double *gb = ds.gb;
        double *rho = ds.rho;
        hipError_t e =
            launch_rho(r.dims, r.split, d.det, c->d_runs, run, d.seg_max, ctl.nspill, r.ncell, rho, c->stream);
        if (e == hipSuccess) e = launch_gauss(c->d_runs, run, r.ncell, run_par(r), rho, gb, c->stream);
        if (e == hipSuccess) e = launch_gauss_max(r.ncell, gb, r.gauss0, rho, gb + r.ncell, nb, c->stream);
        std::vector<double> hm(2 * nb);
        if (e == hipSuccess)
            e = hipMemcpyAsync(hm.data(), gb + r.ncell, (size_t)2 * nb * 8, hipMemcpyDeviceToHost, c->stream);
        if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
        if (e != hipSuccess) return set_err(c, PIC_E_DEVICE, "Gauss residual: %s", hipGetErrorString(e));
        double dg = 0.0, rm = 0.0;
        for (int i = 0; i < nb; ++i) {
            dg = std::max(dg, hm[2 * i]);
            rm = std::max(rm, hm[2 * i + 1]);
        }
        out->gauss_residual = rm > 0.0 ? dg / rm : dg;
    }
    out->n_relayout = ctl.n_relayout;
    out->n_spill = ctl.nspill;
    out->err_flags = ctl.err;
    for (int a = 0; a < 3; ++a) out->patch[a] = d.P[a];
    out->kernel_path[0] = r.px;
    out->kernel_path[1] = r.pc;
    out->kernel_path[2] = r.ytx;
    out->seg_cap = d.seg_cap;
    out->kernel_path[3] = d.det;
    out->det_quantum[0] = d.det ? d.jscale_inv : 0.0;
    out->det_quantum[1] = d.det ? d.rscale_inv : 0.0;
    out->device_bytes = (int64_t)c->bytes;
    out->device_bytes_peak = (int64_t)c->peak_bytes;
    return check_run_err(c, run);
}

extern "C" {

int pic_particles(pic_ctx *c, int32_t run, pic_particles_out *out)
{
    if (!c || !out || run < 0 || run >= (int)c->runs.size() || !c->runs[run].active)
        return set_err(c, PIC_E_INVAL, "bad argument");
    Run &r = c->runs[run];
    const RunDev &d = r.rd;
    HIPCHK(c, hipStreamSynchronize(c->stream));
    hipError_t ce;
    Ctl ctl = read_ctl(c, run, ce);
    HIPCHK(c, ce);
    SegView sv;
    int rc0 = read_segments(c, run, ctl, sv);
    if (rc0) return rc0;
    std::vector<int> off(sv.nseg + 1);
    long long n = 0;
    for (int k = 0; k < sv.nseg; ++k) {
        off[k] = (int)n;
        n += std::min(sv.scnt[k], sv.sseg[k + 1] - sv.sseg[k]);
    }
    off[sv.nseg] = (int)n;
    n += ctl.nspill;
    out->n = n;
    if (out->capacity < n) return set_err(c, PIC_E_INVAL, "capacity %lld < %lld particles", (long long)out->capacity, n);
    if (n == 0) return check_run_err(c, run);
    const size_t nn = (size_t)n;
    Scratch scr(c);
    auto mk = [&](size_t bytes) -> void * { return scr.get(bytes); };
    double *dx[7] = {nullptr};
    double *hx[7] = {out->x, out->y, out->z, out->ux, out->uy, out->uz, out->w};
    bool ok = true;
    for (int i = 0; i < 7; ++i)
        if (hx[i]) {
            dx[i] = (double *)mk(nn * 8);
            ok = ok && dx[i];
        }
    uint32_t *did = out->id ? (uint32_t *)mk(nn * 4) : nullptr;
    int *dpat = out->patch ? (int *)mk(nn * 4) : nullptr;
    int *doff = (int *)mk(off.size() * 4);
    ok = ok && (!out->id || did) && (!out->patch || dpat) && doff;
    int rc = PIC_OK;
    if (!ok) rc = set_err(c, PIC_E_NOMEM, "staging allocation failed");
    hipError_t e = hipSuccess;
    if (!rc) e = hipMemcpyAsync(doff, off.data(), off.size() * 4, hipMemcpyHostToDevice, c->stream);
    if (!rc && e == hipSuccess)
        e = launch_export(r.dims, r.split, c->d_runs, run, d.seg_max, ctl.nspill, doff, dx[0], dx[1], dx[2], dx[3], dx[4],
                          dx[5], dx[6], did, dpat, c->stream);
    for (int i = 0; i < 7 && !rc && e == hipSuccess; ++i)
        if (dx[i]) e = hipMemcpyAsync(hx[i], dx[i], nn * 8, hipMemcpyDeviceToHost, c->stream);
    if (!rc && e == hipSuccess && did) e = hipMemcpyAsync(out->id, did, nn * 4, hipMemcpyDeviceToHost, c->stream);
    if (!rc && e == hipSuccess && dpat) e = hipMemcpyAsync(out->patch, dpat, nn * 4, hipMemcpyDeviceToHost, c->stream);
    if (!rc && e == hipSuccess) e = hipStreamSynchronize(c->stream);
    if (!rc && e != hipSuccess) rc = set_err(c, PIC_E_DEVICE, "particle export: %s", hipGetErrorString(e));
    if (rc) return rc;
    return check_run_err(c, run);
}

int pic_admit(pic_ctx *c, const pic_config *cfg, int32_t *run_id)
{
    if (!c || !cfg || !run_id) return set_err(c, PIC_E_INVAL, "null argument");
    int slot = -1;
    for (int i = 0; i < (int)c->runs.size(); ++i)
        if (!c->runs[i].active) {
            slot = i;
            break;
        }
    if (slot < 0) return set_err(c, PIC_E_CAPACITY, "all %d run slots are taken", (int)c->runs.size());
    int rc = setup_run(c, slot, cfg);
    if (rc) {
        if (c->runs[slot].active) free_run(c, c->runs[slot]);
        return rc;
    }
    if ((rc = rebuild_items(c))) return rc;
    HIPCHK(c, hipStreamSynchronize(c->stream));
    *run_id = slot;
    return PIC_OK;
}

int pic_retire(pic_ctx *c, int32_t run)
{
    if (!c || run < 0 || run >= (int)c->runs.size() || !c->runs[run].active)
        return set_err(c, PIC_E_INVAL, "bad run");
    HIPCHK(c, hipStreamSynchronize(c->stream));
    free_run(c, c->runs[run]);
    return rebuild_items(c);
}

}  // extern "C"
