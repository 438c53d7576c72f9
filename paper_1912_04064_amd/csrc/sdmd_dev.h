// sdmd_dev.h -- device-side data layout shared by the kernels and the host
// runtime of the SDMD PIC library (gfx950).
//
// Layout in HBM (one run):
//   regions  : FP64, all regions of the run back to back,
//              [region][component 0..17][z][y][x] with GH ghost layers per
//              side (none along z in 2D).  Components: E (two buffers, 3
//              each), B (two buffers, 3 each), Bm (B time-centred at t^n),
//              J (current of the last step).  E and B are double-buffered so
//              the fused Ampere/Faraday kernel can recompute a one-node halo
//              of E^{n+1} without reading values another workgroup already
//              overwrote.
//   particles: SoA in segments.  A patch owns 1..K consecutive segments
//              (segments [pseg[p], pseg[p+1])); a re-layout gives a patch
//              as many segments as it needs to keep each at most seg_cap
//              live particles, so a dense patch is worked on by several
//              workgroups at once.  Segment s owns slots [sseg[s],
//              sseg[s+1]) of which the first scnt[s] are live.  A second
//              store with the same segments receives each segment's leavers
//              (at most scnt[s], so they always fit) and serves as the
//              scratch of a re-layout; a third one ("spill") parks
//              particles that found their destination segment full until
//              the next re-layout, and a fourth takes those parked
//              particles when they re-enter.
//   tiles    : per segment, 3 current components on the nodes its patch's
//              particles can reach, [segment][component][z][y][x], extent
//              P+5 per axis, origin = patch origin - 2 (FP32 in the split
//              form, FP64 in the plain form; 64-bit fixed point in the
//              deterministic mode, see to_fixed).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace sdmd {

constexpr int GH = 2;          // ghost layers around each region
constexpr int F_E0 = 0;        // E, buffer 0 (3 components)
constexpr int F_B0 = 6;        // B, buffer 0 (3 components)
constexpr int F_BM = 12;       // Bm
constexpr int F_J = 15;        // J
constexpr int F_NCOMP = 18;
__host__ __device__ inline int f_E(int par) { return F_E0 + 3 * par; }
__host__ __device__ inline int f_B(int par) { return F_B0 + 3 * par; }

constexpr int BLOCK = 256;     // threads per workgroup of the step kernels
constexpr int SPEC_ARRAYS = 5;   // spectral solver: the 9 real E, B, J components, two per complex array
constexpr int SPEC_TW_LEN = 2048;   // spectral solver: longest transform, and entries of the twiddle tables

// A re-layout moves each patch's particles in chunks of MOVE_CHUNK, one
// workgroup per chunk; at most n_patch + ceil(N / MOVE_CHUNK) chunks exist.
constexpr int MOVE_CHUNK = 4096;
__host__ __device__ inline int move_chunk_blocks(int n_patch, long long n_total)
{
    return n_patch + (int)((n_total + MOVE_CHUNK - 1) / MOVE_CHUNK);
}

// error flag bits (Ctl::err)
constexpr int ERR_NONFINITE = 1;
constexpr int ERR_MOVE = 2;
constexpr int ERR_CAPACITY = 4;
constexpr int ERR_RANGE = 8;

// precision traits
struct FP64 {
    using real = double;
    static constexpr bool split = false;
};
struct F32S {
    using real = float;
    static constexpr bool split = true;
};

// one particle store, SoA.  pos: global position (FP64 form) or in-cell
// offset xi in [0,1) (split form).  cell: split form only, the cell inside
// the owning patch packed as lx | ly << 5 | lz << 10.
struct Store {
    void *pos[3];
    uint16_t *cell;
    void *u[3];
    void *w;
    uint32_t *id;   // null when ids are not tracked
};

// per-run device counters
// Per-step counters are kept twice, indexed by the parity of the step (the
// E/B buffer parity at its start): kernels of step s use entry s & 1 only,
// and one workgroup of the field kernel of step s prepares entry 1 - (s & 1)
// for step s + 1.  No kernel needs to know which of its workgroups ends last.
struct Ctl {
    int nleave[2];    // particles appended to the overflow leaver store in the step
    int nspill;       // particles parked in the spill store
    int err;          // ERR_* bits, sticky
    int relayout;     // set by the re-layout planner when a re-layout runs
    int n_relayout;   // re-layouts done
    int max_spill;    // largest nspill seen
    int nseg;         // segments in use
    int remaining[2]; // steps left at the start of the step (-1: unlimited);
                      // 0 makes every kernel skip the run
    int pad[2];
};

struct RunDev {
    int dims, prec;
    int n[3];            // cells per axis (n[2] = 1 in 2D)
    int P[3];            // cells per patch per axis (1 in 2D z)
    int np[3];           // patches per axis
    int n_patch;
    int nreg[3];         // regions per axis
    int rs[3];           // region interior cells per axis
    int ra[3];           // region allocated nodes per axis (rs + 2 GH; 1 in 2D z)
    int n_regions;
    long long rsize;     // nodes per component per region
    int TA[3];           // tile extent per axis (P + 5; 1 in 2D z)
    int tsz;             // nodes per tile component
    int cap_total;       // slots of the patch store
    int seg_max;         // segment slots allocated
    int seg_cap;         // live particles per segment a re-layout aims at
    int n_total;         // particles of the run
    int ins_blocks;      // workgroups inserting the overflow leavers
    int ins_segs;        // segments per leaver-insert workgroup
    int ghosts;          // ghost nodes per region
    int filter;          // binomial current filter passes (0 = off)
    int solver;          // 0 Yee, 1 spectral (PSATD)
    int det;             // deterministic mode: J and rho summed in 64-bit fixed point
    double d[3], L[3];
    double dt, q, m;
    double qmh;          // (q/m) dt/2
    double jscale, jscale_inv;   // deterministic mode: J contribution -> fixed point, and back
    double junit;        // bound on one current contribution, |q| w_max max(1, d/dt)
    double rscale, rscale_inv;   // the same for the charge density
    float f_qmh;
    float f_dtd[3];      // dt / d  (split form displacement in cells per unit velocity)
    float f_cj[3];       // -q d / dt (Esirkepov prefactor, times w)
    float f_q;
    double *fld;         // regions
    void *tiles;
    int *pseg;           // [n_patch + 1] first segment of each patch
    int *sseg, *scnt;    // [seg_max + 1] first slot, [seg_max] live count of each segment
    int *spat;           // [seg_max] patch of each segment
    int *pseg2, *sseg2, *scnt2, *spat2;   // re-layout: the new segment layout
    int *tot, *preg, *fill;               // re-layout: per-patch totals, patch-store part, spill fill
    int *spcnt;                           // [n_patch] particles parked in the spill store for the patch
    int *cpre;                            // re-layout: first move chunk of each patch [n_patch + 1]
    Store st, lv, sp;    // patch store, leaver / scratch store, spill store
    int *lpatch, *spatch;
    int *nlv;            // [seg_max] leavers of each segment this step, in lv at sseg[s]
    int *tflag;          // [seg_max] 1 when the segment's tile in HBM may hold non-zero values
    double2 *spec;       // spectral solver: SPEC_ARRAYS complex arrays [z][y][x] of the grid (components packed in pairs)
    double2 *spec_tw;    // spectral solver: e^{-2 pi i k / N}, k < N/2, for every N = 2..SPEC_TW_LEN, the table of N from N/2 - 1
    Store lo;            // overflow leavers (parked particles re-entering)
    int *lopatch;
    Ctl *ctl;
};

// ---------------------------------------------------------------- helpers
// Device pointers read from memory (the fields of RunDev and Store) are
// generic to the compiler, which then emits flat memory instructions.  A flat
// instruction also counts against the LDS wait counter, so every wait for an
// LDS read would also wait for outstanding HBM loads, and a prefetch could
// never stay in flight across LDS work.  Hot HBM accesses go through global
// (address space 1) pointers instead.
#define SDMD_GLOBAL __attribute__((address_space(1)))
template <class V>
__device__ __forceinline__ SDMD_GLOBAL V *gp(V *p)
{
    return (SDMD_GLOBAL V *)p;
}
template <class V>
__device__ __forceinline__ const SDMD_GLOBAL V *gp(const V *p)
{
    return (const SDMD_GLOBAL V *)p;
}

__device__ __forceinline__ long long rindex(const RunDev &r, int li, int lj, int lk)
{
    const int gz = (r.dims == 3) ? GH : 0;
    return (long long)(li + GH) + (long long)r.ra[0] * ((lj + GH) + (long long)r.ra[1] * (lk + gz));
}

__device__ __forceinline__ double *rcomp(const RunDev &r, int region, int comp)
{
    return r.fld + ((long long)region * F_NCOMP + comp) * r.rsize;
}

// i mod n for i in [-n, 2n).  Every caller steps at most a few nodes
// (the 5-node deposition frame, the ghost layers, the filter margin: <= 4)
// outside [0, n), and n >= 4 because a patch holds at least 4 cells per
// axis; two compares replace an integer division.
__device__ __forceinline__ int wrap1(int i, int n)
{
    i = i < 0 ? i + n : i;
    return i >= n ? i - n : i;
}

// Deterministic mode.  A floating-point sum depends on the order of its
// terms, and the order in which the LDS and global atomics of a deposition
// land is set by timing.  Integer addition is associative, so each
// contribution is rounded once to the nearest integer multiple of
// 1/scale (scale a power of two chosen per run so that no sum of all its
// particles' contributions can leave the 64-bit range) and summed as a
// 64-bit integer: the total is then the same whatever the order, the
// segment split or the decomposition.  v is the contribution times scale,
// |v| < 2^51: adding 1.5 * 2^52 leaves the integer nearest v in the low
// bits of the sum's significand.
__device__ __forceinline__ unsigned long long to_fixed(double v)
{
    const double t = v + 6755399441055744.0;
    return (unsigned long long)(__double_as_longlong(t) - 0x4338000000000000LL);
}

// quadratic B-spline weights at nodes -1, 0, +1 for offset d in [-1/2, 1/2]
template <class R>
__device__ __forceinline__ void shape3(R d, R &w0, R &w1, R &w2)
{
    R a = R(0.5) - d, b = R(0.5) + d;
    w0 = R(0.5) * a * a;
    w1 = R(0.75) - d * d;
    w2 = R(0.5) * b * b;
}

}  // namespace sdmd
