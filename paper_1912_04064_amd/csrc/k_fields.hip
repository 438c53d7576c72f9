// k_fields.hip -- region-side kernels of the SDMD step.
//
//   yee_kernel   : transfer (i) of section 2.2 fused with the optional
//                  binomial current filter and the Yee update (section 3.2).  For every node of its tile (plus a
//                  one-node high halo) a workgroup sums the current of the
//                  patch tiles covering that node (at most 2 patches per
//                  axis when P >= 5, fixed order, FP64 sum), applies Ampere,
//                  keeps E^{n+1} of tile and halo in LDS, then applies
//                  Faraday and forms Bm^{n+1} on the tile.  E and B are read
//                  from buffer `par` and written to buffer 1-par.
//   post_kernel  : region ghost synchronisation of the new E, B, Bm
//                  (section 2.1 "Sync", between regions) and, in the same
//                  launch, insertion of the particles that left their patch.
//                  The per-run step bookkeeping (budget, overflow and spill
//                  counters) is done by one workgroup of yee_kernel.
//   init / readout helpers.
#include <type_traits>

#include "launch.h"
#include "part.h"
#include "sdmd_dev.h"

namespace sdmd {

// --------------------------------------------------------------- J gather
// The current at a node is the sum, over the segment tiles of every patch
// whose node range [p0-2, p0+P+2] covers the node (periodic), in a fixed
// order (patches by offset, then segments).  A workgroup gathers a box of
// nodes; it first tabulates, per box column / row / layer, the offset of the
// node inside its patch and the index of that patch among the patches that
// cover the box (one division per axis entry instead of per node), and the
// segment range of each covering patch, so the per-node work is LDS lookups
// and the tile loads.
__device__ __forceinline__ int floordiv(int g, int P) { return (g + 8 * P) / P - 8; }   // g >= -8P

// i mod n for any i (table entries of tiny periodic grids wrap more than once)
__device__ __forceinline__ int wrapm(int i, int n)
{
    i %= n;
    return i < 0 ? i + n : i;
}

// covering patches per axis over a box of extent E: at most (E-1)/P + 2
// patches hold the box's nodes, plus one neighbour on each side (P >= 4)
constexpr int cover_bound(int E) { return (E - 1) / 4 + 4; }

struct GatherBox {
    int org[3];   // global (unwrapped) coordinate of the box's first node per axis
    int ext[3];   // box extent per axis
    int pu0[3];   // first covering patch (unwrapped) per axis
    int nc[3];    // covering patches per axis
};

template <int DIM, int AXM, int NCM, int NT>
__device__ __forceinline__ void gather_tables(const RunDev &rd, const GatherBox &b, int2 (*s_ax)[AXM], int2 *s_rng,
                                              int tid)
{
    const int P[3] = {rd.P[0], rd.P[1], DIM == 3 ? rd.P[2] : 1};
    const int nax = b.ext[0] + b.ext[1] + (DIM == 3 ? b.ext[2] : 0);
    for (int t = tid; t < nax; t += NT) {
        const int a = t < b.ext[0] ? 0 : (t < b.ext[0] + b.ext[1] ? 1 : 2);
        const int e = t - (a == 0 ? 0 : (a == 1 ? b.ext[0] : b.ext[0] + b.ext[1]));
        const int gu = b.org[a] + e;
        const int pu = floordiv(gu, P[a]);
        s_ax[a][e] = make_int2(gu - pu * P[a], pu - b.pu0[a]);
    }
    if (DIM == 2 && tid == 0) s_ax[2][0] = make_int2(0, 0);
    const SDMD_GLOBAL int *pseg = gp(rd.pseg);
    const int ncov = b.nc[0] * b.nc[1] * b.nc[2];
    for (int t = tid; t < ncov; t += NT) {
        const int cx = t % b.nc[0], cy = (t / b.nc[0]) % b.nc[1], cz = t / (b.nc[0] * b.nc[1]);
        const int qx = wrapm(b.pu0[0] + cx, rd.np[0]), qy = wrapm(b.pu0[1] + cy, rd.np[1]);
        const int qz = DIM == 3 ? wrapm(b.pu0[2] + cz, rd.np[2]) : 0;
        const int q = qx + rd.np[0] * (qy + rd.np[1] * qz);
        // a patch whose one segment holds no current this step (a vacuum
        // patch: the particle kernel left its tile at zero) is skipped
        const int k0 = pseg[q], k1 = pseg[q + 1];
        s_rng[t] = make_int2(k0, (k1 - k0 == 1 && gp(rd.tflag)[k0] == 0) ? k0 : k1);
    }
}

// Sum of tile values: FP64 over FP32 / FP64 tiles; in the deterministic
// mode 64-bit integers (wrapping: only the total has to be in range),
// converted once at the end.
template <class R>
struct TileSum {
    using A = double;
    static __device__ __forceinline__ A of(R v) { return (double)v; }
    static __device__ __forceinline__ double result(A s, const RunDev &) { return s; }
};
template <>
struct TileSum<long long> {
    using A = unsigned long long;
    static __device__ __forceinline__ A of(long long v) { return (unsigned long long)v; }
    static __device__ __forceinline__ double result(A s, const RunDev &rd) { return (double)(long long)s * rd.jscale_inv; }
};

// J at box node (ex, ey, ez): the sum over the covering patches (z, y, x
// ascending) and their segments (ascending) of the segment tiles.
//
// With patches of at least 5 cells a node lies within two nodes of at most
// one edge of its patch per axis, so at most two patches per axis cover it.
// The first SEGU segments of each of those 2^DIM candidates are loaded
// before any is summed -- an absent one reads the first word of the tile
// store instead and is discarded -- so the whole sum waits on memory once
// rather than once per segment; further segments of a heavy patch follow
// in a loop.  The order of the additions is the same in both forms.
template <int DIM, int AXM, int SEGU, class R>
__device__ __forceinline__ void gather_J(const RunDev &rd, const SDMD_GLOBAL R *__restrict__ tiles,
                                         const GatherBox &b, const int2 (*s_ax)[AXM], const int2 *s_rng, int ex,
                                         int ey, int ez, double J[3])
{
    const int P[3] = {rd.P[0], rd.P[1], DIM == 3 ? rd.P[2] : 1};
    const int2 X = s_ax[0][ex], Y = s_ax[1][ey], Z = DIM == 3 ? s_ax[2][ez] : make_int2(0, 0);
    const int l[3] = {X.x, Y.x, Z.x}, c[3] = {X.y, Y.y, Z.y};
    int lo[3] = {0, 0, 0}, hi[3] = {0, 0, 0};
#pragma unroll
    for (int a = 0; a < DIM; ++a) {
        lo[a] = l[a] <= 2 ? -1 : 0;
        hi[a] = l[a] >= P[a] - 2 ? 1 : 0;
    }
    const long long tsz = rd.tsz;
    const int TA0 = rd.TA[0], TA1 = rd.TA[1];
    using S = TileSum<R>;
    typename S::A s0 = 0, s1 = 0, s2 = 0;
    const bool wide = SEGU > 0 && P[0] >= 5 && P[1] >= 5 && (DIM == 2 || P[2] >= 5);
    if (wide) {
        if constexpr (SEGU > 0) {
            constexpr int NC = 1 << DIM;
            int2 rg[NC];
            int off[NC];
            R v[NC][SEGU][3];
#pragma unroll
            for (int k = 0; k < NC; ++k) {
                const int o[3] = {lo[0] + (k & 1), lo[1] + ((k >> 1) & 1), DIM == 3 ? lo[2] + ((k >> 2) & 1) : 0};
                const bool in = o[0] <= hi[0] && o[1] <= hi[1] && (DIM == 2 || o[2] <= hi[2]);
                // o is in [-1, 1] per axis: the table holds one patch beyond the
                // box on every side, so the read is in range even when !in
                const int2 r = s_rng[((c[2] + o[2]) * b.nc[1] + (c[1] + o[1])) * b.nc[0] + (c[0] + o[0])];
                rg[k] = make_int2(r.x, in ? r.y : r.x);
                off[k] = ((DIM == 3 ? l[2] - o[2] * P[2] + 2 : 0) * TA1 + (l[1] - o[1] * P[1] + 2)) * TA0 +
                         (l[0] - o[0] * P[0] + 2);
#pragma unroll
                for (int j = 0; j < SEGU; ++j) {
                    const bool ok = rg[k].x + j < rg[k].y;
                    const SDMD_GLOBAL R *t = tiles + (ok ? (long long)(rg[k].x + j) * 3 * tsz + off[k] : 0ll);
                    v[k][j][0] = t[0];
                    v[k][j][1] = t[tsz];
                    v[k][j][2] = t[2 * tsz];
                }
            }
#pragma unroll
            for (int k = 0; k < NC; ++k) {
#pragma unroll
                for (int j = 0; j < SEGU; ++j)
                    if (rg[k].x + j < rg[k].y) {
                        s0 += S::of(v[k][j][0]);
                        s1 += S::of(v[k][j][1]);
                        s2 += S::of(v[k][j][2]);
                    }
                for (int sg = rg[k].x + SEGU; sg < rg[k].y; ++sg) {
                    const SDMD_GLOBAL R *t = tiles + (long long)sg * 3 * tsz + off[k];
                    s0 += S::of(t[0]);
                    s1 += S::of(t[tsz]);
                    s2 += S::of(t[2 * tsz]);
                }
            }
        }
    } else {
        for (int oz = lo[2]; oz <= hi[2]; ++oz)
            for (int oy = lo[1]; oy <= hi[1]; ++oy)
                for (int ox = lo[0]; ox <= hi[0]; ++ox) {
                    const int2 r = s_rng[((c[2] + oz) * b.nc[1] + (c[1] + oy)) * b.nc[0] + (c[0] + ox)];
                    const int tx = l[0] - ox * P[0] + 2;
                    const int ty = l[1] - oy * P[1] + 2;
                    const int tz = DIM == 3 ? l[2] - oz * P[2] + 2 : 0;
                    const int of = (tz * TA1 + ty) * TA0 + tx;
                    for (int sg = r.x; sg < r.y; ++sg) {
                        const SDMD_GLOBAL R *t = tiles + (long long)sg * 3 * tsz + of;
                        s0 += S::of(t[0]);
                        s1 += S::of(t[tsz]);
                        s2 += S::of(t[2 * tsz]);
                    }
                }
    }
    J[0] = S::result(s0, rd);
    J[1] = S::result(s1, rd);
    J[2] = S::result(s2, rd);
}

// Yee tile shapes: one node per thread, x extent TX chosen per run from the
// region width (64 for wide regions; 32, 16 or 8 when regions are as small
// as patches, so that a tile does not straddle mostly empty space).  Wide 2D
// regions take 64 x 8 tiles of 512 threads (the recomputed high halo is 14 %
// of the tile instead of 27 % at 64 x 4); the others use BLOCK threads.
constexpr int yee_block(int dims, int tx) { return dims == 2 && tx == 64 ? 2 * BLOCK : BLOCK; }

template <int DIM, int TX>
struct YeeTile;
template <int TX>
struct YeeTile<2, TX> {
    static constexpr int NT = yee_block(2, TX);
    static constexpr int X = TX, Y = NT / TX, Z = 1;
};
template <int TX>
struct YeeTile<3, TX> {
    static constexpr int NT = BLOCK;
    static constexpr int X = TX, Y = TX == 32 ? 4 : TX == 16 ? 4 : 8, Z = BLOCK / (TX * Y);
};

// Binomial current filter (section 3.2): when the run asks for k passes, the
// workgroup first gathers the raw current on its tile + halo widened by k
// nodes on every side, then applies the passes in LDS -- a pass smooths each
// component with the 1-2-1 kernel along x, then y, then z -- so the Ampere
// step reads filtered J on tile + halo.  A sweep along an axis leaves the
// outermost layer along that axis stale; after k passes the stale layers
// are exactly the k-wide margin, never read.
template <int DIM, bool FILT>
struct FilterMax {
    static constexpr int K = FILT ? (DIM == 2 ? 4 : 2) : 0;
};

// segments per covering patch that the gather of the Ampere step loads
// before summing (the filter's gather of its widened box, two nodes per
// thread, keeps the plain loop: measured faster there)
template <int DIM, class T>
constexpr int GATHER_SEGU = DIM == 2 ? 2 : 1;

// DET: deterministic mode (64-bit fixed-point tiles summed exactly)
template <int DIM, class T, int TXC, bool FILT, bool DET>
__global__ __launch_bounds__((YeeTile<DIM, TXC>::NT)) void yee_kernel(const RunDev *__restrict__ runs,
                                                                      const int4 *__restrict__ items, int par)
{
    using R = typename std::conditional<DET, long long, typename T::real>::type;   // tile element
    constexpr int NT = YeeTile<DIM, TXC>::NT;
    constexpr int TX = YeeTile<DIM, TXC>::X, TY = YeeTile<DIM, TXC>::Y, TZ = YeeTile<DIM, TXC>::Z;
    static_assert(TX * TY * TZ == NT, "one node per thread");
    constexpr int HX = TX + 1, HY = TY + 1, HZ = DIM == 3 ? TZ + 1 : 1;
    constexpr int HN = HX * HY * HZ;
    constexpr int KM = FilterMax<DIM, FILT>::K;
    constexpr int EXS = HX + 2 * KM, EYS = HY + 2 * KM, EZS = DIM == 3 ? HZ + 2 * KM : 1;
    constexpr int EN = FILT ? EXS * EYS * EZS : 1;
    constexpr int AXM = EXS > EYS ? (EXS > EZS ? EXS : EZS) : (EYS > EZS ? EYS : EZS);
    constexpr int NCM = cover_bound(EXS) * cover_bound(EYS) * (DIM == 3 ? cover_bound(EZS) : 1);
    __shared__ double sE[3][HN];
    __shared__ double sB[3][HN];   // B^{n+1/2} on tile + halo, read again by Faraday
    __shared__ double sJ[FILT ? 4 : 1][EN];   // 3 components + one sweep buffer
    __shared__ int2 s_ax[3][AXM];             // gather tables
    __shared__ int2 s_rng[NCM];
    static_assert(NCM <= 512, "gather table");

    const int4 it = items[blockIdx.x];
    const RunDev &rd = runs[it.x];
    const int tid = threadIdx.x;
    // One workgroup per run ends the bookkeeping of the previous step and
    // prepares the next: the step budget of step s + 1, the overflow counter
    // of step s - 1 (consumed by its post kernel), and the spill store,
    // consumed by this step's particle phase.
    const int rem = rd.ctl->remaining[par];
    if (it.w && tid == 0) {
        rd.ctl->remaining[1 - par] = rem > 0 ? rem - 1 : rem;
        if (rem != 0) {
            rd.ctl->nleave[1 - par] = 0;
            const int ns = rd.ctl->nspill;
            if (ns > rd.ctl->max_spill) rd.ctl->max_spill = ns;
            rd.ctl->nspill = 0;
        }
    }
    if (rem == 0) return;   // the run has taken all its steps

    const int region = it.y;
    const int rr[3] = {region % rd.nreg[0], (region / rd.nreg[0]) % rd.nreg[1],
                       DIM == 3 ? region / (rd.nreg[0] * rd.nreg[1]) : 0};
    const int ro[3] = {rr[0] * rd.rs[0], rr[1] * rd.rs[1], rr[2] * rd.rs[2]};
    const int ntx = (rd.rs[0] + TX - 1) / TX, nty = (rd.rs[1] + TY - 1) / TY;
    const int ti = it.z;
    const int ox = (ti % ntx) * TX, oy = ((ti / ntx) % nty) * TY, oz = DIM == 3 ? (ti / (ntx * nty)) * TZ : 0;
    const int rs0 = rd.rs[0], rs1 = rd.rs[1], rs2 = DIM == 3 ? rd.rs[2] : 1;

    const double dt = rd.dt, dx = rd.d[0], dy = rd.d[1], dz = DIM == 3 ? rd.d[2] : 1.0;
    const SDMD_GLOBAL double *Eo[3], *Bo[3];
    SDMD_GLOBAL double *En[3], *Bn[3], *Bm[3], *Jr[3];
#pragma unroll
    for (int c = 0; c < 3; ++c) {
        Eo[c] = gp((const double *)rcomp(rd, region, f_E(par) + c));
        Bo[c] = gp((const double *)rcomp(rd, region, f_B(par) + c));
        En[c] = gp(rcomp(rd, region, f_E(1 - par) + c));
        Bn[c] = gp(rcomp(rd, region, f_B(1 - par) + c));
        Bm[c] = gp(rcomp(rd, region, F_BM + c));
        Jr[c] = gp(rcomp(rd, region, F_J + c));
    }
    const SDMD_GLOBAL R *tiles = gp((const R *)rd.tiles);
    const long long sx = 1, sy = rd.ra[0], sz = (long long)rd.ra[0] * rd.ra[1];

    int kf = 0;   // filter passes of this run
    if constexpr (FILT) kf = min(max(rd.filter, 0), KM);
    // the gathered box: tile + high halo, widened by kf nodes for the filter
    GatherBox gb;
    {
        const int P[3] = {rd.P[0], rd.P[1], DIM == 3 ? rd.P[2] : 1};
        const int o3[3] = {ro[0] + ox - kf, ro[1] + oy - kf, DIM == 3 ? ro[2] + oz - kf : 0};
        const int e3[3] = {HX + 2 * kf, HY + 2 * kf, DIM == 3 ? HZ + 2 * kf : 1};
#pragma unroll
        for (int a = 0; a < 3; ++a) {
            gb.org[a] = o3[a];
            gb.ext[a] = e3[a];
            if (a < DIM) {
                gb.pu0[a] = floordiv(o3[a], P[a]) - 1;
                gb.nc[a] = floordiv(o3[a] + e3[a] - 1, P[a]) + 2 - gb.pu0[a];
            } else {
                gb.pu0[a] = 0;
                gb.nc[a] = 1;
            }
        }
    }
    gather_tables<DIM, AXM, NCM, NT>(rd, gb, s_ax, s_rng, tid);
    __syncthreads();

    if constexpr (FILT) {
        const int bx = gb.ext[0], by = gb.ext[1], bz = gb.ext[2];
        const int nb = bx * by * bz;
        // raw current on the widened box
        for (int h = tid; h < nb; h += NT) {
            const int ex = h % bx, ey = (h / bx) % by, ez = h / (bx * by);
            double J[3];
            gather_J<DIM, AXM, 0, R>(rd, tiles, gb, s_ax, s_rng, ex, ey, ez, J);
            const int e = (ez * EYS + ey) * EXS + ex;
            sJ[0][e] = J[0];
            sJ[1][e] = J[1];
            sJ[2][e] = J[2];
        }
        __syncthreads();
        for (int c = 0; c < 3; ++c) {
            double *a = sJ[c], *b = sJ[3];
            for (int pass = 0; pass < kf; ++pass)
                for (int axis = 0; axis < DIM; ++axis) {
                    const int st = axis == 0 ? 1 : axis == 1 ? EXS : EXS * EYS;
                    const int ext = axis == 0 ? bx : axis == 1 ? by : bz;
                    for (int h = tid; h < nb; h += NT) {
                        const int ex = h % bx, ey = (h / bx) % by, ez = h / (bx * by);
                        const int co = axis == 0 ? ex : axis == 1 ? ey : ez;
                        if (co < 1 || co > ext - 2) continue;
                        const int e = (ez * EYS + ey) * EXS + ex;
                        b[e] = (a[e - st] + 2.0 * a[e] + a[e + st]) * 0.25;
                    }
                    __syncthreads();
                    double *t = a;
                    a = b;
                    b = t;
                }
            if (a != sJ[c]) {
                for (int h = tid; h < nb; h += NT) {
                    const int ex = h % bx, ey = (h / bx) % by, ez = h / (bx * by);
                    const int e = (ez * EYS + ey) * EXS + ex;
                    sJ[c][e] = a[e];
                }
                __syncthreads();
            }
        }
    }

    // phase 1: J (gathered, or filtered from LDS) and Ampere on tile + high halo
    for (int h = tid; h < HN; h += NT) {
        const int hx = h % HX, hy = (h / HX) % HY, hz = h / (HX * HY);
        const int li = ox + hx, lj = oy + hy, lk = oz + hz;
        if (li > rs0 || lj > rs1 || (DIM == 3 && lk > rs2)) continue;
        const long long p = rindex(rd, li, lj, DIM == 3 ? lk : 0);
        // E^n, B^{n+1/2} and the B neighbours Ampere needs are loaded before
        // the current, so their latency overlaps the gather's
        double fe[3] = {0, 0, 0}, fb[3] = {0, 0, 0}, fn[6] = {0, 0, 0, 0, 0, 0};
        if (!rd.solver) {
#pragma unroll
            for (int c = 0; c < 3; ++c) {
                fb[c] = Bo[c][p];
                fe[c] = Eo[c][p];
            }
            fn[0] = Bo[2][p - sy];
            fn[1] = Bo[2][p - sx];
            fn[2] = Bo[1][p - sx];
            fn[3] = Bo[0][p - sy];
            if constexpr (DIM == 3) {
                fn[4] = Bo[1][p - sz];
                fn[5] = Bo[0][p - sz];
            }
        }
        double J[3];
        if constexpr (FILT) {
            const int e = ((DIM == 3 ? hz + kf : 0) * EYS + hy + kf) * EXS + hx + kf;
            J[0] = sJ[0][e];
            J[1] = sJ[1][e];
            J[2] = sJ[2][e];
        } else {
            gather_J<DIM, AXM, GATHER_SEGU<DIM, T>, R>(rd, tiles, gb, s_ax, s_rng, hx, hy, hz, J);
        }
        if (rd.solver) {
            // spectral solver: this kernel only provides J (the tiles' sum,
            // filtered); E and B are advanced in Fourier space
            if (hx < TX && hy < TY && (DIM == 2 || hz < TZ) && li < rs0 && lj < rs1 && (DIM == 2 || lk < rs2)) {
                Jr[0][p] = J[0];
                Jr[1][p] = J[1];
                Jr[2][p] = J[2];
            }
            continue;
        }
        double e0, e1, e2;
        const double b0 = fb[0], b1 = fb[1], b2 = fb[2];
        sB[0][h] = b0;
        sB[1][h] = b1;
        sB[2][h] = b2;
        if constexpr (DIM == 2) {
            e0 = fe[0] + dt * ((b2 - fn[0]) / dy - J[0]);
            e1 = fe[1] + dt * (-((b2 - fn[1]) / dx) - J[1]);
            e2 = fe[2] + dt * ((b1 - fn[2]) / dx - (b0 - fn[3]) / dy - J[2]);
        } else {
            e0 = fe[0] + dt * ((b2 - fn[0]) / dy - (b1 - fn[4]) / dz - J[0]);
            e1 = fe[1] + dt * ((b0 - fn[5]) / dz - (b2 - fn[1]) / dx - J[1]);
            e2 = fe[2] + dt * ((b1 - fn[2]) / dx - (b0 - fn[3]) / dy - J[2]);
        }
        sE[0][h] = e0;
        sE[1][h] = e1;
        sE[2][h] = e2;
        if (hx < TX && hy < TY && (DIM == 2 || hz < TZ) && li < rs0 && lj < rs1 && (DIM == 2 || lk < rs2)) {
            En[0][p] = e0;
            En[1][p] = e1;
            En[2][p] = e2;
            Jr[0][p] = J[0];
            Jr[1][p] = J[1];
            Jr[2][p] = J[2];
        }
    }
    if (rd.solver) return;
    __syncthreads();

    // phase 2: Faraday and Bm on the tile
    {
        const int tx = tid % TX, ty = (tid / TX) % TY, tz = DIM == 3 ? tid / (TX * TY) : 0;
        const int li = ox + tx, lj = oy + ty, lk = oz + tz;
        if (li < rs0 && lj < rs1 && (DIM == 2 || lk < rs2)) {
            const int h = (tz * HY + ty) * HX + tx;
            const int hxp = h + 1, hyp = h + HX, hzp = h + HX * HY;
            const long long p = rindex(rd, li, lj, DIM == 3 ? lk : 0);
            const double bx = sB[0][h], by = sB[1][h], bz = sB[2][h];
            double nbx, nby, nbz;
            if constexpr (DIM == 2) {
                nbx = bx - dt * ((sE[2][hyp] - sE[2][h]) / dy);
                nby = by - dt * (-((sE[2][hxp] - sE[2][h]) / dx));
                nbz = bz - dt * ((sE[1][hxp] - sE[1][h]) / dx - (sE[0][hyp] - sE[0][h]) / dy);
            } else {
                nbx = bx - dt * ((sE[2][hyp] - sE[2][h]) / dy - (sE[1][hzp] - sE[1][h]) / dz);
                nby = by - dt * ((sE[0][hzp] - sE[0][h]) / dz - (sE[2][hxp] - sE[2][h]) / dx);
                nbz = bz - dt * ((sE[1][hxp] - sE[1][h]) / dx - (sE[0][hyp] - sE[0][h]) / dy);
            }
            Bn[0][p] = nbx;
            Bn[1][p] = nby;
            Bn[2][p] = nbz;
            Bm[0][p] = 0.5 * (bx + nbx);
            Bm[1][p] = 0.5 * (by + nby);
            Bm[2][p] = 0.5 * (bz + nbz);
        }
    }
}

// ------------------------------------------------------------ ghosts
// Ghost node number k of a region -> local coordinates (li, lj, lk).
__device__ __forceinline__ void ghost_coords(const RunDev &rd, int k, int &li, int &lj, int &lk)
{
    const int ra0 = rd.ra[0], ra1 = rd.ra[1];
    const int rs0 = rd.rs[0], rs1 = rd.rs[1];
    const int G2 = 2 * GH;
    if (rd.dims == 2) {
        lk = 0;
        const int rowsN = G2 * ra0;
        if (k < rowsN) {
            const int r = k / ra0;
            lj = r < GH ? r - GH : rs1 + (r - GH);
            li = k % ra0 - GH;
        } else {
            k -= rowsN;
            lj = k / G2;
            const int c = k % G2;
            li = c < GH ? c - GH : rs0 + (c - GH);
        }
        return;
    }
    const int rs2 = rd.rs[2];
    const int slabN = G2 * ra0 * ra1;
    if (k < slabN) {
        const int r = k / (ra0 * ra1), rem = k % (ra0 * ra1);
        lk = r < GH ? r - GH : rs2 + (r - GH);
        lj = rem / ra0 - GH;
        li = rem % ra0 - GH;
        return;
    }
    k -= slabN;
    const int rowN = rs2 * G2 * ra0;
    if (k < rowN) {
        lk = k / (G2 * ra0);
        const int rem = k % (G2 * ra0);
        const int r = rem / ra0;
        lj = r < GH ? r - GH : rs1 + (r - GH);
        li = rem % ra0 - GH;
        return;
    }
    k -= rowN;
    lk = k / (rs1 * G2);
    const int rem = k % (rs1 * G2);
    lj = rem / G2;
    const int c = rem % G2;
    li = c < GH ? c - GH : rs0 + (c - GH);
}

// copy components [c0, c0+nc) of ghost node gk (run-global ghost index)
// from the interior of the region that owns the wrapped node
__device__ __forceinline__ void ghost_copy(const RunDev &rd, int gk, const int *comps, int nc)   // nc <= 9
{
    const int region = gk / rd.ghosts;
    int li, lj, lk;
    ghost_coords(rd, gk - region * rd.ghosts, li, lj, lk);
    const int rr[3] = {region % rd.nreg[0], (region / rd.nreg[0]) % rd.nreg[1], region / (rd.nreg[0] * rd.nreg[1])};
    const int g[3] = {wrap1(rr[0] * rd.rs[0] + li, rd.n[0]), wrap1(rr[1] * rd.rs[1] + lj, rd.n[1]),
                      rd.dims == 3 ? wrap1(rr[2] * rd.rs[2] + lk, rd.n[2]) : 0};
    const int sr[3] = {g[0] / rd.rs[0], g[1] / rd.rs[1], rd.dims == 3 ? g[2] / rd.rs[2] : 0};
    const int src = sr[0] + rd.nreg[0] * (sr[1] + rd.nreg[1] * sr[2]);
    const long long ps = rindex(rd, g[0] - sr[0] * rd.rs[0], g[1] - sr[1] * rd.rs[1],
                                rd.dims == 3 ? g[2] - sr[2] * rd.rs[2] : 0);
    const long long pd = rindex(rd, li, lj, lk);
    // all loads, then all stores: a ghost node is never an interior node, so
    // one round trip to memory replaces nc dependent ones
    double v[9];
#pragma unroll
    for (int i = 0; i < 9; ++i)
        if (i < nc) v[i] = gp((const double *)rcomp(rd, src, comps[i]))[ps];
#pragma unroll
    for (int i = 0; i < 9; ++i)
        if (i < nc) gp(rcomp(rd, region, comps[i]))[pd] = v[i];
}

// ------------------------------------------------------------ post kernel
// Ghost synchronisation and leaver insertion of step s.  The step budget
// and the overflow counter it reads are the entries of step s's parity; the
// field kernel of step s has already prepared those of step s + 1 (so a run
// stops exactly on its last step without any end-of-kernel arrival count).
template <int DIM, class T>
__global__ __launch_bounds__(BLOCK) void post_kernel(const RunDev *__restrict__ runs, const int4 *__restrict__ items,
                                                     int par_new)
{
    const int4 it = items[blockIdx.x];
    const RunDev &rd = runs[it.x];
    const int tid = threadIdx.x;
    const int par = 1 - par_new;   // parity of this step
    const bool active = rd.ctl->remaining[par] != 0;
    int err = 0;
    if (active && it.y == 0) {
        const int comps[9] = {f_E(par_new), f_E(par_new) + 1, f_E(par_new) + 2, f_B(par_new), f_B(par_new) + 1,
                              f_B(par_new) + 2, F_BM, F_BM + 1, F_BM + 2};
        const int gk = it.z + tid;
        if (gk < rd.ghosts * rd.n_regions) ghost_copy(rd, gk, comps, 9);
    } else if (active) {
        // insert the leavers of this step into their destination patch
        auto insert = [&](const int *srcpatch, long long i) -> long long {
            // the destination patch's segments take leavers in turn
            const int q = srcpatch[i];
            const int k0 = rd.pseg[q], nk = rd.pseg[q + 1] - k0;
            const int t = k0 + (nk > 1 ? (int)(i % nk) : 0);
            const int slot = atomicAdd(&rd.scnt[t], 1);
            const int cap = rd.sseg[t + 1] - rd.sseg[t];
            return slot < cap ? (long long)rd.sseg[t] + slot : -1ll - q;
        };
        // The same with the slot claims of a wavefront aggregated: the lanes
        // bound for one destination segment share one atomic (claims on one
        // counter serialise), and the claims for all its destinations are in
        // flight together.  Called by every lane of the wavefront.
        auto insert_wave = [&](const int *srcpatch, long long i, bool valid) -> long long {
            const int lane = tid & 63;
            int q = 0, t = -1;
            if (valid) {
                q = srcpatch[i];
                const int k0 = rd.pseg[q], nk = rd.pseg[q + 1] - k0;
                t = k0 + (nk > 1 ? (int)(i % nk) : 0);
            }
            unsigned long long todo = __ballot(valid), mine = 0;
            bool lead = false;
            while (todo) {
                const int l = __builtin_ctzll(todo);
                const int tl = __shfl(t, l);
                const unsigned long long same = __ballot(valid && t == tl);
                if (valid && t == tl) {
                    mine = same;
                    lead = lane == l;
                }
                todo &= ~same;
            }
            int base = 0;
            if (lead) base = atomicAdd(&rd.scnt[t], __popcll(mine));
            base = __shfl(base, valid ? __builtin_ctzll(mine) : lane);
            if (!valid) return 0;
            const int slot = base + __popcll(mine & ((1ull << lane) - 1ull));
            const int cap = rd.sseg[t + 1] - rd.sseg[t];
            return slot < cap ? (long long)rd.sseg[t] + slot : -1ll - q;
        };
        // parking (full destination segment) claims its slots once per wavefront
        auto place = [&](const Store &src, long long i, bool valid, long long dst) {
            const bool park = valid && dst < 0;
            const unsigned long long mp = __ballot(park);
            int pbase = 0;
            if (mp) {
                if ((tid & 63) == 0) pbase = atomicAdd(&rd.ctl->nspill, __popcll(mp));
                pbase = __shfl(pbase, 0);
            }
            if (valid && dst >= 0) copy_part<DIM, T>(src, i, rd.st, dst);
            if (park) {
                const int s = pbase + __popcll(mp & ((1ull << (tid & 63)) - 1ull));
                if (s < rd.n_total) {
                    copy_part<DIM, T>(src, i, rd.sp, s);
                    rd.spatch[s] = (int)(-1ll - dst);
                    atomicAdd(&rd.spcnt[-1ll - dst], 1);
                } else {
                    err |= ERR_CAPACITY;
                }
            }
        };
        if (it.y == 1) {
            // one wavefront per segment: the segment's leavers sit in its own
            // region of the leaver store
            const int wave = tid >> 6, lane = tid & 63;
            const int s1 = min(it.z + it.w, rd.ctl->nseg);
            for (int sg = it.z + wave; sg < s1; sg += BLOCK / 64) {
                const int nl = rd.nlv[sg];
                const long long b = rd.sseg[sg];
                for (int k0 = 0; k0 < nl; k0 += 64) {
                    const int k = k0 + lane;
                    const bool v = k < nl;
                    place(rd.lv, b + k, v, insert_wave(rd.lpatch, b + k, v));
                }
            }
        } else {
            // overflow leavers (parked particles that re-entered): a few
            // workgroups stride over them
            const int nb = it.w;
            const int nl = min(rd.ctl->nleave[par], rd.n_total);
            for (int i0 = it.z * BLOCK; i0 < nl; i0 += nb * BLOCK) {
                const int i = i0 + tid;
                const bool v = i < nl;
                place(rd.lo, i, v, v ? insert(rd.lopatch, i) : 0);
            }
        }
    }
    if (err) atomicOr(&rd.ctl->err, err);
}

// ------------------------------------------------------------ launchers
#define DT_CASE(D, TT, KERNEL, ...)                                                                   \
    if (dims == D && split == TT::split) {                                                            \
        KERNEL<D, TT><<<n_items, BLOCK, 0, s>>>(__VA_ARGS__);                                         \
        return hipGetLastError();                                                                     \
    }

#define YEE_CASE(D, TT, X, FL)                                                                        \
    if (dims == D && split == TT::split && tx == X && filt == FL) {                                   \
        if (det)                                                                                      \
            yee_kernel<D, TT, X, FL, true><<<n_items, yee_block(D, X), 0, s>>>(runs, items, par);      \
        else                                                                                          \
            yee_kernel<D, TT, X, FL, false><<<n_items, yee_block(D, X), 0, s>>>(runs, items, par);     \
        return hipGetLastError();                                                                     \
    }

int yee_tile_x(int dims, int rs0, bool filt)
{
    if (dims == 3 && filt) return 8;   // the widened box of the filter fits LDS at 8 x 8 x 4
    const int top = dims == 2 ? 64 : 32;
    for (int x = top; x > 8; x /= 2)
        if (rs0 >= x) return x;
    return 8;
}

void yee_tile_shape(int dims, int tx, int shape[3])
{
    shape[0] = tx;
    if (dims == 2) {
        shape[1] = yee_block(2, tx) / tx;
        shape[2] = 1;
    } else {
        shape[1] = tx >= 16 ? 4 : 8;
        shape[2] = BLOCK / (tx * shape[1]);
    }
}

hipError_t launch_yee(int dims, bool split, int tx, bool filt, bool det, const RunDev *runs, const int4 *items,
                      int n_items, int par, hipStream_t s)
{
    if (n_items <= 0) return hipSuccess;
    YEE_CASE(2, F32S, 64, false) YEE_CASE(2, F32S, 32, false) YEE_CASE(2, F32S, 16, false)
    YEE_CASE(2, F32S, 8, false) YEE_CASE(2, FP64, 64, false) YEE_CASE(2, FP64, 32, false)
    YEE_CASE(2, FP64, 16, false) YEE_CASE(2, FP64, 8, false)
    YEE_CASE(3, F32S, 32, false) YEE_CASE(3, F32S, 16, false) YEE_CASE(3, F32S, 8, false)
    YEE_CASE(3, FP64, 32, false) YEE_CASE(3, FP64, 16, false) YEE_CASE(3, FP64, 8, false)
    YEE_CASE(2, F32S, 64, true) YEE_CASE(2, F32S, 32, true) YEE_CASE(2, F32S, 16, true)
    YEE_CASE(2, F32S, 8, true) YEE_CASE(2, FP64, 64, true) YEE_CASE(2, FP64, 32, true)
    YEE_CASE(2, FP64, 16, true) YEE_CASE(2, FP64, 8, true)
    YEE_CASE(3, F32S, 8, true) YEE_CASE(3, FP64, 8, true)
    return hipErrorInvalidValue;
}

hipError_t launch_post(int dims, bool split, const RunDev *runs, const int4 *items, int n_items, int par_new,
                       hipStream_t s)
{
    if (n_items <= 0) return hipSuccess;
    DT_CASE(2, F32S, post_kernel, runs, items, par_new)
    DT_CASE(2, FP64, post_kernel, runs, items, par_new)
    DT_CASE(3, F32S, post_kernel, runs, items, par_new)
    DT_CASE(3, FP64, post_kernel, runs, items, par_new)
    return hipErrorInvalidValue;
}

// ------------------------------------------------------------ init / readout
__global__ void ghosts_kernel(const RunDev *__restrict__ runs, int run, int total, int c0, int nc)
{
    const RunDev &rd = runs[run];
    const int gk = blockIdx.x * BLOCK + threadIdx.x;
    if (gk >= total) return;
    int comps[9];
    for (int i = 0; i < nc && i < 9; ++i) comps[i] = c0 + i;
    ghost_copy(rd, gk, comps, nc < 9 ? nc : 9);
}

hipError_t launch_ghosts(const RunDev *runs, int run, int total_ghosts, int c0, int nc, hipStream_t s)
{
    if (total_ghosts <= 0) return hipSuccess;
    ghosts_kernel<<<(total_ghosts + BLOCK - 1) / BLOCK, BLOCK, 0, s>>>(runs, run, total_ghosts, c0, nc);
    return hipGetLastError();
}

// global node id -> (region, region-local index)
__device__ __forceinline__ void node_of(const RunDev &rd, long long gid, int &region, long long &p)
{
    const int nx = rd.n[0], ny = rd.n[1];
    const int i = (int)(gid % nx), j = (int)((gid / nx) % ny), k = (int)(gid / ((long long)nx * ny));
    const int r0 = i / rd.rs[0], r1 = j / rd.rs[1], r2 = k / rd.rs[2];
    region = r0 + rd.nreg[0] * (r1 + rd.nreg[1] * r2);
    p = rindex(rd, i - r0 * rd.rs[0], j - r1 * rd.rs[1], k - r2 * rd.rs[2]);
}

__global__ void scatter_fields_kernel(const RunDev *__restrict__ runs, int run, int ncell,
                                      const double *__restrict__ src, int c0)
{
    const RunDev &rd = runs[run];
    const long long gid = (long long)blockIdx.x * BLOCK + threadIdx.x;
    if (gid >= ncell) return;
    int region;
    long long p;
    node_of(rd, gid, region, p);
    for (int c = 0; c < 3; ++c) rcomp(rd, region, c0 + c)[p] = src[(long long)c * ncell + gid];
}

hipError_t launch_scatter_fields(const RunDev *runs, int run, int ncell, const double *src, int c0, hipStream_t s)
{
    scatter_fields_kernel<<<(ncell + BLOCK - 1) / BLOCK, BLOCK, 0, s>>>(runs, run, ncell, src, c0);
    return hipGetLastError();
}

__global__ void assemble_kernel(const RunDev *__restrict__ runs, int run, int ncell, int comp, double *__restrict__ dst)
{
    const RunDev &rd = runs[run];
    const long long gid = (long long)blockIdx.x * BLOCK + threadIdx.x;
    if (gid >= ncell) return;
    int region;
    long long p;
    node_of(rd, gid, region, p);
    dst[gid] = rcomp(rd, region, comp)[p];
}

hipError_t launch_assemble(const RunDev *runs, int run, int ncell, int comp, double *dst, hipStream_t s)
{
    assemble_kernel<<<(ncell + BLOCK - 1) / BLOCK, BLOCK, 0, s>>>(runs, run, ncell, comp, dst);
    return hipGetLastError();
}

// Bm = B^0; B^{1/2} = B^0 - dt/2 curl E^0 (region interiors, E ghosts valid)
__global__ void half_faraday_kernel(const RunDev *__restrict__ runs, int run, int ncell, int par)
{
    const RunDev &rd = runs[run];
    const long long gid = (long long)blockIdx.x * BLOCK + threadIdx.x;
    if (gid >= ncell) return;
    int region;
    long long p;
    node_of(rd, gid, region, p);
    const double h = 0.5 * rd.dt, dx = rd.d[0], dy = rd.d[1], dz = rd.dims == 3 ? rd.d[2] : 1.0;
    const long long sx = 1, sy = rd.ra[0], sz = (long long)rd.ra[0] * rd.ra[1];
    const double *E[3];
    double *B[3], *Bm[3];
    for (int c = 0; c < 3; ++c) {
        E[c] = rcomp(rd, region, f_E(par) + c);
        B[c] = rcomp(rd, region, f_B(par) + c);
        Bm[c] = rcomp(rd, region, F_BM + c);
    }
    const double bx = B[0][p], by = B[1][p], bz = B[2][p];
    Bm[0][p] = bx;
    Bm[1][p] = by;
    Bm[2][p] = bz;
    if (rd.dims == 2) {
        B[0][p] = bx - h * ((E[2][p + sy] - E[2][p]) / dy);
        B[1][p] = by - h * (-((E[2][p + sx] - E[2][p]) / dx));
        B[2][p] = bz - h * ((E[1][p + sx] - E[1][p]) / dx - (E[0][p + sy] - E[0][p]) / dy);
    } else {
        B[0][p] = bx - h * ((E[2][p + sy] - E[2][p]) / dy - (E[1][p + sz] - E[1][p]) / dz);
        B[1][p] = by - h * ((E[0][p + sz] - E[0][p]) / dz - (E[2][p + sx] - E[2][p]) / dx);
        B[2][p] = bz - h * ((E[1][p + sx] - E[1][p]) / dx - (E[0][p + sy] - E[0][p]) / dy);
    }
}

hipError_t launch_half_faraday(const RunDev *runs, int run, int ncell, int par, hipStream_t s)
{
    half_faraday_kernel<<<(ncell + BLOCK - 1) / BLOCK, BLOCK, 0, s>>>(runs, run, ncell, par);
    return hipGetLastError();
}

// partial sums of E^2 (buffer par) and Bm^2 over region interiors
__global__ void field_energy_kernel(const RunDev *__restrict__ runs, int run, int ncell, int par,
                                    double *__restrict__ partial)
{
    const RunDev &rd = runs[run];
    __shared__ double se[BLOCK], sb[BLOCK];
    double e = 0.0, b = 0.0;
    for (long long gid = (long long)blockIdx.x * BLOCK + threadIdx.x; gid < ncell; gid += (long long)gridDim.x * BLOCK) {
        int region;
        long long p;
        node_of(rd, gid, region, p);
        for (int c = 0; c < 3; ++c) {
            const double ev = rcomp(rd, region, f_E(par) + c)[p];
            const double bv = rcomp(rd, region, F_BM + c)[p];
            e += ev * ev;
            b += bv * bv;
        }
    }
    se[threadIdx.x] = e;
    sb[threadIdx.x] = b;
    __syncthreads();
    for (int w = BLOCK / 2; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) {
            se[threadIdx.x] += se[threadIdx.x + w];
            sb[threadIdx.x] += sb[threadIdx.x + w];
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        partial[2 * blockIdx.x] = se[0];
        partial[2 * blockIdx.x + 1] = sb[0];
    }
}

hipError_t launch_field_energy(const RunDev *runs, int run, int ncell, int par, double *partial, int nblocks,
                               hipStream_t s)
{
    field_energy_kernel<<<nblocks, BLOCK, 0, s>>>(runs, run, ncell, par, partial);
    return hipGetLastError();
}

// Gauss-law residual g = div_h E - rho at every primal node (x fastest),
// from E of buffer par (ghost layers hold the neighbours) and the deposited
// electron density rho.
__global__ void gauss_kernel(const RunDev *__restrict__ runs, int run, int ncell, int par,
                             const double *__restrict__ rho, double *__restrict__ g)
{
    const RunDev &rd = runs[run];
    const long long gid = (long long)blockIdx.x * BLOCK + threadIdx.x;
    if (gid >= ncell) return;
    int region;
    long long p;
    node_of(rd, gid, region, p);
    const long long st[3] = {1, rd.ra[0], (long long)rd.ra[0] * rd.ra[1]};
    double div = 0.0;
    for (int a = 0; a < rd.dims; ++a) {
        const double *E = rcomp(rd, region, f_E(par) + a);
        div += (E[p] - E[p - st[a]]) / rd.d[a];
    }
    g[gid] = div - rho[gid];
}

// per-block maxima of |g - g0| and |rho|
__global__ void gauss_max_kernel(int ncell, const double *__restrict__ g, const double *__restrict__ g0,
                                 const double *__restrict__ rho, double *__restrict__ partial)
{
    __shared__ double sa[BLOCK], sb[BLOCK];
    double a = 0.0, b = 0.0;
    for (long long i = (long long)blockIdx.x * BLOCK + threadIdx.x; i < ncell; i += (long long)gridDim.x * BLOCK) {
        a = fmax(a, fabs(g[i] - g0[i]));
        b = fmax(b, fabs(rho[i]));
    }
    sa[threadIdx.x] = a;
    sb[threadIdx.x] = b;
    __syncthreads();
    for (int w = BLOCK / 2; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) {
            sa[threadIdx.x] = fmax(sa[threadIdx.x], sa[threadIdx.x + w]);
            sb[threadIdx.x] = fmax(sb[threadIdx.x], sb[threadIdx.x + w]);
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        partial[2 * blockIdx.x] = sa[0];
        partial[2 * blockIdx.x + 1] = sb[0];
    }
}

hipError_t launch_gauss(const RunDev *runs, int run, int ncell, int par, const double *rho, double *g, hipStream_t s)
{
    gauss_kernel<<<(ncell + BLOCK - 1) / BLOCK, BLOCK, 0, s>>>(runs, run, ncell, par, rho, g);
    return hipGetLastError();
}

hipError_t launch_gauss_max(int ncell, const double *g, const double *g0, const double *rho, double *partial,
                            int nblocks, hipStream_t s)
{
    gauss_max_kernel<<<nblocks, BLOCK, 0, s>>>(ncell, g, g0, rho, partial);
    return hipGetLastError();
}

}  // namespace sdmd
