// k_push.hip -- the "Particles" phase of one SDMD step (section 3.3 of the
// paper: interpolation, push, deposition), one workgroup per segment of a
// patch.
//
// Per workgroup:
//   1. transfer (ii) of section 2.2: the patch's window of E^n and Bm^n
//      (nodes [p0-1, p0+P+1] per axis) is read from its region into LDS,
//      converted to the particle precision;
//   2. every particle of the segment (coalesced SoA loads, one chunk per
//      workgroup width, the next chunk prefetched): quadratic B-spline
//      interpolation from the LDS window, Boris push, position update,
//      Esirkepov order-2 deposition (section 3.2) into the segment's LDS
//      current tile with LDS atomics, 64-bit fixed point in the split form
//      and the deterministic mode, FP64 in the plain FP64 form (at most 40
//      adds in 2D, 144 in 3D: the 4-node sub-frame that holds both the old
//      and new shapes; the 3-node core for every particle and the rest only
//      for the particles that change node, structurally zero slots masked
//      lane by lane);
//   3. particles that stay are compacted in place in the patch segment;
//      particles that leave go to the leaver store with their new patch;
//   4. the LDS tile is written to the segment's tile slot in HBM (converted
//      back to the particle precision from fixed point), where the field
//      kernel sums it into the region (transfer (i)).
// The work item is a segment: a patch denser than the segment cap is split
// into several segments (the paper's task decomposition of one patch) that
// load the same window and deposit into their own tiles.
// Particles parked in the spill store that belong to this patch are pushed
// here too (by the patch's first segment) and re-enter through the overflow
// leaver store.  A segment with nothing to push skips all of this.
#include <hip/hip_ext.h>

#include <type_traits>

#include "launch.h"
#include "part.h"
#include "sdmd_dev.h"

namespace sdmd {

// LDS plane stride (in elements) of the 3D window and tile: the smallest
// value >= the plane size n that is 8 modulo 16.  A wavefront's 64 lanes
// take the 8 x 8 cells of an x-z slice of an 8^3 patch (the relayout's
// cell order is y-major), i.e. 8 rows of 8 nodes in consecutive planes.
// With this stride the 8 rows of a window read start on 8 different groups
// of 8 of the 64 LDS banks, and the 2 rows of each 16-lane group of an FP64
// tile add on the 2 halves of the 16 eight-byte banks -- no bank conflicts
// when the lanes' frames are shifted alike (the in-cell order by sub-cell
// half).  Measured on gfx950: an FP64 LDS add with a 2-way bank conflict
// costs 2x, an FP32 read 1.7x.  2D planes are not padded (one plane).
template <int DIM>
__host__ __device__ constexpr int lds_plane(int n)
{
    return DIM == 3 ? (n + 7) / 16 * 16 + 8 : n;
}

// Element index in the LDS field window of component c (Ex, Ey, Ez, Bmx,
// Bmy, Bmz) at window node n (x fastest).  3D: one plane of WS elements per
// component.  2D: the components interpolated from the same nodes with the
// same weights sit side by side -- (Ex, Bmy) and (Ey, Bmx) -- so that one
// two-element LDS read fetches both; then Ez and Bmz.
template <int DIM>
__device__ __forceinline__ int win_index(int c, int n, int WS)
{
    if constexpr (DIM == 3) {
        return c * WS + n;
    } else {
        switch (c) {
        case 0: return 2 * n;
        case 4: return 2 * n + 1;
        case 1: return 2 * WS + 2 * n;
        case 3: return 2 * WS + 2 * n + 1;
        case 2: return 4 * WS + n;
        default: return 5 * WS + n;
        }
    }
}

// Old/new shape factors of one axis on the 4-node sub-frame starting at
// node ip + k0 (k0 = -2 or -1) of the 5-node Esirkepov frame centred on the
// old primal node ip.  d0: old offset from ip in [-1/2, 1/2); d1: new
// position relative to ip in (-3/2, 3/2).  t0: tile index of the first node.
// Plain form: DS = S(new) - S(old), node by node.
template <class R>
__device__ __forceinline__ void esirkepov_axis(R d0, R d1, int ip, R S0[4], R DS[4], int &t0, bool &moved)
{
    R a0, a1, a2, b0, b1, b2;
    shape3(d0, a0, a1, a2);
    R f = floor(d1 + R(0.5));
    int i1 = (int)f;
    shape3(d1 - f, b0, b1, b2);
    const bool lo = i1 < 0, hi = i1 > 0;
    S0[0] = lo ? R(0) : a0;
    S0[1] = lo ? a0 : a1;
    S0[2] = lo ? a1 : a2;
    S0[3] = lo ? a2 : R(0);
    R S1[4];
    S1[0] = hi ? R(0) : b0;
    S1[1] = hi ? b0 : b1;
    S1[2] = hi ? b1 : b2;
    S1[3] = hi ? b2 : R(0);
#pragma unroll
    for (int m = 0; m < 4; ++m) DS[m] = S1[m] - S0[m];
    t0 = ip + (lo ? 0 : 1);   // tile origin is patch origin - 2
    moved = lo || hi;
}

// Split form: the same DS written as polynomials in the displacement D, so
// its rounding error is relative to D rather than to the shape values (a
// cold particle moving 1e-6 cell would otherwise lose most digits of DS in
// FP32).  d0: old offset from ip in [-1/2, 1/2); D: displacement in cells.
// Three cases by where the new position falls: the same primal node, the
// next one up (u, v = distances below / above the half-node knot), or the
// next one down (mirror image).
// MIRROR: one set of formulas for both directions (fewer instructions, more
// values live at once: used where registers allow it, the 2D kernels).
template <class R, bool MIRROR>
__device__ __forceinline__ void esirkepov_axis_delta(R d0, R D, int ip, R S0[4], R DS[4], int &t0, bool &moved)
{
    if constexpr (MIRROR) {
        R a0, a1, a2;
        shape3(d0, a0, a1, a2);
        const R d1 = d0 + D;
        const bool up = d1 >= R(0.5), dn = d1 < R(-0.5), mv = up || dn;
        // same node
        const R t = R(2) * d0 + D;
        const R s0 = R(-0.5) * D * (R(1) - t);
        const R s1 = -D * t;
        const R s2 = R(0.5) * D * (R(1) + t);
        // next node: the move down is the mirror image of the move up (offset
        // and displacement negated, frame slots reversed), so one set of
        // formulas serves both
        const R e = dn ? -d0 : d0, E = dn ? -D : D;
        const R u = R(0.5) - e, v = E - u;
        const R uu = u * u, vv = v * v;
        const R g0 = R(-0.5) * uu;
        const R g1 = (uu - E) + R(0.5) * vv;
        const R g2 = (E - vv) - R(0.5) * uu;
        const R g3 = R(0.5) * vv;
        DS[0] = mv ? (dn ? g3 : g0) : s0;
        DS[1] = mv ? (dn ? g2 : g1) : s1;
        DS[2] = mv ? (dn ? g1 : g2) : s2;
        DS[3] = mv ? (dn ? g0 : g3) : R(0);
        S0[0] = dn ? R(0) : a0;
        S0[1] = dn ? a0 : a1;
        S0[2] = dn ? a1 : a2;
        S0[3] = dn ? a2 : R(0);
        t0 = ip + (dn ? 0 : 1);
        moved = mv;
    } else {
        R a0, a1, a2;
        shape3(d0, a0, a1, a2);
        const R d1 = d0 + D;
        const bool up = d1 >= R(0.5), dn = d1 < R(-0.5);
        // same node
        R c0 = R(-0.5) * D * (R(1) - R(2) * d0 - D);
        R c1 = -D * (R(2) * d0 + D);
        R c2 = R(0.5) * D * (R(1) + R(2) * d0 + D);
        R c3 = R(0);
        if (up) {
            const R u = R(0.5) - d0, v = D - u;
            c0 = R(-0.5) * u * u;
            c1 = -D + R(0.5) * v * v + u * u;
            c2 = D - v * v - R(0.5) * u * u;
            c3 = R(0.5) * v * v;
        } else if (dn) {
            const R u = R(0.5) + d0, v = -D - u;
            c0 = R(0.5) * v * v;
            c1 = -D - v * v - R(0.5) * u * u;
            c2 = D + R(0.5) * v * v + u * u;
            c3 = R(-0.5) * u * u;
        }
        S0[0] = dn ? R(0) : a0;
        S0[1] = dn ? a0 : a1;
        S0[2] = dn ? a1 : a2;
        S0[3] = dn ? a2 : R(0);
        DS[0] = c0;
        DS[1] = c1;
        DS[2] = c2;
        DS[3] = c3;
        t0 = ip + (dn ? 0 : 1);
        moved = up || dn;
    }
}

// One contribution into the LDS tile: an FP64 atomic add, or (FIX) a
// 64-bit integer add of the contribution in fixed point (js: the scale),
// whose sum does not depend on the order of the adds.
template <bool FIX>
__device__ __forceinline__ void tile_add(double *p, double v, double js)
{
    if constexpr (FIX)
        atomicAdd((unsigned long long *)p, to_fixed(v * js));
    else
        atomicAdd(p, v);
}

// Fixed-point scale of one segment's tile in the split form: a power of two
// 2^e with unit * count * 2^e <= 2^62 and unit * 2^e <= 2^50, so that count
// contributions of modulus at most unit sum without leaving the signed
// 64-bit range and each scaled one stays exact in to_fixed.  The tile of a
// segment receives at most one contribution per particle it pushes (its own
// and the parked ones of its patch) per node and component.
__device__ __forceinline__ double seg_fixed_scale(double unit, double count)
{
    if (!(unit > 0.0) || !(unit < 0x1p1000)) return 1.0;
    const double lim = fmin(0x1p62 / (unit * fmax(count, 1.0)), 0x1p50 / unit);
    const int e = ilogb(lim);   // INT_MAX when lim overflows (a tiny unit): clamped below
    return ldexp(1.0, e < -1000 ? -1000 : (e > 1000 ? 1000 : e));
}

// Esirkepov deposition of one particle into the LDS tile.  On the 4-slot
// frame of an axis, a particle that keeps its nearest primal node has zeros
// in the last slot (and its running sum ends one slot early), so every
// particle that keeps its node on all axes deposits only on the first three
// slots of every axis -- the core, 21 adds in 2D and 54 in 3D -- and a
// particle that changes node along some axis also needs the rest of the
// 4-slot frame (19 more adds in 2D, 90 in 3D).  PART selects the core or the
// rest; in the rest, the slots that are structurally zero for a lane (an
// axis along which it kept its node) are masked lane by lane, and `on`
// switches a lane off altogether.  A masked lane takes no part in the
// same-address collisions that serialise an LDS add, and an add no lane
// needs is branched over.
//
// The weights factor as outer products: Jx = cx Cx[m] yf[n] with Cx the
// running sum of DSx and yf = S0y + DSy/2; Jz (2D) = cz (S0x[m] yf[n] +
// DSx[m] (S0y[n]/2 + DSy[n]/3)); in 3D component c flows along axis c and
// the two transverse axes (u, v) carry the time-averaged product
// S0u (S0v + DSv/2) + DSu (S0v/2 + DSv/3).
enum { DEP_CORE = 0, DEP_REST = 1 };

template <int PART, bool FIX, class R>
__device__ __forceinline__ void deposit2d(double *Jb, int T0, int TS, const R S0[3][4], const R DS[3][4],
                                          const R cj[3], R cz, bool mx, bool my, bool on, double js)
{
    constexpr int NF = PART == DEP_CORE ? 3 : 4;
    const R third = R(1) / R(3);
    R hf[2][4], qf[2][4], cs[2][3];
#pragma unroll
    for (int a = 0; a < 2; ++a) {
        R acc = R(0);
#pragma unroll
        for (int m = 0; m < NF; ++m) {
            hf[a][m] = S0[a][m] + R(0.5) * DS[a][m];
            qf[a][m] = R(0.5) * S0[a][m] + third * DS[a][m];
            if (m < NF - 1) {
                acc += DS[a][m];
                cs[a][m] = cj[a] * acc;
            }
        }
    }
    // PART == DEP_CORE: NF = 3, every slot is a core slot; DEP_REST: the
    // slots outside the core that the lane needs
    auto need = [&](bool core, bool cond) { return PART == DEP_CORE || (!core && on && cond); };
#pragma unroll
    for (int n = 0; n < NF; ++n)
#pragma unroll
        for (int m = 0; m < NF - 1; ++m)
            if (need(m < 2 && n < 3, (m < 2 || mx) && (n < 3 || my)))
                tile_add<FIX>(&Jb[n * T0 + m], (double)(cs[0][m] * hf[1][n]), js);
#pragma unroll
    for (int n = 0; n < NF - 1; ++n)
#pragma unroll
        for (int m = 0; m < NF; ++m)
            if (need(n < 2 && m < 3, (n < 2 || my) && (m < 3 || mx)))
                tile_add<FIX>(&Jb[TS + n * T0 + m], (double)(cs[1][n] * hf[0][m]), js);
#pragma unroll
    for (int m = 0; m < NF; ++m) {
        const R a = cz * S0[0][m], b = cz * DS[0][m];
#pragma unroll
        for (int n = 0; n < NF; ++n)
            if (need(m < 3 && n < 3, (m < 3 || mx) && (n < 3 || my)))
                tile_add<FIX>(&Jb[2 * TS + n * T0 + m], (double)(a * hf[1][n] + b * qf[1][n]), js);
    }
}

template <int PART, bool FIX, class R>
__device__ __forceinline__ void deposit3d(double *Jb, int T0, int TP, int TS, const R S0[3][4], const R DS[3][4],
                                          const R cj[3], const bool mv[3], bool on, double js)
{
    constexpr int NF = PART == DEP_CORE ? 3 : 4;
    const R third = R(1) / R(3);
    R hf[3][4], qf[3][4], cs[3][3];
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        R acc = R(0);
#pragma unroll
        for (int m = 0; m < NF; ++m) {
            hf[a][m] = S0[a][m] + R(0.5) * DS[a][m];
            qf[a][m] = R(0.5) * S0[a][m] + third * DS[a][m];
            if (m < NF - 1) {
                acc += DS[a][m];
                cs[a][m] = cj[a] * acc;
            }
        }
    }
#pragma unroll
    for (int c = 0; c < 3; ++c) {
        const int u = c == 0 ? 1 : 0, v = c == 2 ? 1 : 2;
        const int su = u == 0 ? 1 : (u == 1 ? T0 : TP);
        const int sv = v == 1 ? T0 : TP;
        const int sc = c == 0 ? 1 : (c == 1 ? T0 : TP);
#pragma unroll
        for (int i = 0; i < NF; ++i) {
#pragma unroll
            for (int j = 0; j < NF; ++j) {
                const R tr = S0[u][i] * hf[v][j] + DS[u][i] * qf[v][j];
#pragma unroll
                for (int m = 0; m < NF - 1; ++m) {
                    const bool core = m < 2 && i < 3 && j < 3;
                    if (PART == DEP_CORE ||
                        (!core && on && (m < 2 || mv[c]) && (i < 3 || mv[u]) && (j < 3 || mv[v])))
                        tile_add<FIX>(&Jb[c * TS + i * su + j * sv + m * sc], (double)(cs[c][m] * tr), js);
                }
            }
        }
    }
}

// Particles that change their nearest primal node (the movers) need the
// rest of the 4-slot frame besides the core.  Depositing it inline costs a
// wavefront the full set of adds as soon as one of its 64 lanes moved, and
// in a warm plasma almost every wavefront holds a mover while few lanes do.
// So a mover leaves what its rest needs in a per-workgroup queue in LDS
// (the old offset, the second argument of the frame function and the
// nearest node per axis, the current prefactors), and the queue is drained
// once per segment by full wavefronts, one mover per lane.  Recomputing the
// frame from the same inputs with the same code gives the same values the
// core was deposited from.  Movers that find the queue full deposit their
// rest inline.  Queue capacity per workgroup: what the LDS left by the
// window and tile allows without lowering the kernel's occupancy.
//
// The deterministic mode deposits every mover's rest inline (capacity 0):
// which movers find the queue full depends on timing, and the compiler may
// round the frame arithmetic of the inline and the drained copy
// differently, so a particle's contribution must not depend on the path.
template <int DIM, class T, int PC, bool DET>
__host__ __device__ constexpr int mover_cap()
{
    return DET ? 0 : DIM == 3 ? (T::split ? 1024 : 256) : (T::split ? (PC == 8 ? 512 : PC == 16 ? 224 : 256) : 256);
}
// queue fields (arrays of mover_cap entries): per axis the old offset, the
// frame function's second argument and the current prefactor, then (2D) cz
template <int DIM>
__host__ __device__ constexpr int mover_fields()
{
    return 3 * DIM + (DIM == 2 ? 1 : 0);
}

// Esirkepov frame of one axis from the recorded arguments (split form:
// displacement in cells; FP64 form: new position relative to the node)
template <class T, class R, int DIM>
__device__ __forceinline__ void frame_axis(R d0, R a1, int ip, R S0[4], R DS[4], int &t0, bool &moved)
{
    if constexpr (T::split)
        esirkepov_axis_delta<R, DIM == 2>(d0, a1, ip, S0, DS, t0, moved);
    else
        esirkepov_axis<R>(d0, a1, ip, S0, DS, t0, moved);
}

// The rest of a mover's frame from its record: per axis the old offset d0,
// the frame function's second argument a1 and the nearest node (packed 8
// bits per axis in ipk), the current prefactors cj and (2D) cz.  `on`
// switches the lane off.  FIX: fixed-point tile (see tile_add).
template <int DIM, class T, bool FIX>
__device__ __forceinline__ void deposit_rest(const typename T::real d0[3], const typename T::real a1[3], int ipk,
                                             const typename T::real cj[3], typename T::real cz, bool on,
                                             double *tile, int T0, int TP, int TS, double js)
{
    using R = typename T::real;
    R S0[3][4], DS[3][4];
    int t0[3] = {0, 0, 0};
    bool mv[3] = {false, false, false};
#pragma unroll
    for (int a = 0; a < DIM; ++a) frame_axis<T, R, DIM>(d0[a], a1[a], (ipk >> (8 * a)) & 255, S0[a], DS[a], t0[a], mv[a]);
    double *Jb = tile + (DIM == 3 ? t0[2] * TP + t0[1] * T0 + t0[0] : t0[1] * T0 + t0[0]);
    if constexpr (DIM == 2)
        deposit2d<DEP_REST, FIX, R>(Jb, T0, TS, S0, DS, cj, cz, mv[0], mv[1], on, js);
    else
        deposit3d<DEP_REST, FIX, R>(Jb, T0, TP, TS, S0, DS, cj, mv, on, js);
}

// drain the mover queue: the rest of each queued mover's frame
template <int DIM, class T, int QC, bool FIX, int NT>
__device__ __forceinline__ void drain_movers(const typename T::real *q, const int *qi, int nq, double *tile, int T0,
                                             int TP, int TS, double js)
{
    using R = typename T::real;
    for (int e = threadIdx.x; e < nq; e += NT) {
        R d0[3] = {R(0), R(0), R(0)}, a1[3] = {R(0), R(0), R(0)}, cj[3] = {R(0), R(0), R(0)};
#pragma unroll
        for (int a = 0; a < DIM; ++a) {
            d0[a] = q[a * QC + e];
            a1[a] = q[(DIM + a) * QC + e];
            cj[a] = q[(2 * DIM + a) * QC + e];
        }
        deposit_rest<DIM, T, FIX>(d0, a1, qi[e], cj, DIM == 2 ? q[6 * QC + e] : R(0), true, tile, T0, TP, TS, js);
    }
}

// Push one particle: interpolate, Boris, move, deposit.  `p` is updated in
// place (position, cell relative to the destination patch, momentum);
// returns the destination patch.
//
// PX > 0: square (cubic) patches of PX cells, so every LDS stride is a
// compile-time constant and the 54 (2D) window reads and 40 tile updates of
// a particle are one base address plus immediate offsets.  PX = 0: patch
// sizes read from the run descriptor.
//
// The current tile accumulates in 64-bit fixed point (FIX: the split form
// and the deterministic mode; js: the tile's scale) or in FP64 (the plain
// FP64 form); contributions are computed in the particle precision.  On
// gfx950 a wavefront's ds_add_f32 costs ~193 clocks of a CU's LDS against
// ~8.4 for ds_add_f64, and integer adds serialise far less than FP64 adds
// when lanes hit the same node (measured: 6.2 against 20.5 clocks when
// lanes share addresses in pairs).
// q, qi, qn: the workgroup's mover queue (QC entries) and its counter.
template <int DIM, class T, int PX, bool FIX, int QC>
__device__ __forceinline__ int push_one(const RunDev &rd, const typename T::real *__restrict__ win, double *tile,
                                        const int p0[3], const int Prt[3], Part<T> &p, int &err,
                                        typename T::real *q, int *qi, int *qn, double js)
{
    using R = typename T::real;
    const int P0 = PX ? PX : Prt[0], P1 = PX ? PX : Prt[1], P2 = DIM == 3 ? (PX ? PX : Prt[2]) : 1;
    const int P[3] = {P0, P1, P2};
    // LDS strides: rows of P0 + 3 (window) / P0 + 5 (tile) nodes, padded planes
    const int W0 = P0 + 3, WP = lds_plane<DIM>(W0 * (P1 + 3)), WS = WP * (DIM == 3 ? P2 + 3 : 1);
    const int T0 = P0 + 5, TP = lds_plane<DIM>(T0 * (P1 + 5)), TS = TP * (DIM == 3 ? P2 + 5 : 1);

    int lc[3] = {0, 0, 0}, ip[3] = {0, 0, 0};
    R wp[3][3], wd[3][3], dp[3];
    R h[3] = {R(0), R(0), R(0)};   // split form: 1 when the primal node is the upper one
    double X0[3] = {0, 0, 0};
    int ipg[3] = {0, 0, 0};
#pragma unroll
    for (int a = 0; a < DIM; ++a) {
        if constexpr (T::split) {
            int c = (p.cell >> (5 * a)) & 31;
            c = c < P[a] ? c : P[a] - 1;
            lc[a] = c;
            const R xi = p.pos[a];
            h[a] = xi >= R(0.5) ? R(1) : R(0);
            ip[a] = c + (int)h[a];
            dp[a] = xi - h[a];
            shape3(dp[a], wp[a][0], wp[a][1], wp[a][2]);
            shape3(xi - R(0.5), wd[a][0], wd[a][1], wd[a][2]);
        } else {
            const double X = (double)p.pos[a] / rd.d[a];
            X0[a] = X;
            const double fp = floor(X + 0.5), fd = floor(X);
            ipg[a] = (int)fp;
            dp[a] = (R)(X - fp);
            shape3(dp[a], wp[a][0], wp[a][1], wp[a][2]);
            shape3((R)(X - fd - 0.5), wd[a][0], wd[a][1], wd[a][2]);
            const int i = ipg[a] - p0[a];
            ip[a] = i < 0 ? 0 : (i > P[a] ? P[a] : i);
            const int l = (int)fd - p0[a];
            lc[a] = l < 0 ? 0 : (l > P[a] ? P[a] : l);
        }
    }

    // ---- interpolation from the LDS window (window node = local node + 1)
    R E[3], B[3];
    if constexpr (DIM == 2) {
        // window layout: see win_index
        using V2 = typename std::conditional<std::is_same<R, float>::value, float2, double2>::type;
        // The element offset of a stencil's first node is kept in one
        // register (the empty asm hides its sum from the compiler), so the
        // nine reads take the rest of their offsets from the instructions'
        // immediate fields.
        auto sum2 = [&](int plane, const R *wx, int bx, const R *wy, int by) {
            int o = plane + by * W0 + bx;
            asm("" : "+v"(o));
            const R *A = win + o;
            R s = R(0);
#pragma unroll
            for (int b = 0; b < 3; ++b) {
                const R r = wx[0] * A[b * W0] + wx[1] * A[b * W0 + 1] + wx[2] * A[b * W0 + 2];
                s = b == 0 ? wy[0] * r : s + wy[b] * r;
            }
            return s;
        };
        auto pair2 = [&](int plane, const R *wx, int bx, const R *wy, int by, R &s0, R &s1) {
            int o = plane / 2 + by * W0 + bx;   // in pairs
            asm("" : "+v"(o));
            const V2 *A = reinterpret_cast<const V2 *>(win) + o;
#pragma unroll
            for (int b = 0; b < 3; ++b) {
                const V2 q0 = A[b * W0], q1 = A[b * W0 + 1], q2 = A[b * W0 + 2];
                const R r0 = wx[0] * q0.x + wx[1] * q1.x + wx[2] * q2.x;
                const R r1 = wx[0] * q0.y + wx[1] * q1.y + wx[2] * q2.y;
                s0 = b == 0 ? wy[0] * r0 : s0 + wy[b] * r0;
                s1 = b == 0 ? wy[0] * r1 : s1 + wy[b] * r1;
            }
        };
        pair2(0, wd[0], lc[0], wp[1], ip[1], E[0], B[1]);
        pair2(2 * WS, wp[0], ip[0], wd[1], lc[1], E[1], B[0]);
        E[2] = sum2(4 * WS, wp[0], ip[0], wp[1], ip[1]);
        B[2] = sum2(5 * WS, wd[0], lc[0], wd[1], lc[1]);
    } else {
        // one register per plane of the stencil holds its first node's
        // offset (as in 2D); the plane's nine reads add immediates to it
        auto sum3 = [&](int c, const R *wx, int bx, const R *wy, int by, const R *wz, int bz) {
            const int o0 = c * WS + bz * WP + by * W0 + bx;
            R s = R(0);
#pragma unroll
            for (int k = 0; k < 3; ++k) {
                int o = o0 + k * WP;
                asm("" : "+v"(o));
                const R *A = win + o;
                R sk = R(0);
#pragma unroll
                for (int b = 0; b < 3; ++b) {
                    const R *row = A + b * W0;
                    const R r = wx[0] * row[0] + wx[1] * row[1] + wx[2] * row[2];
                    sk = b == 0 ? wy[0] * r : sk + wy[b] * r;
                }
                s = k == 0 ? wz[0] * sk : s + wz[k] * sk;
            }
            return s;
        };
        E[0] = sum3(0, wd[0], lc[0], wp[1], ip[1], wp[2], ip[2]);
        E[1] = sum3(1, wp[0], ip[0], wd[1], lc[1], wp[2], ip[2]);
        E[2] = sum3(2, wp[0], ip[0], wp[1], ip[1], wd[2], lc[2]);
        B[0] = sum3(3, wp[0], ip[0], wd[1], lc[1], wd[2], lc[2]);
        B[1] = sum3(4, wd[0], lc[0], wp[1], ip[1], wd[2], lc[2]);
        B[2] = sum3(5, wd[0], lc[0], wd[1], lc[1], wp[2], ip[2]);
    }

    // ---- Boris push: half E kick, B rotation, half E kick
    R un[3], ig;   // new momentum, 1/gamma
    if constexpr (T::split) {
        // FP32: one hardware reciprocal square root and one reciprocal
        // (1 ulp each) instead of correctly rounded divisions
        const R hq = rd.f_qmh;
        const R um[3] = {p.u[0] + hq * E[0], p.u[1] + hq * E[1], p.u[2] + hq * E[2]};
        const R igm = __builtin_amdgcn_rsqf(R(1) + um[0] * um[0] + um[1] * um[1] + um[2] * um[2]);
        const R f = hq * igm;
        const R t[3] = {f * B[0], f * B[1], f * B[2]};
        const R k2 = R(2) * __builtin_amdgcn_rcpf(R(1) + t[0] * t[0] + t[1] * t[1] + t[2] * t[2]);
        const R s[3] = {k2 * t[0], k2 * t[1], k2 * t[2]};
        const R up[3] = {um[0] + (um[1] * t[2] - um[2] * t[1]), um[1] + (um[2] * t[0] - um[0] * t[2]),
                         um[2] + (um[0] * t[1] - um[1] * t[0])};
        un[0] = um[0] + (up[1] * s[2] - up[2] * s[1]) + hq * E[0];
        un[1] = um[1] + (up[2] * s[0] - up[0] * s[2]) + hq * E[1];
        un[2] = um[2] + (up[0] * s[1] - up[1] * s[0]) + hq * E[2];
        ig = __builtin_amdgcn_rsqf(R(1) + un[0] * un[0] + un[1] * un[1] + un[2] * un[2]);
    } else {
        const R hq = (R)rd.qmh;
        const R um[3] = {p.u[0] + hq * E[0], p.u[1] + hq * E[1], p.u[2] + hq * E[2]};
        const R gm = sqrt(R(1) + um[0] * um[0] + um[1] * um[1] + um[2] * um[2]);
        const R t[3] = {hq * B[0] / gm, hq * B[1] / gm, hq * B[2] / gm};
        const R t2 = t[0] * t[0] + t[1] * t[1] + t[2] * t[2];
        const R s[3] = {R(2) * t[0] / (R(1) + t2), R(2) * t[1] / (R(1) + t2), R(2) * t[2] / (R(1) + t2)};
        const R up[3] = {um[0] + (um[1] * t[2] - um[2] * t[1]), um[1] + (um[2] * t[0] - um[0] * t[2]),
                         um[2] + (um[0] * t[1] - um[1] * t[0])};
        un[0] = um[0] + (up[1] * s[2] - up[2] * s[1]);
        un[1] = um[1] + (up[2] * s[0] - up[0] * s[2]);
        un[2] = um[2] + (up[0] * s[1] - up[1] * s[0]);
        un[0] += hq * E[0];
        un[1] += hq * E[1];
        un[2] += hq * E[2];
        ig = R(1) / sqrt(R(1) + un[0] * un[0] + un[1] * un[1] + un[2] * un[2]);
    }
    if (!(fabs(un[0]) < R(1e30) && fabs(un[1]) < R(1e30) && fabs(un[2]) < R(1e30))) err |= ERR_NONFINITE;

    // ---- move, new cell, Esirkepov frames
    R S0[3][4], DS[3][4];
    R fa[3] = {R(0), R(0), R(0)};          // second argument of each axis's frame function
    int t0[3] = {0, 0, 0};
    bool mv[3] = {false, false, false};   // nearest primal node changed on that axis
    int gcell[3] = {0, 0, 0};   // new global cell
#pragma unroll
    for (int a = 0; a < DIM; ++a) {
        if constexpr (T::split) {
            R delta = (un[a] * ig) * rd.f_dtd[a];
            if (!(fabs(delta) < R(1))) {
                err |= ERR_MOVE;
                delta = R(0);
            }
            const R xn = p.pos[a] + delta;
            fa[a] = delta;
            frame_axis<T, R, DIM>(dp[a], delta, ip[a], S0[a], DS[a], t0[a], mv[a]);
            const R f = floor(xn);
            int sh = (int)f;
            R xi2 = xn - f;
            if (xi2 >= R(1)) {
                xi2 = R(0);
                sh += 1;
            }
            if (xi2 < R(0)) xi2 = R(0);
            p.pos[a] = xi2;
            gcell[a] = wrap1(p0[a] + lc[a] + sh, rd.n[a]);
        } else {
            double xn = (double)p.pos[a] + rd.dt * (double)un[a] * (double)ig;
            double X1 = xn / rd.d[a];
            if (!(fabs(X1 - X0[a]) < 1.0)) {
                err |= ERR_MOVE;
                xn = (double)p.pos[a];
                X1 = X0[a];
            }
            fa[a] = (R)(X1 - (double)ipg[a]);
            frame_axis<T, R, DIM>(dp[a], fa[a], ip[a], S0[a], DS[a], t0[a], mv[a]);
            const double L = rd.L[a];
            if (xn >= L) xn -= L;
            if (xn < 0.0) xn += L;
            if (xn == L) xn = 0.0;
            p.pos[a] = xn;
            int c = (int)floor(xn / rd.d[a]);
            c = c > rd.n[a] - 1 ? rd.n[a] - 1 : (c < 0 ? 0 : c);
            gcell[a] = c;
        }
    }

    // ---- Esirkepov deposition into the LDS tile (deposit2d / deposit3d)
    R cj[3] = {R(0), R(0), R(0)};
#pragma unroll
    for (int a = 0; a < DIM; ++a) cj[a] = (T::split ? (R)rd.f_cj[a] : (R)(-rd.q * rd.d[a] / rd.dt)) * p.w;
    double *Jb = tile + (DIM == 3 ? t0[2] * TP + t0[1] * T0 + t0[0] : t0[1] * T0 + t0[0]);
    // the core of the frame now; the rest, for movers only, through the queue
    bool mover = false;
#pragma unroll
    for (int a = 0; a < DIM; ++a) mover = mover || mv[a];
    const R cz = DIM == 2 ? (T::split ? (R)rd.f_q : (R)rd.q) * p.w * (un[2] * ig) : R(0);
    if constexpr (DIM == 2)
        deposit2d<DEP_CORE, FIX, R>(Jb, T0, TS, S0, DS, cj, cz, false, false, true, js);
    else
        deposit3d<DEP_CORE, FIX, R>(Jb, T0, TP, TS, S0, DS, cj, mv, true, js);
    const unsigned long long mm = __ballot(mover);
    if (mm) {
        // one queue claim per wavefront, by its first active lane
        const int lane = threadIdx.x & 63;
        int base = QC;
        if (QC > 0) {
            const unsigned long long act = __ballot(1);
            if (lane == __builtin_ctzll(act)) base = atomicAdd(qn, __popcll(mm));
            base = __builtin_amdgcn_readfirstlane(base);
        }
        const int slot = base + __popcll(mm & ((1ull << lane) - 1ull));
        const bool queued = mover && slot < QC;
        int ipk = 0;
#pragma unroll
        for (int a = 0; a < DIM; ++a) ipk |= ip[a] << (8 * a);
        if (queued) {
#pragma unroll
            for (int a = 0; a < DIM; ++a) {
                q[a * QC + slot] = dp[a];
                q[(DIM + a) * QC + slot] = fa[a];
                q[(2 * DIM + a) * QC + slot] = cj[a];
            }
            if constexpr (DIM == 2) q[6 * QC + slot] = cz;
            qi[slot] = ipk;
        }
        // the queue is full: the rest inline, from the same record
        const bool now = mover && !queued;
        if (__any(now)) deposit_rest<DIM, T, FIX>(dp, fa, ipk, cj, cz, now, tile, T0, TP, TS, js);
    }

    p.u[0] = un[0];
    p.u[1] = un[1];
    p.u[2] = un[2];

    // ---- destination patch and cell inside it
    // (gcell is in [0, n): unsigned division, a shift for power-of-two patches)
    int dest = 0, mul = 1, packed = 0;
#pragma unroll
    for (int a = 0; a < DIM; ++a) {
        const unsigned g = (unsigned)gcell[a], pe = (unsigned)P[a];
        const unsigned pa = g / pe;
        dest += (int)pa * mul;
        mul *= rd.np[a];
        packed |= (int)(g - pa * pe) << (5 * a);
    }
    p.cell = packed;
    return dest;
}

// PX: exact patch edge (0 = sizes from the run descriptor); PC: LDS sizing
// class (the largest patch edge the instantiation accepts)
// threads per particle-kernel workgroup: 3D workgroups hold an 85 KB LDS
// window + tile, so only one fits per CU; 16 wavefronts keep it busy
// (FP64 3D: 512, its 128+ registers per lane do not fit 16 wavefronts)
template <int DIM, class T>
constexpr int push_block() { return DIM == 3 ? (T::split ? 1024 : 512) : 256; }

// Wavefronts per SIMD the compiler must leave room for: the 2D split-form
// kernel of patches up to 16 cells holds five 256-thread workgroups per CU
// (its LDS allows that), which needs at most 96 registers per lane; the
// others are bound by their LDS or registers anyway.
template <int DIM, class T, int PC>
constexpr int push_min_waves() { return DIM == 2 && T::split && PC <= 16 ? 5 : 1; }

// DET: deterministic mode (64-bit fixed-point tiles, see to_fixed)
template <int DIM, class T, int PX, int PC, bool DET>
__global__ __launch_bounds__((push_block<DIM, T>()), (push_min_waves<DIM, T, PC>())) void push_kernel(const RunDev *__restrict__ runs,
                                                                 const int2 *__restrict__ items, int par)
{
    using R = typename T::real;
    constexpr int BLOCK = push_block<DIM, T>();
    constexpr int WN = lds_plane<DIM>((PC + 3) * (PC + 3)) * (DIM == 3 ? PC + 3 : 1);
    constexpr int TN = lds_plane<DIM>((PC + 5) * (PC + 5)) * (DIM == 3 ? PC + 5 : 1);
    constexpr int NW = BLOCK / 64;
    constexpr int SPC = 1024;                          // spill entries scanned per round
    constexpr int SPK = (SPC + BLOCK - 1) / BLOCK;
    // The window sits at LDS address 0, so the interpolation's paired
    // reads of neighbouring nodes take their offsets from the instruction's
    // immediate fields instead of an address add per read; the tile follows.
    struct alignas(16) WinTile {
        R win[6 * WN];
        double tile[3 * TN];
    };
    __shared__ WinTile s_wt;
    R *const s_win = s_wt.win;
    double *const s_tile = s_wt.tile;
    __shared__ int s_wsum[NW], s_left, s_sw[NW];
    __shared__ int s_hole[BLOCK];
    __shared__ int s_sl[SPC];                          // this patch's parked particles found in a round
    __shared__ int s_ns;
    constexpr int QC = mover_cap<DIM, T, PC, DET>();
    __shared__ R s_q[mover_fields<DIM>() * (QC > 0 ? QC : 1)];   // mover queue (see mover_cap)
    __shared__ int s_qi[QC > 0 ? QC : 1];
    __shared__ int s_qn;

    // Work item l of a run runs on XCD l % 8 (workgroups are dealt to the
    // 8 XCDs in turn, and every run's items start at a multiple of 8).  The
    // live segments are cut into 8 contiguous bands, one per XCD: each
    // XCD's L2 sees neighbouring patches (shared window halos), and the
    // live work is spread evenly however many slots are in use.
    const int2 item = items[blockIdx.x];
    const RunDev &rd = runs[item.x];
    const int nseg = rd.ctl->nseg;
    const int band = (nseg + 7) >> 3;
    const int jb = item.y >> 3;
    const int sg = (item.y & 7) * band + jb;   // segment
    if (jb >= band || sg >= nseg || rd.ctl->remaining[par] == 0) return;   // slot unused, or run finished
    const int q = rd.spat[sg];           // its patch
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;

    const int P[3] = {PX ? PX : rd.P[0], PX ? PX : rd.P[1], DIM == 3 ? (PX ? PX : rd.P[2]) : 1};
    const int pq[3] = {q % rd.np[0], (q / rd.np[0]) % rd.np[1], DIM == 3 ? q / (rd.np[0] * rd.np[1]) : 0};
    const int p0[3] = {pq[0] * P[0], pq[1] * P[1], pq[2] * P[2]};
    const int rr[3] = {p0[0] / rd.rs[0], p0[1] / rd.rs[1], DIM == 3 ? p0[2] / rd.rs[2] : 0};
    const int region = rr[0] + rd.nreg[0] * (rr[1] + rd.nreg[1] * rr[2]);
    const int o[3] = {p0[0] - rr[0] * rd.rs[0], p0[1] - rr[1] * rd.rs[1], DIM == 3 ? p0[2] - rr[2] * rd.rs[2] : 0};
    const int W0 = P[0] + 3, W1 = P[1] + 3, W2 = DIM == 3 ? P[2] + 3 : 1;
    const int WS = W0 * W1 * W2;
    const int T0 = P[0] + 5, T1 = P[1] + 5, TS = T0 * T1 * (DIM == 3 ? P[2] + 5 : 1);   // tile in HBM
    const int WPs = lds_plane<DIM>(W0 * W1), WSs = WPs * W2;                           // LDS layout
    const int TPs = lds_plane<DIM>(T0 * T1), TSs = TPs * (DIM == 3 ? P[2] + 5 : 1);

    const SDMD_GLOBAL int *sseg = gp(rd.sseg);
    // segment bounds and count: uniform values, kept in scalar registers so
    // that the particle addresses below are scalar bases + 32-bit offsets
    const long long seg0 = __builtin_amdgcn_readfirstlane(sseg[sg]);
    const int cap = __builtin_amdgcn_readfirstlane(sseg[sg + 1]) - (int)seg0;
    int n = __builtin_amdgcn_readfirstlane(gp(rd.scnt)[sg]);
    n = n < cap ? n : cap;
    // parked particles are pushed by the patch's first segment, which scans
    // the spill store only when some are parked for its patch.  Their count
    // is loaded here but read only after the window loads have gone out;
    // only an empty segment waits for it first.  (The empty asm statements
    // keep the compiler from moving those waits.)
    int first = gp(rd.pseg)[q], cnt = gp(rd.spcnt)[q];
    SDMD_GLOBAL int *tflag = gp(rd.tflag);
    int idle = 1;   // 0: nothing to push
    if (n == 0) {
        idle = sg == first ? cnt : 0;
        asm volatile("" : "+v"(idle));
    }
    if (idle == 0) {
        // nothing to push (a vacuum patch): no window, no tile work; the
        // tile in HBM is cleared only if an earlier step left current in it
        const int dirty = tflag[sg];
        if (dirty) {
            using TE = typename std::conditional<DET, long long, R>::type;   // tile element in HBM
            SDMD_GLOBAL TE *dst = gp((TE *)rd.tiles) + (long long)sg * 3 * TS;
            for (int idx = tid; idx < 3 * TS; idx += BLOCK) dst[idx] = TE(0);
        }
        __syncthreads();
        if (tid == 0) {
            tflag[sg] = 0;
            gp(rd.nlv)[sg] = 0;
        }
        return;
    }

    // transfer (ii): region E^n, Bm^n -> LDS window.  A thread takes WB
    // window nodes (stride BLOCK) at a time and loads all six components of
    // each before storing any, so the fill of a 16 x 16 (2D) or 8^3 (3D)
    // patch's window waits on memory once; a node's index arithmetic is
    // shared by its six loads, whose bases are uniform.
    constexpr int WB = 2;
    const SDMD_GLOBAL double *Ereg = gp((const double *)rcomp(rd, region, f_E(par)));
    const SDMD_GLOBAL double *Breg = gp((const double *)rcomp(rd, region, F_BM));
    const long long cst = rd.rsize;   // component stride of a region
    for (int n0 = 0; n0 < WS; n0 += WB * BLOCK) {
        double wv[WB][6];
        int wl[WB];
        // lanes past the window's end load its last node again and store
        // nothing: no branch between the loads, so they wait on memory once
#pragma unroll
        for (int u = 0; u < WB; ++u) {
            const int nr = n0 + u * BLOCK + tid, nd = nr < WS ? nr : WS - 1;
            const int wx = nd % W0, tq = nd / W0, wy = tq % W1, wz = tq / W1;
            wl[u] = nr < WS ? wz * WPs + wy * W0 + wx : -1;
            const long long g = rindex(rd, o[0] - 1 + wx, o[1] - 1 + wy, DIM == 3 ? o[2] - 1 + wz : 0);
#pragma unroll
            for (int c = 0; c < 3; ++c) {
                wv[u][c] = Ereg[g + c * cst];
                wv[u][3 + c] = Breg[g + c * cst];
            }
        }
#pragma unroll
        for (int u = 0; u < WB; ++u)
            if (wl[u] >= 0) {
#pragma unroll
                for (int c = 0; c < 6; ++c) s_win[win_index<DIM>(c, wl[u], WSs)] = (R)wv[u][c];
            }
    }
    for (int idx = tid; idx < 3 * TSs; idx += BLOCK) s_tile[idx] = 0.0;
    asm volatile("" : "+v"(first), "+v"(cnt));
    const int want = sg == first ? cnt : 0;
    // current tile: 64-bit fixed point in the split form (scale from this
    // segment's particle count) and in the deterministic mode (the run's
    // scale, the same for every segment); FP64 in the plain FP64 form
    constexpr bool FIX = DET || T::split;
    const double js = DET ? rd.jscale : (T::split ? seg_fixed_scale(rd.junit, (double)n + (double)want) : 0.0);
    if (tid == 0) {
        s_left = 0;
        s_qn = 0;
    }
    __syncthreads();

    int err = 0;
    int sw = 0;   // stayers of this wavefront so far (uniform over the wavefront)
    const unsigned long long lt = (1ull << lane) - 1ull;
    // slot k of wavefront w's sequence (the slots it visits, chunk by chunk)
    auto wslot = [&](int w, int k) { return (k >> 6) * BLOCK + (w << 6) + (k & 63); };

    // Each wavefront compacts its stayers into its own sequence of slots: its
    // k-th stayer goes to wslot(w, k), never above the slot it was read from,
    // so no wavefront overwrites a particle another has not read yet and the
    // chunks need no barrier.  Leavers take slots of the segment's leaver
    // region from an LDS counter.  The stayers left at or above the final
    // count then fill the holes below it.  The next chunk's particles are
    // loaded before this chunk is pushed.
    const SegStore sst = seg_store<T>(rd.st, seg0), slv = seg_store<T>(rd.lv, seg0);
    SDMD_GLOBAL int *lpatch = gp(rd.lpatch) + seg0;
    Part<T> nxt;
    if (tid < n) load_part<DIM, T>(sst, (uint32_t)tid, nxt);
    for (int base = 0; base < n; base += BLOCK) {
        const int i = base + tid;
        const bool valid = i < n;
        Part<T> pt = nxt;
        if (i + BLOCK < n) load_part<DIM, T>(sst, (uint32_t)(i + BLOCK), nxt);
        int dest = q;
        if (valid) dest = push_one<DIM, T, PX, FIX, QC>(rd, s_win, s_tile, p0, P, pt, err, s_q, s_qi, &s_qn, js);
        const bool st = valid && dest == q;
        const bool lv = valid && dest != q;
        const unsigned long long ms = __ballot(st), ml = __ballot(lv);
        if (st) {
            const int slot = wslot(wave, sw + __popcll(ms & lt));
            store_part<DIM, T>(sst, (uint32_t)slot, pt, slot != i);
        }
        sw += __popcll(ms);
        if (ml) {
            // the segment's own leaver region: stayers + leavers <= n <= capacity
            int lb = 0;
            if (lane == 0) lb = atomicAdd(&s_left, __popcll(ml));
            lb = __shfl(lb, 0);
            if (lv) {
                const int slot = lb + __popcll(ml & lt);
                store_part<DIM, T>(slv, (uint32_t)slot, pt, true);
                lpatch[slot] = dest;
            }
        }
    }
    if (lane == 0) s_sw[wave] = sw;
    __syncthreads();   // every stayer is in its wavefront's sequence
    const int left = s_left;
    const int stay = n - left;
    if (left > 0) {
        // Slot p < n is a hole when its wavefront kept fewer stayers than p's
        // rank in that wavefront's sequence.  The holes below `stay` and the
        // stayers at or above it are equally many; the r-th of each are
        // paired (slot order), BLOCK pairs per round.
        auto hole = [&](int p) { return (p / BLOCK) * 64 + (p & 63) >= s_sw[(p % BLOCK) >> 6]; };
        int lo = stay;   // the first hole
#pragma unroll
        for (int w = 0; w < NW; ++w) lo = min(lo, wslot(w, s_sw[w]));
        // rank of each flagged slot of the block starting at b among the flagged slots so far
        auto rank_in = [&](bool f, int &run, int &tot) {
            const unsigned long long m = __ballot(f);
            if (lane == 0) s_wsum[wave] = __popcll(m);
            __syncthreads();
            int before = run;
            tot = 0;
#pragma unroll
            for (int w = 0; w < NW; ++w) {
                before += w < wave ? s_wsum[w] : 0;
                tot += s_wsum[w];
            }
            __syncthreads();   // s_wsum is reused by the next block
            run += tot;
            return before + __popcll(m & lt);
        };
        for (int r0 = 0;; r0 += BLOCK) {
            int run = 0, tot = 0;
            for (int b = lo; b < stay; b += BLOCK) {
                const int pz = b + tid;
                const bool f = pz < stay && hole(pz);
                const int rk = rank_in(f, run, tot);
                if (f && rk >= r0 && rk < r0 + BLOCK) s_hole[rk - r0] = pz;
            }
            const int nh = min(run - r0, BLOCK);   // run: all holes below `stay`
            if (nh <= 0) break;
            __syncthreads();
            int run2 = 0;
            for (int b = stay; b < n; b += BLOCK) {
                const int pz = b + tid;
                const bool f = pz < n && !hole(pz);
                const int rk = rank_in(f, run2, tot);
                if (f && rk >= r0 && rk < r0 + nh) {
                    Part<T> mv;
                    load_part<DIM, T>(sst, (uint32_t)pz, mv);
                    store_part<DIM, T>(sst, (uint32_t)s_hole[rk - r0], mv, true);
                }
            }
            if (run <= r0 + BLOCK) break;
            __syncthreads();   // s_hole is rewritten by the next round
        }
    }

    // particles parked in the spill store that belong to this patch re-enter
    // through the overflow leaver store.  The spill store is scanned in
    // rounds of SPC entries, all loads of a round in flight at once; the
    // round's matches are listed in LDS and pushed.
    int found = 0;   // parked particles of this patch pushed so far (uniform)
    const int nsp = want > 0 ? min(rd.ctl->nspill, rd.n_total) : 0;
    for (int c0 = 0; c0 < nsp && found < want; c0 += SPC) {
        if (tid == 0) s_ns = 0;
        __syncthreads();
        int pv[SPK];
#pragma unroll
        for (int k = 0; k < SPK; ++k) {
            const int r = k * BLOCK + tid, i = c0 + r;
            pv[k] = (r < SPC && i < nsp) ? gp(rd.spatch)[i] : -1;
        }
#pragma unroll
        for (int k = 0; k < SPK; ++k) {
            const bool mine = pv[k] == q;
            const unsigned long long mm = __ballot(mine);
            int wb = 0;
            if (mm) {
                if (lane == 0) wb = atomicAdd(&s_ns, __popcll(mm));
                wb = __shfl(wb, 0);
            }
            if (mine) s_sl[wb + __popcll(mm & lt)] = c0 + k * BLOCK + tid;
        }
        __syncthreads();
        const int ns = s_ns;
        found += ns;
        for (int base = 0; base < ns; base += BLOCK) {
            const int j = base + tid;
            const bool mine = j < ns;
            Part<T> pt;
            int dest = q;
            if (mine) {
                load_part<DIM, T>(rd.sp, s_sl[j], pt);
                dest = push_one<DIM, T, PX, FIX, QC>(rd, s_win, s_tile, p0, P, pt, err, s_q, s_qi, &s_qn, js);
            }
            const unsigned long long ml = __ballot(mine);
            int lbase = 0;
            if (ml) {
                if (lane == 0) lbase = atomicAdd(&rd.ctl->nleave[par], __popcll(ml));
                lbase = __shfl(lbase, 0);
            }
            if (mine) {
                const int slot = lbase + __popcll(ml & lt);
                if (slot < rd.n_total) {
                    store_part<DIM, T>(rd.lo, slot, pt, true);
                    gp(rd.lopatch)[slot] = dest;
                } else {
                    err |= ERR_CAPACITY;
                }
            }
        }
        __syncthreads();   // s_sl and s_ns are reused by the next round
    }

    if (err) atomicOr(&rd.ctl->err, err);
    if (tid == 0) {
        gp(rd.scnt)[sg] = stay;
        gp(rd.nlv)[sg] = left;
        if (want > 0) gp(rd.spcnt)[q] = 0;   // consumed; this step's post kernel parks anew
    }
    __syncthreads();   // every push of the segment is done: the queue is complete
    // the rest of the movers' frames, from the queue
    if constexpr (QC > 0) {
        drain_movers<DIM, T, QC, FIX, BLOCK>(s_q, s_qi, min(s_qn, QC), s_tile, T0, TPs, TSs, js);
        __syncthreads();
    }
    // flush the tile in the tile precision (transfer (i) reads it); the
    // deterministic mode keeps the 64-bit integers
    if constexpr (DET) {
        SDMD_GLOBAL long long *dst = gp((long long *)rd.tiles) + (long long)sg * 3 * TS;
        const long long *st = (const long long *)s_tile;
        for (int idx = tid; idx < 3 * TS; idx += BLOCK) {
            const int pl = idx / (T0 * T1), rem = idx - pl * (T0 * T1);
            dst[idx] = st[pl * TPs + rem];
        }
    } else if constexpr (FIX) {
        // back from the segment's fixed point (the scale is a power of two)
        SDMD_GLOBAL R *dst = gp((R *)rd.tiles) + (long long)sg * 3 * TS;
        const long long *st = (const long long *)s_tile;
        const double inv = 1.0 / js;
        for (int idx = tid; idx < 3 * TS; idx += BLOCK) {
            const int pl = idx / (T0 * T1), rem = idx - pl * (T0 * T1);
            dst[idx] = (R)((double)st[pl * TPs + rem] * inv);
        }
    } else {
        SDMD_GLOBAL R *dst = gp((R *)rd.tiles) + (long long)sg * 3 * TS;
        for (int idx = tid; idx < 3 * TS; idx += BLOCK) {
            const int pl = idx / (T0 * T1), rem = idx - pl * (T0 * T1);   // plane (component and z), node in it
            dst[idx] = (R)s_tile[pl * TPs + rem];
        }
    }
    if (tid == 0) tflag[sg] = 1;
}

// With events, the launch goes through hipExtLaunchKernelGGL, which records
// ev0 when the kernel starts and ev1 when it ends (its own duration, without
// the dispatch gap that events recorded between launches include).
template <class K>
static hipError_t push_launch(K kern, int n_items, int block, hipStream_t s, hipEvent_t ev0, hipEvent_t ev1,
                              const RunDev *runs, const int2 *items, int par)
{
    if (ev0 || ev1)
        hipExtLaunchKernelGGL(kern, dim3(n_items), dim3(block), 0, s, ev0, ev1, 0, runs, items, par);
    else
        kern<<<n_items, block, 0, s>>>(runs, items, par);
    return hipGetLastError();
}

#define PUSH_CASE(D, TT, PXV, PCV)                                                                  \
    if (dims == D && split == TT::split && px == PXV && pc == PCV) {                                \
        if (det)                                                                                    \
            return push_launch(push_kernel<D, TT, PXV, PCV, true>, n_items, push_block<D, TT>(), s, \
                               ev0, ev1, runs, items, par);                                         \
        return push_launch(push_kernel<D, TT, PXV, PCV, false>, n_items, push_block<D, TT>(), s,    \
                           ev0, ev1, runs, items, par);                                             \
    }

// px: exact square/cubic patch edge with a compiled fast path, else 0;
// pc: LDS sizing class 8 / 16 / 32; det: deterministic mode; ev0 / ev1:
// events recorded at the kernel's start and end (may be null)
hipError_t launch_push(int dims, bool split, int px, int pc, bool det, const RunDev *runs, const int2 *items,
                       int n_items, int par, hipStream_t s, hipEvent_t ev0, hipEvent_t ev1)
{
    if (n_items <= 0) return hipSuccess;
    PUSH_CASE(2, F32S, 8, 8)
    PUSH_CASE(2, F32S, 16, 16)
    PUSH_CASE(2, F32S, 32, 32)
    PUSH_CASE(2, F32S, 0, 8)
    PUSH_CASE(2, F32S, 0, 16)
    PUSH_CASE(2, F32S, 0, 32)
    PUSH_CASE(2, FP64, 8, 8)
    PUSH_CASE(2, FP64, 16, 16)
    PUSH_CASE(2, FP64, 0, 8)
    PUSH_CASE(2, FP64, 0, 16)
    PUSH_CASE(2, FP64, 0, 32)
    PUSH_CASE(3, F32S, 8, 8)
    PUSH_CASE(3, F32S, 0, 8)
    PUSH_CASE(3, FP64, 8, 8)
    PUSH_CASE(3, FP64, 0, 8)
    return hipErrorInvalidValue;
}

}  // namespace sdmd
