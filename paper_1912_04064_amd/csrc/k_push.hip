// k_push.hip -- the "Particles" phase of one SDMD step (section 3.3 of the
// paper: interpolation, push, deposition), one workgroup per patch.
//
// Per patch workgroup:
//   1. transfer (ii) of section 2.2: the patch's window of E^n and Bm^n
//      (nodes [p0-1, p0+P+1] per axis) is read from its region into LDS,
//      converted to the particle precision;
//   2. every particle of the patch (coalesced SoA loads, 256 at a time):
//      quadratic B-spline interpolation from the LDS window, Boris push,
//      position update, Esirkepov order-2 deposition (section 3.2) into the
//      patch's LDS current tile with LDS float atomics (40 adds in 2D, 144 in
//      3D: the 4-node sub-frame that holds both the old and new shapes);
//   3. particles that stay are compacted in place in the patch segment;
//      particles that leave go to the leaver store with their new patch;
//   4. the LDS tile is written to the patch's tile slot in HBM, where the
//      field kernel sums it into the region (transfer (i)).
// Particles parked in the spill store that belong to this patch are pushed
// here too and all re-enter through the leaver store.
#include "launch.h"
#include "part.h"
#include "sdmd_dev.h"

namespace sdmd {

// Old/new shape factors of one axis on the 4-node sub-frame starting at
// node ip + k0 (k0 = -2 or -1) of the 5-node Esirkepov frame centred on the
// old primal node ip.  d0: old offset from ip in [-1/2, 1/2); d1: new
// position relative to ip in (-3/2, 3/2).  t0: tile index of the first node.
template <class R>
__device__ __forceinline__ void esirkepov_axis(R d0, R d1, int ip, R S0[4], R DS[4], int &t0)
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
}

// Push one particle: interpolate, Boris, move, deposit.  `p` is updated in
// place (position, cell relative to the destination patch, momentum);
// returns the destination patch.
template <int DIM, class T>
__device__ __forceinline__ int push_one(const RunDev &rd, const typename T::real *__restrict__ win,
                                        typename T::real *tile, const int W0, const int W1, const int WS,
                                        const int T0, const int T1, const int TS, const int p0[3], const int P[3],
                                        Part<T> &p, int &err)
{
    using R = typename T::real;
    int lc[3] = {0, 0, 0}, ip[3] = {0, 0, 0};
    R wp[3][3], wd[3][3], dp[3];
    R h[3];                  // split form: 1 when the primal node is the upper one
    double X0[3] = {0, 0, 0};
    int ipg[3] = {0, 0, 0};
#pragma unroll
    for (int a = 0; a < DIM; ++a) {
        if constexpr (T::split) {
            int c = (p.cell >> (5 * a)) & 31;
            c = c < P[a] ? c : P[a] - 1;
            lc[a] = c;
            R xi = p.pos[a];
            h[a] = xi >= R(0.5) ? R(1) : R(0);
            ip[a] = c + (int)h[a];
            dp[a] = xi - h[a];
            shape3(dp[a], wp[a][0], wp[a][1], wp[a][2]);
            shape3(xi - R(0.5), wd[a][0], wd[a][1], wd[a][2]);
        } else {
            double X = (double)p.pos[a] / rd.d[a];
            X0[a] = X;
            double fp = floor(X + 0.5), fd = floor(X);
            ipg[a] = (int)fp;
            dp[a] = (R)(X - fp);
            shape3(dp[a], wp[a][0], wp[a][1], wp[a][2]);
            shape3((R)(X - fd - 0.5), wd[a][0], wd[a][1], wd[a][2]);
            int i = ipg[a] - p0[a];
            ip[a] = i < 0 ? 0 : (i > P[a] ? P[a] : i);
            int l = (int)fd - p0[a];
            lc[a] = l < 0 ? 0 : (l > P[a] ? P[a] : l);
        }
    }

    // ---- interpolation from the LDS window (window node = local node + 1)
    R E[3], B[3];
    if constexpr (DIM == 2) {
        auto sum2 = [&](int c, const R *wx, int bx, const R *wy, int by) {
            const R *A = win + c * WS;
            R s = R(0);
#pragma unroll
            for (int b = 0; b < 3; ++b) {
                const R *row = A + (by + b) * W0 + bx;
                s += wy[b] * (wx[0] * row[0] + wx[1] * row[1] + wx[2] * row[2]);
            }
            return s;
        };
        E[0] = sum2(0, wd[0], lc[0], wp[1], ip[1]);
        E[1] = sum2(1, wp[0], ip[0], wd[1], lc[1]);
        E[2] = sum2(2, wp[0], ip[0], wp[1], ip[1]);
        B[0] = sum2(3, wp[0], ip[0], wd[1], lc[1]);
        B[1] = sum2(4, wd[0], lc[0], wp[1], ip[1]);
        B[2] = sum2(5, wd[0], lc[0], wd[1], lc[1]);
    } else {
        auto sum3 = [&](int c, const R *wx, int bx, const R *wy, int by, const R *wz, int bz) {
            const R *A = win + c * WS;
            R s = R(0);
#pragma unroll
            for (int k = 0; k < 3; ++k) {
                R sk = R(0);
#pragma unroll
                for (int b = 0; b < 3; ++b) {
                    const R *row = A + ((bz + k) * W1 + by + b) * W0 + bx;
                    sk += wy[b] * (wx[0] * row[0] + wx[1] * row[1] + wx[2] * row[2]);
                }
                s += wz[k] * sk;
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
    const R hq = T::split ? (R)rd.f_qmh : (R)rd.qmh;
    R um[3] = {p.u[0] + hq * E[0], p.u[1] + hq * E[1], p.u[2] + hq * E[2]};
    R gm = sqrt(R(1) + um[0] * um[0] + um[1] * um[1] + um[2] * um[2]);
    R t[3] = {hq * B[0] / gm, hq * B[1] / gm, hq * B[2] / gm};
    R t2 = t[0] * t[0] + t[1] * t[1] + t[2] * t[2];
    R s[3] = {R(2) * t[0] / (R(1) + t2), R(2) * t[1] / (R(1) + t2), R(2) * t[2] / (R(1) + t2)};
    R up[3] = {um[0] + (um[1] * t[2] - um[2] * t[1]), um[1] + (um[2] * t[0] - um[0] * t[2]),
               um[2] + (um[0] * t[1] - um[1] * t[0])};
    R un[3] = {um[0] + (up[1] * s[2] - up[2] * s[1]), um[1] + (up[2] * s[0] - up[0] * s[2]),
               um[2] + (up[0] * s[1] - up[1] * s[0])};
    un[0] += hq * E[0];
    un[1] += hq * E[1];
    un[2] += hq * E[2];
    if (!(fabs(un[0]) < R(1e30) && fabs(un[1]) < R(1e30) && fabs(un[2]) < R(1e30))) err |= ERR_NONFINITE;
    const R g = sqrt(R(1) + un[0] * un[0] + un[1] * un[1] + un[2] * un[2]);

    // ---- move, new cell, Esirkepov frames
    R S0[3][4], DS[3][4];
    int t0[3] = {0, 0, 0};
    int gcell[3] = {0, 0, 0};   // new global cell
#pragma unroll
    for (int a = 0; a < DIM; ++a) {
        if constexpr (T::split) {
            R delta = (un[a] / g) * rd.f_dtd[a];
            if (!(fabs(delta) < R(1))) {
                err |= ERR_MOVE;
                delta = R(0);
            }
            R xn = p.pos[a] + delta;
            esirkepov_axis<R>(dp[a], xn - h[a], ip[a], S0[a], DS[a], t0[a]);
            R f = floor(xn);
            int sh = (int)f;
            R xi2 = xn - f;
            if (xi2 >= R(1)) {
                xi2 = R(0);
                sh += 1;
            }
            if (xi2 < R(0)) xi2 = R(0);
            p.pos[a] = xi2;
            gcell[a] = wrapi(p0[a] + lc[a] + sh, rd.n[a]);
        } else {
            double xn = (double)p.pos[a] + rd.dt * (double)un[a] / (double)g;
            double X1 = xn / rd.d[a];
            if (!(fabs(X1 - X0[a]) < 1.0)) {
                err |= ERR_MOVE;
                xn = (double)p.pos[a];
                X1 = X0[a];
            }
            esirkepov_axis<R>(dp[a], (R)(X1 - (double)ipg[a]), ip[a], S0[a], DS[a], t0[a]);
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

    // ---- Esirkepov deposition into the LDS tile
    const R third = R(1) / R(3);
    R cj[3];
#pragma unroll
    for (int a = 0; a < DIM; ++a) cj[a] = (T::split ? (R)rd.f_cj[a] : (R)(-rd.q * rd.d[a] / rd.dt)) * p.w;
    if constexpr (DIM == 2) {
        const R cz = (T::split ? (R)rd.f_q : (R)rd.q) * p.w * (un[2] / g);
        R *Jx = tile, *Jy = tile + TS, *Jz = tile + 2 * TS;
#pragma unroll
        for (int n = 0; n < 4; ++n) {
            const R yf = S0[1][n] + R(0.5) * DS[1][n];
            R acc = R(0);
#pragma unroll
            for (int m = 0; m < 3; ++m) {
                acc += DS[0][m] * yf;
                atomicAdd(&Jx[(t0[1] + n) * T0 + t0[0] + m], cj[0] * acc);
            }
        }
#pragma unroll
        for (int m = 0; m < 4; ++m) {
            const R xf = S0[0][m] + R(0.5) * DS[0][m];
            R acc = R(0);
#pragma unroll
            for (int n = 0; n < 3; ++n) {
                acc += DS[1][n] * xf;
                atomicAdd(&Jy[(t0[1] + n) * T0 + t0[0] + m], cj[1] * acc);
            }
        }
#pragma unroll
        for (int n = 0; n < 4; ++n)
#pragma unroll
            for (int m = 0; m < 4; ++m) {
                const R wz = S0[0][m] * S0[1][n] + R(0.5) * DS[0][m] * S0[1][n] + R(0.5) * S0[0][m] * DS[1][n] +
                             third * DS[0][m] * DS[1][n];
                atomicAdd(&Jz[(t0[1] + n) * T0 + t0[0] + m], cz * wz);
            }
    } else {
        R *Jc[3] = {tile, tile + TS, tile + 2 * TS};
        // component c flows along axis c; the other two axes (u, v) carry
        // the time-averaged transverse shape product
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            const int u = (c + 1) % 3, v = (c + 2) % 3;
            R tr[4][4];
#pragma unroll
            for (int i = 0; i < 4; ++i)
#pragma unroll
                for (int j = 0; j < 4; ++j) {
                    // keep the operand order of the transverse product in
                    // (y,z), (x,z), (x,y) axis order
                    const int lo = u < v ? u : v, hi = u < v ? v : u;
                    const int il = u < v ? i : j, ih = u < v ? j : i;
                    tr[i][j] = S0[lo][il] * S0[hi][ih] + R(0.5) * DS[lo][il] * S0[hi][ih] +
                               R(0.5) * S0[lo][il] * DS[hi][ih] + third * DS[lo][il] * DS[hi][ih];
                }
#pragma unroll
            for (int i = 0; i < 4; ++i)
#pragma unroll
                for (int j = 0; j < 4; ++j) {
                    R acc = R(0);
#pragma unroll
                    for (int m = 0; m < 3; ++m) {
                        acc += DS[c][m] * tr[i][j];
                        int idx[3];
                        idx[c] = t0[c] + m;
                        idx[u] = t0[u] + i;
                        idx[v] = t0[v] + j;
                        atomicAdd(&Jc[c][(idx[2] * T1 + idx[1]) * T0 + idx[0]], cj[c] * acc);
                    }
                }
        }
    }

    p.u[0] = un[0];
    p.u[1] = un[1];
    p.u[2] = un[2];

    // ---- destination patch and cell inside it
    int dest = 0, mul = 1, packed = 0;
#pragma unroll
    for (int a = 0; a < DIM; ++a) {
        int pa = gcell[a] / P[a];
        dest += pa * mul;
        mul *= rd.np[a];
        packed |= (gcell[a] - pa * P[a]) << (5 * a);
    }
    p.cell = packed;
    return dest;
}

template <int DIM, class T, int PC>
__global__ __launch_bounds__(BLOCK) void push_kernel(const RunDev *__restrict__ runs, const int2 *__restrict__ items,
                                                     int par)
{
    using R = typename T::real;
    constexpr int WN = (PC + 3) * (PC + 3) * (DIM == 3 ? PC + 3 : 1);
    constexpr int TN = (PC + 5) * (PC + 5) * (DIM == 3 ? PC + 5 : 1);
    constexpr int NW = BLOCK / 64;
    __shared__ R s_win[6 * WN];
    __shared__ R s_tile[3 * TN];
    __shared__ int s_wsum[2][NW];

    const int2 item = items[blockIdx.x];
    const RunDev &rd = runs[item.x];
    const int q = item.y;
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;

    const int P[3] = {rd.P[0], rd.P[1], DIM == 3 ? rd.P[2] : 1};
    const int pq[3] = {q % rd.np[0], (q / rd.np[0]) % rd.np[1], DIM == 3 ? q / (rd.np[0] * rd.np[1]) : 0};
    const int p0[3] = {pq[0] * P[0], pq[1] * P[1], pq[2] * P[2]};
    const int rr[3] = {p0[0] / rd.rs[0], p0[1] / rd.rs[1], DIM == 3 ? p0[2] / rd.rs[2] : 0};
    const int region = rr[0] + rd.nreg[0] * (rr[1] + rd.nreg[1] * rr[2]);
    const int o[3] = {p0[0] - rr[0] * rd.rs[0], p0[1] - rr[1] * rd.rs[1], DIM == 3 ? p0[2] - rr[2] * rd.rs[2] : 0};
    const int W0 = P[0] + 3, W1 = P[1] + 3, W2 = DIM == 3 ? P[2] + 3 : 1;
    const int WS = W0 * W1 * W2;
    const int T0 = rd.TA[0], T1 = rd.TA[1];
    const int TS = rd.tsz;

    // transfer (ii): region E^n, Bm^n -> LDS window
    for (int idx = tid; idx < 6 * WS; idx += BLOCK) {
        const int c = idx / WS, rem = idx - c * WS;
        const int wx = rem % W0, tq = rem / W0, wy = tq % W1, wz = tq / W1;
        const int comp = c < 3 ? f_E(par) + c : F_BM + (c - 3);
        const double *A = rcomp(rd, region, comp);
        s_win[idx] = (R)A[rindex(rd, o[0] - 1 + wx, o[1] - 1 + wy, DIM == 3 ? o[2] - 1 + wz : 0)];
    }
    for (int idx = tid; idx < 3 * TS; idx += BLOCK) s_tile[idx] = R(0);
    __syncthreads();

    const long long seg0 = rd.seg[q];
    const int cap = rd.seg[q + 1] - rd.seg[q];
    int n = rd.cnt[q];
    n = n < cap ? n : cap;
    int err = 0;
    int stay = 0;   // stayers compacted so far (uniform)
    int chunk = 0;
    const unsigned long long lt = (1ull << lane) - 1ull;

    for (int base = 0; base < n; base += BLOCK, ++chunk) {
        const int i = base + tid;
        const bool valid = i < n;
        Part<T> pt;
        int dest = q;
        if (valid) {
            load_part<DIM, T>(rd.st, seg0 + i, pt);
            dest = push_one<DIM, T>(rd, s_win, s_tile, W0, W1, WS, T0, T1, TS, p0, P, pt, err);
        }
        const bool st = valid && dest == q;
        const bool lv = valid && dest != q;
        const unsigned long long ms = __ballot(st), ml = __ballot(lv);
        int lbase = 0;
        if (ml) {
            if (lane == 0) lbase = atomicAdd(&rd.ctl->nleave, __popcll(ml));
            lbase = __shfl(lbase, 0);
        }
        if (lane == 0) s_wsum[chunk & 1][wave] = __popcll(ms);
        __syncthreads();   // every particle of the chunk is loaded before any store
        int wb = stay, tot = 0;
#pragma unroll
        for (int w = 0; w < NW; ++w) {
            const int c = s_wsum[chunk & 1][w];
            wb += w < wave ? c : 0;
            tot += c;
        }
        if (st) {
            const int slot = wb + __popcll(ms & lt);
            store_part<DIM, T>(rd.st, seg0 + slot, pt, slot != i);
        }
        if (lv) {
            const int slot = lbase + __popcll(ml & lt);
            if (slot < rd.cap_total) {
                store_part<DIM, T>(rd.lv, slot, pt, true);
                rd.lpatch[slot] = dest;
            } else {
                err |= ERR_CAPACITY;
            }
        }
        stay += tot;
    }

    // particles parked in the spill store that belong to this patch
    const int nsp = min(rd.ctl->nspill, rd.n_total);
    for (int base = 0; base < nsp; base += BLOCK) {
        const int i = base + tid;
        const bool mine = i < nsp && rd.spatch[i] == q;
        Part<T> pt;
        int dest = q;
        if (mine) {
            load_part<DIM, T>(rd.sp, i, pt);
            dest = push_one<DIM, T>(rd, s_win, s_tile, W0, W1, WS, T0, T1, TS, p0, P, pt, err);
        }
        const unsigned long long ml = __ballot(mine);
        int lbase = 0;
        if (ml) {
            if (lane == 0) lbase = atomicAdd(&rd.ctl->nleave, __popcll(ml));
            lbase = __shfl(lbase, 0);
        }
        if (mine) {
            const int slot = lbase + __popcll(ml & lt);
            if (slot < rd.cap_total) {
                store_part<DIM, T>(rd.lv, slot, pt, true);
                rd.lpatch[slot] = dest;
            } else {
                err |= ERR_CAPACITY;
            }
        }
    }

    if (err) atomicOr(&rd.ctl->err, err);
    if (tid == 0) rd.cnt[q] = stay;
    __syncthreads();
    // flush the tile (transfer (i) reads it)
    R *dst = (R *)rd.tiles + (long long)q * 3 * TS;
    for (int idx = tid; idx < 3 * TS; idx += BLOCK) dst[idx] = s_tile[idx];
}

#define PUSH_CASE(D, TT, PCV)                                                                       \
    if (dims == D && split == TT::split && pc == PCV) {                                             \
        push_kernel<D, TT, PCV><<<n_items, BLOCK, 0, s>>>(runs, items, par);                        \
        return hipGetLastError();                                                                   \
    }

hipError_t launch_push(int dims, bool split, int pc, const RunDev *runs, const int2 *items, int n_items, int par,
                       hipStream_t s)
{
    if (n_items <= 0) return hipSuccess;
    PUSH_CASE(2, F32S, 8)
    PUSH_CASE(2, F32S, 16)
    PUSH_CASE(2, F32S, 32)
    PUSH_CASE(2, FP64, 8)
    PUSH_CASE(2, FP64, 16)
    PUSH_CASE(2, FP64, 32)
    PUSH_CASE(3, F32S, 8)
    PUSH_CASE(3, FP64, 8)
    return hipErrorInvalidValue;
}

}  // namespace sdmd
