// k_particles.hip -- particle-store kernels: initial conversion and binning,
// re-layout of the patch-segmented store, export and particle diagnostics.
//
// Binning (the patch decomposition of section 2.2): a particle belongs to
// the patch holding its cell; cell = floor(x/d) clamped to [0, n-1] in the
// FP64 form, the integer cell in the split form.  The store keeps the
// particles of a patch in its segments.  A re-layout gives every patch new
// segments (live count + 50 % + 32 capacity each) and moves the live and
// parked particles into them; it runs at init (binning of the initial
// state) and whenever particles had to be parked because a segment was full.
#include "launch.h"
#include "part.h"
#include "sdmd_dev.h"

namespace sdmd {

// ---------------------------------------------------------------- convert
template <int DIM, class T>
__global__ __launch_bounds__(BLOCK) void convert_kernel(const RunDev *__restrict__ runs, int run, int n,
                                                        const double *__restrict__ x, const double *__restrict__ y,
                                                        const double *__restrict__ z, const double *__restrict__ ux,
                                                        const double *__restrict__ uy, const double *__restrict__ uz,
                                                        const double *__restrict__ w, const uint32_t *__restrict__ id)
{
    using R = typename T::real;
    const RunDev &rd = runs[run];
    const int i = blockIdx.x * BLOCK + threadIdx.x;
    if (i == 0) rd.ctl->nspill = n;
    if (i >= n) return;
    const double *pos[3] = {x, y, z};
    int err = 0;
    Part<T> p;
    int dest = 0, mul = 1, packed = 0;
#pragma unroll
    for (int a = 0; a < DIM; ++a) {
        double xa = pos[a][i];
        if (!(xa >= 0.0 && xa < rd.L[a])) {
            err |= ERR_RANGE;
            xa = 0.0;
        }
        int c = (int)floor(xa / rd.d[a]);
        c = c > rd.n[a] - 1 ? rd.n[a] - 1 : (c < 0 ? 0 : c);
        if constexpr (T::split) {
            float f = (float)(xa / rd.d[a] - (double)c);
            if (f < 0.0f) f = 0.0f;
            if (f >= 1.0f) {
                f = 0.0f;
                c += 1;
                if (c >= rd.n[a]) c -= rd.n[a];
            }
            p.pos[a] = f;
        } else {
            p.pos[a] = xa;
        }
        const int pa = c / rd.P[a];
        dest += pa * mul;
        mul *= rd.np[a];
        packed |= (c - pa * rd.P[a]) << (5 * a);
    }
    p.cell = packed;
    const double u[3] = {ux[i], uy[i], uz[i]};
    for (int a = 0; a < 3; ++a) {
        if (!(fabs(u[a]) < 1e30)) err |= ERR_NONFINITE;
        p.u[a] = (R)u[a];
    }
    if (!(fabs(w[i]) < 1e300)) err |= ERR_NONFINITE;
    p.w = (R)w[i];
    p.id = id ? id[i] : (uint32_t)i;
    store_part<DIM, T>(rd.sp, i, p, true);
    rd.spatch[i] = dest;
    if (err) atomicOr(&rd.ctl->err, err);
}

// ---------------------------------------------------------------- re-layout
constexpr int PLAN_BLOCK = 1024;

// block-wide exclusive scan of per-thread values (PLAN_BLOCK threads)
__device__ long long block_exclusive_scan(long long v, long long *buf, long long &total)
{
    const int tid = threadIdx.x;
    buf[tid] = v;
    __syncthreads();
    for (int off = 1; off < PLAN_BLOCK; off <<= 1) {
        const long long t = tid >= off ? buf[tid - off] : 0;
        __syncthreads();
        buf[tid] += t;
        __syncthreads();
    }
    total = buf[PLAN_BLOCK - 1];
    const long long ex = buf[tid] - v;
    __syncthreads();
    return ex;
}

constexpr int MAX_OLD_SEGS = 1024;      // segments per patch (LDS prefix of the move kernel)
constexpr int PLAN_LDS_PATCHES = 16384; // patch counts the planner histograms in LDS

// segments of a patch holding t particles
__device__ __forceinline__ int segs_for(int t, int cs) { return min(MAX_OLD_SEGS, max(1, (t + cs - 1) / cs)); }

// Plan a re-layout of one run, in three launches:
//   relayout_tally_kernel (one workgroup per run): whether to re-lay out at
//     all (parked particles, or forced), then per patch the live particles
//     of its segments and the first move chunk of each patch;
//   relayout_count_kernel (many workgroups per run): the parked particles
//     of each patch, added to those totals;
//   relayout_plan_kernel (one workgroup per run): the number of segments of
//     each patch K_p = ceil(total / seg_cap), an even split of the total
//     over them, and each segment's capacity (live + 50 % + 32, or an even
//     share of the free slots if that does not fit).
__global__ __launch_bounds__(PLAN_BLOCK) void relayout_tally_kernel(const RunDev *__restrict__ runs,
                                                                    const int *__restrict__ slots, int force)
{
    const RunDev &rd = runs[slots[blockIdx.x]];
    __shared__ long long buf[PLAN_BLOCK];
    const int tid = threadIdx.x;
    const int nsp = min(rd.ctl->nspill, rd.n_total);
    if (!force && nsp == 0) {
        if (tid == 0) rd.ctl->relayout = 0;
        return;
    }
    if (tid == 0) rd.ctl->relayout = 1;   // tentative: the planner decides
    const int np = rd.n_patch;
    const int nseg = rd.ctl->nseg;
    for (int p = tid; p < np; p += PLAN_BLOCK) {
        rd.tot[p] = 0;
        rd.fill[p] = 0;
    }
    __syncthreads();
    for (int sg = tid; sg < nseg; sg += PLAN_BLOCK) {
        const int cap = rd.sseg[sg + 1] - rd.sseg[sg];
        atomicAdd(&rd.tot[rd.spat[sg]], min(rd.scnt[sg], cap));
    }
    __syncthreads();
    for (int p = tid; p < np; p += PLAN_BLOCK) rd.preg[p] = rd.tot[p];
    __syncthreads();
    {
        // move chunks of each patch's segment particles -> first chunk per patch
        const int per = (np + PLAN_BLOCK - 1) / PLAN_BLOCK;
        const int q0 = tid * per, q1 = min(np, q0 + per);
        long long nc = 0;
        for (int p = q0; p < q1; ++p) nc += (rd.preg[p] + MOVE_CHUNK - 1) / MOVE_CHUNK;
        long long ncall;
        long long o = block_exclusive_scan(nc, buf, ncall);
        for (int p = q0; p < q1; ++p) {
            rd.cpre[p] = (int)o;
            o += (rd.preg[p] + MOVE_CHUNK - 1) / MOVE_CHUNK;
        }
        if (tid == 0) rd.cpre[np] = (int)ncall;
    }
}

// Parked particles per patch, added to the totals: workgroup b of nb takes
// an even slice of the spill store, counts it in an LDS histogram when the
// patch count fits (global atomics otherwise) and adds the non-zero counts.
// A wavefront whose parked particles all belong to one patch (the usual
// case at set-up, when every particle is parked in input order) adds once:
// 64 lanes on one counter would serialise.
__global__ __launch_bounds__(BLOCK) void relayout_count_kernel(const RunDev *__restrict__ runs,
                                                               const int *__restrict__ slots)
{
    const RunDev &rd = runs[slots[blockIdx.y]];
    if (!rd.ctl->relayout) return;
    __shared__ int s_hist[PLAN_LDS_PATCHES];
    const int tid = threadIdx.x, lane = tid & 63;
    const int nsp = min(rd.ctl->nspill, rd.n_total);
    const int np = rd.n_patch;
    const int nb = gridDim.x;
    const long long i_begin = (long long)nsp * blockIdx.x / nb, i_end = (long long)nsp * (blockIdx.x + 1) / nb;
    if (i_begin >= i_end) return;
    const bool lds = np <= PLAN_LDS_PATCHES;
    if (lds) {
        for (int p = tid; p < np; p += BLOCK) s_hist[p] = 0;
        __syncthreads();
    }
    int *hist = lds ? s_hist : rd.tot;
    constexpr int HU = 8;   // rounds of loads in flight per thread
    for (long long i0 = i_begin; i0 < i_end; i0 += HU * BLOCK) {
        int qv[HU];
#pragma unroll
        for (int u = 0; u < HU; ++u) {
            const long long i = i0 + u * BLOCK + tid;
            qv[u] = i < i_end ? gp(rd.spatch)[i] : -1;
        }
#pragma unroll
        for (int u = 0; u < HU; ++u) {
            const int q = qv[u];
            const bool v = q >= 0 && q < np;
            const int q0 = __shfl(q, 0);
            if (__all(!v || q == q0)) {
                const unsigned long long mv = __ballot(v);
                if (lane == 0 && mv) atomicAdd(&hist[q0], __popcll(mv));
            } else if (v) {
                atomicAdd(&hist[q], 1);
            }
        }
    }
    if (lds) {
        __syncthreads();
        for (int p = tid; p < np; p += BLOCK) {
            const int c = s_hist[p];
            if (c) atomicAdd(&rd.tot[p], c);
        }
    }
}

__global__ __launch_bounds__(PLAN_BLOCK) void relayout_plan_kernel(const RunDev *__restrict__ runs,
                                                                   const int *__restrict__ slots)
{
    const RunDev &rd = runs[slots[blockIdx.x]];
    __shared__ long long buf[PLAN_BLOCK];
    const int tid = threadIdx.x;
    if (!rd.ctl->relayout) return;
    const int np = rd.n_patch;
    const int cs = rd.seg_cap > 0 ? rd.seg_cap : 1;
    const int chunk = (np + PLAN_BLOCK - 1) / PLAN_BLOCK;
    const int p0 = tid * chunk, p1 = min(np, p0 + chunk);
    // segments per patch -> first segment of each patch
    long long nk = 0;
    for (int p = p0; p < p1; ++p) nk += segs_for(rd.tot[p], cs);
    long long nseg2;
    long long koff = block_exclusive_scan(nk, buf, nseg2);
    for (int p = p0; p < p1; ++p) {
        rd.pseg2[p] = (int)koff;
        koff += segs_for(rd.tot[p], cs);
    }
    if (tid == 0) rd.pseg2[np] = (int)nseg2;
    // capacities
    long long want = 0;
    for (int p = p0; p < p1; ++p) {
        const int t = rd.tot[p], K = segs_for(t, cs);
        for (int k = 0; k < K; ++k) {
            const int l = t / K + (k < t % K ? 1 : 0);
            want += l + l / 2 + 32;
        }
    }
    long long total;
    block_exclusive_scan(want, buf, total);
    const bool tight = total > rd.cap_total;
    const int slack = tight ? (int)((rd.cap_total - rd.n_total) / (nseg2 > 0 ? nseg2 : 1)) : 0;
    long long mine = 0;
    for (int p = p0; p < p1; ++p) {
        const int t = rd.tot[p], K = segs_for(t, cs);
        for (int k = 0; k < K; ++k) {
            const int l = t / K + (k < t % K ? 1 : 0);
            mine += tight ? l + slack : l + l / 2 + 32;
        }
    }
    long long tot2;
    long long off = block_exclusive_scan(mine, buf, tot2);
    for (int p = p0; p < p1; ++p) {
        const int t = rd.tot[p], K = segs_for(t, cs);
        const int k0 = rd.pseg2[p];
        for (int k = 0; k < K && k0 + k < rd.seg_max; ++k) {
            const int l = t / K + (k < t % K ? 1 : 0);
            rd.sseg2[k0 + k] = (int)off;
            rd.scnt2[k0 + k] = l;
            rd.spat2[k0 + k] = p;
            off += tight ? l + slack : l + l / 2 + 32;
        }
    }
    if (tid == 0) {
        if (nseg2 <= rd.seg_max) rd.sseg2[nseg2] = (int)tot2;
        rd.ctl->relayout = (nseg2 <= rd.seg_max && tot2 <= rd.cap_total) ? 1 : 0;
        if (!rd.ctl->relayout) atomicOr(&rd.ctl->err, ERR_CAPACITY);
    }
}

// Sort key of a stored particle's cell inside its patch, for the in-patch
// ordering of a re-layout: x fastest, then y (2D); x, then z, then y (3D,
// so that the 64 lanes of a wavefront take an x-z slice of an 8^3 patch,
// the footprint the particle kernel's padded LDS planes are laid out for).
template <int DIM, class T>
__device__ __forceinline__ int local_cell(const RunDev &rd, const Store &s, long long i, int q)
{
    int v[3] = {0, 0, 0};
    if constexpr (T::split) {
        const int c = s.cell[i];
#pragma unroll
        for (int a = 0; a < DIM; ++a) {
            const int w = (c >> (5 * a)) & 31;
            v[a] = w < rd.P[a] ? w : rd.P[a] - 1;
        }
    } else {
        const int pq[3] = {q % rd.np[0], (q / rd.np[0]) % rd.np[1], DIM == 3 ? q / (rd.np[0] * rd.np[1]) : 0};
#pragma unroll
        for (int a = 0; a < DIM; ++a) {
            const int w = (int)floor(((const double *)s.pos[a])[i] / rd.d[a]) - pq[a] * rd.P[a];
            v[a] = w < 0 ? 0 : (w > rd.P[a] - 1 ? rd.P[a] - 1 : w);
        }
    }
    if constexpr (DIM == 3) return v[0] + rd.P[0] * (v[2] + rd.P[2] * v[1]);
    return v[0] + rd.P[0] * v[1];
}

// Sub-cell half of a stored particle: bit a is set when it lies in the upper
// half of its cell along axis a, i.e. when its nearest primal node is the
// cell's upper one.  Within a cell particles are ordered by these bits, so
// that the lanes of a wavefront (one particle of each of 64 cells, all of
// the same rank in their cells) mostly share them: their interpolation and
// deposition frames are then all shifted alike and no two lanes of a
// wavefront update the same LDS tile node in one instruction (two lanes on
// one address serialise an LDS atomic, measured ~2.4x the cost on gfx950).
template <int DIM, class T>
__device__ __forceinline__ int half_bits(const RunDev &rd, const Store &s, long long i)
{
    int b = 0;
#pragma unroll
    for (int a = 0; a < DIM; ++a) {
        bool up;
        if constexpr (T::split) {
            up = gp((const float *)s.pos[a])[i] >= 0.5f;
        } else {
            const double X = gp((const double *)s.pos[a])[i] / rd.d[a];
            up = X - floor(X) >= 0.5;
        }
        b |= (up ? 1 : 0) << a;
    }
    return b;
}

// position j of a patch's new particle list -> slot in its new segments
// (segment k of K holds the k-th even share of the patch's t particles)
__device__ __forceinline__ long long new_slot(const RunDev &rd, int p, int t, int j)
{
    const int k0 = rd.pseg2[p], K = rd.pseg2[p + 1] - k0;
    const int base = t / K, extra = t % K;
    int k, o;
    if (j < extra * (base + 1)) {
        k = j / (base + 1);
        o = j - k * (base + 1);
    } else {
        const int jj = j - extra * (base + 1);
        k = extra + (base > 0 ? jj / base : 0);
        o = jj - (k - extra) * base;
    }
    return (long long)rd.sseg2[k0 + k] + o;
}

constexpr int MAX_PATCH_CELLS = 1024;   // 32 x 32 (2D) / 8 x 8 x 8 (3D)
constexpr int NEW_SEGS_LDS = 64;        // new segments of a patch whose first slots the move kernel keeps in LDS
constexpr int MAX_SORT_BINS = 4096;     // cells x sub-cell halves (32 x 32 x 4, 8^3 x 8)

template <int DIM, class T>
__global__ __launch_bounds__(BLOCK) void relayout_move_kernel(const RunDev *__restrict__ runs,
                                                             const int *__restrict__ slots)
{
    const RunDev &rd = runs[slots[blockIdx.y]];
    if (!rd.ctl->relayout) return;
    const int np = rd.n_patch;
    const int cb = move_chunk_blocks(np, rd.n_total);
    const int n_spill_blocks = (int)gridDim.x - cb;   // >= 1 by construction
    if ((int)blockIdx.x < cb) {
        // One chunk of a patch's segment particles: with nch chunks, chunk
        // k takes every nch-th particle of the old storage order starting at
        // k (so that each chunk samples the whole patch), at most MOVE_CHUNK
        // of them.  The chunk is sorted by cell and, inside a cell, by
        // sub-cell half (counting sort in LDS), which gives every particle
        // its rank r inside its cell.  It is stored round-robin over the
        // cells: all rank-0 particles in cell order, then all rank-1
        // particles, ...; the particle of rank r in cell k goes to position
        // base[r] + (cells before k holding more than r particles), with
        // base[r] the number of particles of rank < r.  Consecutive
        // positions -- the lanes of a wavefront -- then hold distinct
        // neighbouring cells whatever the occupancy (uneven cells of a
        // plasma wake included), so their field-window reads and tile
        // updates fall on different LDS addresses.  Chunks take consecutive
        // ranges of the patch's positions, which are split evenly over its
        // new segments.
        __shared__ int s_off[MAX_SORT_BINS];
        __shared__ int s_pos[MOVE_CHUNK];    // sorted index -> position in the chunk
        __shared__ int s_sum[BLOCK];
        __shared__ int s_ws[2][BLOCK / 64];
        __shared__ int s_seg[MAX_OLD_SEGS + 1];
        __shared__ int s_p, s_cmax;
        __shared__ int s_new[NEW_SEGS_LDS];
        const int b = blockIdx.x;
        if (b >= rd.cpre[np]) return;        // more chunk blocks than chunks
        const int tid = threadIdx.x;
        // the patch p with cpre[p] <= b < cpre[p + 1]: cpre is nondecreasing
        // and cpre[0] = 0, so p + 1 is the number of entries <= b, counted
        // by all threads with their loads in flight together
        if (tid == 0) s_p = -1;
        __syncthreads();
        {
            int c = 0;
#pragma unroll 8
            for (int k = tid; k < np; k += BLOCK) c += rd.cpre[k] <= b ? 1 : 0;
            if (c) atomicAdd(&s_p, c);
        }
        __syncthreads();
        const int p = s_p;
        const int kc = b - rd.cpre[p], nch = rd.cpre[p + 1] - rd.cpre[p];
        const int k0 = rd.pseg[p], K = min(rd.pseg[p + 1] - k0, MAX_OLD_SEGS);
        // prefix of the old segments' live counts
        if (tid == 0) {
            int acc = 0;
            for (int k = 0; k < K; ++k) {
                s_seg[k] = acc;
                const int cap = rd.sseg[k0 + k + 1] - rd.sseg[k0 + k];
                acc += min(rd.scnt[k0 + k], cap);
            }
            s_seg[K] = acc;
        }
        const int ncell = rd.P[0] * rd.P[1] * (DIM == 3 ? rd.P[2] : 1);
        constexpr int Q = 1 << DIM;                                      // bins per cell
        for (int k = tid; k < ncell * Q; k += BLOCK) s_off[k] = 0;
        if (tid == 0) s_cmax = 0;
        __syncthreads();
        const int r = min(s_seg[K], rd.preg[p]);
        const int m = r / nch + (kc < r % nch ? 1 : 0);                  // particles of this chunk
        const int base = kc * (r / nch) + min(kc, r % nch);             // its first position
        const int t = rd.tot[p];
        // the patch's new segments: their first slots in LDS when they are
        // few (the usual case), so placing a particle needs no dependent load
        const int kn0 = rd.pseg2[p], Kn = rd.pseg2[p + 1] - kn0;
        const bool new_lds = Kn <= NEW_SEGS_LDS;
        if (new_lds)
            for (int k = tid; k < Kn; k += BLOCK) s_new[k] = rd.sseg2[kn0 + k];
        const int nbase = Kn > 0 ? t / Kn : 0, nextra = Kn > 0 ? t % Kn : 0;
        auto slot_of = [&](int j) -> long long {   // as new_slot(rd, p, t, j)
            int k, o;
            if (j < nextra * (nbase + 1)) {
                k = j / (nbase + 1);
                o = j - k * (nbase + 1);
            } else {
                const int jj = j - nextra * (nbase + 1);
                k = nextra + (nbase > 0 ? jj / nbase : 0);
                o = jj - (k - nextra) * nbase;
            }
            return (long long)(new_lds ? s_new[k] : rd.sseg2[kn0 + k]) + o;
        };
        auto src = [&](int i) -> long long {   // i-th live particle of the patch
            int lo = 0, hi = K;                // s_seg[lo] <= i < s_seg[hi]
            while (hi - lo > 1) {
                const int mid = (lo + hi) >> 1;
                if (s_seg[mid] <= i) lo = mid; else hi = mid;
            }
            return (long long)rd.sseg[k0 + lo] + (i - s_seg[lo]);
        };
        auto bin = [&](long long si) {
            return local_cell<DIM, T>(rd, rd.st, si, p) * Q + half_bits<DIM, T>(rd, rd.st, si);
        };
        // Both passes over the chunk take MU particles per thread per round,
        // the round's loads written ahead of its LDS updates so that they
        // can be in flight together.
        constexpr int MU = 4;
        for (int i0 = 0; i0 < m; i0 += MU * BLOCK) {
            int bn[MU];
#pragma unroll
            for (int u = 0; u < MU; ++u) {
                const int i = i0 + u * BLOCK + tid;
                bn[u] = i < m ? bin(src(kc + i * nch)) : -1;
            }
#pragma unroll
            for (int u = 0; u < MU; ++u)
                if (bn[u] >= 0) atomicAdd(&s_off[bn[u]], 1);
        }
        __syncthreads();
        // exclusive scan of the bin counts: contiguous runs of whole cells
        // per thread
        const int per = (ncell + BLOCK - 1) / BLOCK;
        const int c0 = tid * per * Q, c1 = min(ncell, tid * per + per) * Q;
        int run = 0;
        for (int k = c0; k < c1; ++k) run += s_off[k];
        s_sum[tid] = run;
        __syncthreads();
        for (int off = 1; off < BLOCK; off <<= 1) {
            const int v = tid >= off ? s_sum[tid - off] : 0;
            __syncthreads();
            s_sum[tid] += v;
            __syncthreads();
        }
        int acc = s_sum[tid] - run;
        for (int k = c0; k < c1; ++k) {
            const int v = s_off[k];
            s_off[k] = acc;
            acc += v;
        }
        __syncthreads();
        // cells of this thread (the same contiguous run): first sorted
        // index and particle count
        constexpr int CPT = MAX_PATCH_CELLS / BLOCK;
        const int lane = tid & 63, wave = tid >> 6;
        int cst[CPT], ccnt[CPT];
        int cmax = 0;
#pragma unroll
        for (int u = 0; u < CPT; ++u) {
            const int k = tid * per + u;
            const bool own = u < per && k < ncell;
            cst[u] = own ? s_off[k * Q] : 0;
            ccnt[u] = own ? (k + 1 < ncell ? s_off[(k + 1) * Q] : m) - cst[u] : 0;
            cmax = max(cmax, ccnt[u]);
        }
        if (cmax) atomicMax(&s_cmax, cmax);
        __syncthreads();
        const int rmax = s_cmax;
        int rb = 0;   // base[r]
        for (int rk = 0; rk < rmax; ++rk) {
            int f = 0;
#pragma unroll
            for (int u = 0; u < CPT; ++u) f += ccnt[u] > rk ? 1 : 0;
            int x = f;   // inclusive scan over the wavefront
#pragma unroll
            for (int o = 1; o < 64; o <<= 1) {
                const int y = __shfl_up(x, o);
                if (lane >= o) x += y;
            }
            if (lane == 63) s_ws[rk & 1][wave] = x;
            __syncthreads();   // s_ws[rk & 1] is rewritten two ranks later, after the next barrier
            int pre = 0, tot = 0;
#pragma unroll
            for (int w = 0; w < BLOCK / 64; ++w) {
                const int v = s_ws[rk & 1][w];
                pre += w < wave ? v : 0;
                tot += v;
            }
            int ex = rb + pre + x - f;
#pragma unroll
            for (int u = 0; u < CPT; ++u)
                if (ccnt[u] > rk) s_pos[cst[u] + rk] = ex++;
            rb += tot;
        }
        __syncthreads();
        for (int i0 = 0; i0 < m; i0 += MU * BLOCK) {
            Part<T> pt[MU];
            int bn[MU];
#pragma unroll
            for (int u = 0; u < MU; ++u) {
                const int i = i0 + u * BLOCK + tid;
                bn[u] = -1;
                if (i < m) {
                    const long long si = src(kc + i * nch);
                    bn[u] = bin(si);
                    load_part<DIM, T>(rd.st, si, pt[u]);
                }
            }
#pragma unroll
            for (int u = 0; u < MU; ++u)
                if (bn[u] >= 0) {
                    const int j = atomicAdd(&s_off[bn[u]], 1);
                    store_part<DIM, T>(rd.lv, slot_of(base + s_pos[j]), pt[u], true);
                }
        }
        return;
    }
    // parked particles follow the patch-store ones in their patch's list;
    // the lanes of a wavefront bound for one patch share one position claim
    // (claims on one counter serialise, and parked particles crowd into the
    // few patches that overflowed)
    const int nsp = min(rd.ctl->nspill, rd.n_total);
    const int lane = threadIdx.x & 63;
    for (int i0 = (blockIdx.x - cb) * BLOCK; i0 < nsp; i0 += n_spill_blocks * BLOCK) {
        const int i = i0 + (int)threadIdx.x;
        const bool valid = i < nsp;
        const int q = valid ? rd.spatch[i] : -1;
        unsigned long long todo = __ballot(valid), mine = 0;
        bool lead = false;
        while (todo) {
            const int l = __builtin_ctzll(todo);
            const int ql = __shfl(q, l);
            const unsigned long long same = __ballot(valid && q == ql);
            if (valid && q == ql) {
                mine = same;
                lead = lane == l;
            }
            todo &= ~same;
        }
        int b = 0;
        if (lead) b = atomicAdd(&rd.fill[q], __popcll(mine));
        b = __shfl(b, valid ? __builtin_ctzll(mine) : lane);
        if (valid) {
            const int pos = rd.preg[q] + b + __popcll(mine & ((1ull << lane) - 1ull));
            copy_part<DIM, T>(rd.sp, i, rd.lv, new_slot(rd, q, rd.tot[q], pos));
        }
    }
}

// The moved particles are in the scratch store: the scratch store becomes
// the patch store (a swap of the two store descriptors in the run table, no
// copy) and the new segment table is installed.
template <int DIM, class T>
__global__ __launch_bounds__(BLOCK) void relayout_commit_kernel(RunDev *__restrict__ runs, const int *__restrict__ slots)
{
    RunDev &rd = runs[slots[blockIdx.y]];
    if (!rd.ctl->relayout) return;
    const int np = rd.n_patch;
    const int S = rd.pseg2[np];
    const int stride = gridDim.x * BLOCK;
    for (int k = blockIdx.x * BLOCK + threadIdx.x; k <= S; k += stride) {
        rd.sseg[k] = rd.sseg2[k];
        if (k < S) {
            rd.scnt[k] = rd.scnt2[k];
            rd.spat[k] = rd.spat2[k];
            rd.nlv[k] = 0;
        }
    }
    // every tile slot may now hold another patch's stale current: the next
    // particle phase rewrites all of them
    for (int k = blockIdx.x * BLOCK + threadIdx.x; k < rd.seg_max; k += stride) rd.tflag[k] = 1;
    for (int p = blockIdx.x * BLOCK + threadIdx.x; p <= np; p += stride) {
        rd.pseg[p] = rd.pseg2[p];
        rd.spcnt[p] = 0;   // the parked particles are in the patch store now
    }
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        const Store t = rd.st;
        rd.st = rd.lv;
        rd.lv = t;
        rd.ctl->nspill = 0;
        rd.ctl->nseg = S;
        rd.ctl->n_relayout += 1;
    }
}

// ---------------------------------------------------------------- export
template <int DIM, class T>
__device__ __forceinline__ void export_one(const RunDev &rd, const Store &s, long long i, int q, long long o, double *x,
                                           double *y, double *z, double *ux, double *uy, double *uz, double *w,
                                           uint32_t *id, int *patch)
{
    Part<T> p;
    load_part<DIM, T>(s, i, p);
    double *pos[3] = {x, y, z};
    const int pq[3] = {q % rd.np[0], (q / rd.np[0]) % rd.np[1], DIM == 3 ? q / (rd.np[0] * rd.np[1]) : 0};
#pragma unroll
    for (int a = 0; a < DIM; ++a) {
        if (!pos[a]) continue;
        if constexpr (T::split) {
            const int c = pq[a] * rd.P[a] + ((p.cell >> (5 * a)) & 31);
            pos[a][o] = ((double)c + (double)p.pos[a]) * rd.d[a];
        } else {
            pos[a][o] = (double)p.pos[a];
        }
    }
    if (DIM == 2 && z) z[o] = 0.0;
    if (ux) ux[o] = (double)p.u[0];
    if (uy) uy[o] = (double)p.u[1];
    if (uz) uz[o] = (double)p.u[2];
    if (w) w[o] = (double)p.w;
    if (id) id[o] = s.id ? p.id : 0u;
    if (patch) patch[o] = q;
}

template <int DIM, class T>
__global__ __launch_bounds__(BLOCK) void export_kernel(const RunDev *__restrict__ runs, int run, int nspill,
                                                       const int *__restrict__ off, double *x, double *y, double *z,
                                                       double *ux, double *uy, double *uz, double *w, uint32_t *id,
                                                       int *patch)
{
    // blocks [0, seg_max): one segment each; the rest: the spill store.
    // off[s] = output offset of segment s, off[nseg] = start of the spill part
    const RunDev &rd = runs[run];
    const int S = rd.ctl->nseg;
    if ((int)blockIdx.x < rd.seg_max) {
        const int sg = blockIdx.x;
        if (sg >= S) return;
        const int cap = rd.sseg[sg + 1] - rd.sseg[sg];
        const int r = min(rd.scnt[sg], cap);
        const int q = rd.spat[sg];
        for (int i = threadIdx.x; i < r; i += BLOCK)
            export_one<DIM, T>(rd, rd.st, (long long)rd.sseg[sg] + i, q, (long long)off[sg] + i, x, y, z, ux, uy, uz,
                               w, id, patch);
        return;
    }
    const int nb = gridDim.x - rd.seg_max;
    for (int i = (blockIdx.x - rd.seg_max) * BLOCK + threadIdx.x; i < nspill; i += nb * BLOCK)
        export_one<DIM, T>(rd, rd.sp, i, rd.spatch[i], (long long)off[S] + i, x, y, z, ux, uy, uz, w, id, patch);
}

// ---------------------------------------------------------------- kinetic energy
template <int DIM, class T>
__global__ __launch_bounds__(BLOCK) void kinetic_kernel(const RunDev *__restrict__ runs, int run, int nspill,
                                                        double *__restrict__ partial)
{
    using R = typename T::real;
    const RunDev &rd = runs[run];
    __shared__ double sk[BLOCK];
    double k = 0.0;
    auto add = [&](const Store &s, long long i) {
        const double a = ((const R *)s.u[0])[i], b = ((const R *)s.u[1])[i], c = ((const R *)s.u[2])[i];
        const double g = sqrt(1.0 + a * a + b * b + c * c);
        k += rd.m * (double)((const R *)s.w)[i] * (g - 1.0);
    };
    if ((int)blockIdx.x < rd.seg_max) {
        const int sg = blockIdx.x;
        if (sg < rd.ctl->nseg) {
            const int cap = rd.sseg[sg + 1] - rd.sseg[sg];
            const int r = min(rd.scnt[sg], cap);
            for (int i = threadIdx.x; i < r; i += BLOCK) add(rd.st, (long long)rd.sseg[sg] + i);
        }
    } else {
        for (int i = threadIdx.x; i < nspill; i += BLOCK) add(rd.sp, i);
    }
    sk[threadIdx.x] = k;
    __syncthreads();
    for (int w = BLOCK / 2; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) sk[threadIdx.x] += sk[threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0) partial[blockIdx.x] = sk[0];
}

// ---------------------------------------------------------------- charge density
// rho = sum q w S(X - node) at the primal nodes (quadratic shapes).  A
// particle of a patch with origin p0 and edge P touches nodes p0-1 ..
// p0+P+1 per axis, so a segment's charge is first summed in an LDS tile of
// (P+3)^DIM nodes and then added into the global array once per node (one
// global atomic per tile node instead of 3^DIM per particle).  Parked
// particles, and any particle found outside its patch's tile, add straight
// into the global array.  The deterministic mode sums 64-bit fixed-point
// charges (see to_fixed) in both places.
// nodes of the largest tile: (P+3)^2 = 1225 for P <= 32 in 2D, (P+3)^3 = 1331
// for P <= 8 in 3D
constexpr int RHO_TILE_ALLOC = 11 * 11 * 11;
static_assert(35 * 35 <= RHO_TILE_ALLOC, "2D charge tile");

template <int DIM, class T>
__device__ __forceinline__ void rho_weights(const RunDev &rd, const Part<T> &p, int q, int base[3], double wt[3][3])
{
    const int pq[3] = {q % rd.np[0], (q / rd.np[0]) % rd.np[1], DIM == 3 ? q / (rd.np[0] * rd.np[1]) : 0};
#pragma unroll
    for (int a = 0; a < DIM; ++a) {
        double X;
        if constexpr (T::split)
            X = (double)(pq[a] * rd.P[a] + ((p.cell >> (5 * a)) & 31)) + (double)p.pos[a];
        else
            X = (double)p.pos[a] / rd.d[a];
        const double f = floor(X + 0.5);
        base[a] = (int)f - 1;
        shape3(X - f, wt[a][0], wt[a][1], wt[a][2]);
    }
}

__device__ __forceinline__ void rho_add(double *dst, double v, const RunDev &rd)
{
    if (rd.det)
        atomicAdd((unsigned long long *)dst, to_fixed(v * rd.rscale));
    else
        atomicAdd(dst, v);
}

// one particle straight into the global array
template <int DIM, class T>
__device__ __forceinline__ void rho_global(const RunDev &rd, const Part<T> &p, int q, double *rho)
{
    int base[3] = {0, 0, 0};
    double wt[3][3] = {{1, 0, 0}, {1, 0, 0}, {1, 0, 0}};
    rho_weights<DIM, T>(rd, p, q, base, wt);
    const double qw = rd.q * (double)p.w;
    const int nk = DIM == 3 ? 3 : 1;
    for (int k = 0; k < nk; ++k)
        for (int j = 0; j < 3; ++j)
            for (int ii = 0; ii < 3; ++ii) {
                const int gi = wrap1(base[0] + ii, rd.n[0]), gj = wrap1(base[1] + j, rd.n[1]);
                const int gk = DIM == 3 ? wrap1(base[2] + k, rd.n[2]) : 0;
                const double v = qw * wt[0][ii] * wt[1][j] * (DIM == 3 ? wt[2][k] : 1.0);
                rho_add(&rho[gi + (long long)rd.n[0] * (gj + (long long)rd.n[1] * gk)], v, rd);
            }
}

template <int DIM, class T>
__global__ __launch_bounds__(BLOCK) void rho_kernel(const RunDev *__restrict__ runs, int run, int nspill,
                                                    double *__restrict__ rho)
{
    const RunDev &rd = runs[run];
    if ((int)blockIdx.x >= rd.seg_max) {
        for (int i = threadIdx.x; i < nspill; i += BLOCK) {
            Part<T> p;
            load_part<DIM, T>(rd.sp, i, p);
            rho_global<DIM, T>(rd, p, rd.spatch[i], rho);
        }
        return;
    }
    const int sg = blockIdx.x;
    if (sg >= rd.ctl->nseg) return;
    __shared__ double s_r[RHO_TILE_ALLOC];
    const int cap = rd.sseg[sg + 1] - rd.sseg[sg];
    const int r = min(rd.scnt[sg], cap);
    if (r <= 0) return;
    const int q = rd.spat[sg];
    const int P[3] = {rd.P[0], rd.P[1], DIM == 3 ? rd.P[2] : 1};
    const int E0 = P[0] + 3, E1 = P[1] + 3, E2 = DIM == 3 ? P[2] + 3 : 1;   // tile extent
    const int pq[3] = {q % rd.np[0], (q / rd.np[0]) % rd.np[1], DIM == 3 ? q / (rd.np[0] * rd.np[1]) : 0};
    const int o[3] = {pq[0] * P[0] - 1, pq[1] * P[1] - 1, DIM == 3 ? pq[2] * P[2] - 1 : 0};   // tile origin
    for (int t = threadIdx.x; t < E0 * E1 * E2; t += BLOCK) s_r[t] = 0.0;   // also the integer 0
    __syncthreads();
    const double qw0 = rd.q;
    for (int i = threadIdx.x; i < r; i += BLOCK) {
        Part<T> p;
        load_part<DIM, T>(rd.st, (long long)rd.sseg[sg] + i, p);
        int base[3] = {0, 0, 0};
        double wt[3][3] = {{1, 0, 0}, {1, 0, 0}, {1, 0, 0}};
        rho_weights<DIM, T>(rd, p, q, base, wt);
        const int l0 = base[0] - o[0], l1 = base[1] - o[1], l2 = DIM == 3 ? base[2] - o[2] : 0;
        if (l0 < 0 || l0 + 2 >= E0 || l1 < 0 || l1 + 2 >= E1 || (DIM == 3 && (l2 < 0 || l2 + 2 >= E2))) {
            rho_global<DIM, T>(rd, p, q, rho);   // not inside the patch's tile
            continue;
        }
        const double qw = qw0 * (double)p.w;
        const int nk = DIM == 3 ? 3 : 1;
        for (int k = 0; k < nk; ++k)
            for (int j = 0; j < 3; ++j)
                for (int ii = 0; ii < 3; ++ii) {
                    const double v = qw * wt[0][ii] * wt[1][j] * (DIM == 3 ? wt[2][k] : 1.0);
                    double *dst = &s_r[((l2 + k) * E1 + (l1 + j)) * E0 + l0 + ii];
                    if (rd.det)
                        atomicAdd((unsigned long long *)dst, to_fixed(v * rd.rscale));
                    else
                        atomicAdd(dst, v);
                }
    }
    __syncthreads();
    for (int t = threadIdx.x; t < E0 * E1 * E2; t += BLOCK) {
        const int a0 = t % E0, a1 = (t / E0) % E1, a2 = t / (E0 * E1);
        const int gi = wrap1(o[0] + a0, rd.n[0]), gj = wrap1(o[1] + a1, rd.n[1]);
        const int gk = DIM == 3 ? wrap1(o[2] + a2, rd.n[2]) : 0;
        double *dst = &rho[gi + (long long)rd.n[0] * (gj + (long long)rd.n[1] * gk)];
        if (rd.det) {
            const unsigned long long v = ((const unsigned long long *)s_r)[t];
            if (v) atomicAdd((unsigned long long *)dst, v);
        } else {
            const double v = s_r[t];
            if (v != 0.0) atomicAdd(dst, v);
        }
    }
}

__global__ void fill_kernel(double *p, long long n, double v)
{
    const long long i = (long long)blockIdx.x * BLOCK + threadIdx.x;
    if (i < n) p[i] = v;
}

// deterministic mode: the fixed-point charge density back to FP64, in place
__global__ void rho_from_fixed_kernel(const RunDev *__restrict__ runs, int run, double *p, long long n)
{
    const long long i = (long long)blockIdx.x * BLOCK + threadIdx.x;
    if (i < n) p[i] = (double)((const long long *)p)[i] * runs[run].rscale_inv;
}

// ---------------------------------------------------------------- launchers
#define DISPATCH(D, TT, BODY)                      \
    if (dims == D && split == TT::split) {         \
        BODY(D, TT);                               \
        return hipGetLastError();                  \
    }
#define DISPATCH_ALL(BODY)       \
    DISPATCH(2, F32S, BODY)      \
    DISPATCH(2, FP64, BODY)      \
    DISPATCH(3, F32S, BODY)      \
    DISPATCH(3, FP64, BODY)      \
    return hipErrorInvalidValue;

hipError_t launch_convert(int dims, bool split, const RunDev *runs, int run, int n, const double *x, const double *y,
                          const double *z, const double *ux, const double *uy, const double *uz, const double *w,
                          const uint32_t *id, hipStream_t s)
{
    const int nb = n > 0 ? (n + BLOCK - 1) / BLOCK : 1;
#define CONVERT_BODY(D, TT) convert_kernel<D, TT><<<nb, BLOCK, 0, s>>>(runs, run, n, x, y, z, ux, uy, uz, w, id)
    DISPATCH_ALL(CONVERT_BODY)
}

static int spill_blocks(int n_total)
{
    int b = n_total / (BLOCK * 64);
    return b < 1 ? 1 : (b > 1024 ? 1024 : b);
}

hipError_t launch_relayout(int dims, bool split, RunDev *runs, const int *slots, int n_slots, int count_gx,
                           int move_gx, int commit_gx, int force, hipStream_t s)
{
    if (n_slots <= 0) return hipSuccess;
    relayout_tally_kernel<<<n_slots, PLAN_BLOCK, 0, s>>>(runs, slots, force);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    relayout_count_kernel<<<dim3(count_gx < 1 ? 1 : count_gx, n_slots), BLOCK, 0, s>>>(runs, slots);
    e = hipGetLastError();
    if (e != hipSuccess) return e;
    relayout_plan_kernel<<<n_slots, PLAN_BLOCK, 0, s>>>(runs, slots);
    e = hipGetLastError();
    if (e != hipSuccess) return e;
#define RELAYOUT_BODY(D, TT)                                                                   \
    relayout_move_kernel<D, TT><<<dim3(move_gx, n_slots), BLOCK, 0, s>>>(runs, slots);         \
    e = hipGetLastError();                                                                     \
    if (e != hipSuccess) return e;                                                             \
    relayout_commit_kernel<D, TT><<<dim3(commit_gx, n_slots), BLOCK, 0, s>>>(runs, slots)
    DISPATCH_ALL(RELAYOUT_BODY)
}

hipError_t launch_export(int dims, bool split, const RunDev *runs, int run, int seg_max, int nspill, const int *off,
                         double *x, double *y, double *z, double *ux, double *uy, double *uz, double *w, uint32_t *id,
                         int *patch, hipStream_t s)
{
    const int nb = seg_max + spill_blocks(nspill > 0 ? nspill * 64 : 1);
#define EXPORT_BODY(D, TT) \
    export_kernel<D, TT><<<nb, BLOCK, 0, s>>>(runs, run, nspill, off, x, y, z, ux, uy, uz, w, id, patch)
    DISPATCH_ALL(EXPORT_BODY)
}

hipError_t launch_kinetic(int dims, bool split, const RunDev *runs, int run, int seg_max, int nspill, double *partial,
                          hipStream_t s)
{
#define KIN_BODY(D, TT) kinetic_kernel<D, TT><<<seg_max + 1, BLOCK, 0, s>>>(runs, run, nspill, partial)
    DISPATCH_ALL(KIN_BODY)
}

static hipError_t launch_rho_deposit(int dims, bool split, const RunDev *runs, int run, int seg_max, int nspill,
                                     double *rho, hipStream_t s)
{
#define RHO_BODY(D, TT) rho_kernel<D, TT><<<seg_max + 1, BLOCK, 0, s>>>(runs, run, nspill, rho)
    DISPATCH_ALL(RHO_BODY)
}

hipError_t launch_rho(int dims, bool split, bool det, const RunDev *runs, int run, int seg_max, int nspill, int ncell,
                      double *rho, hipStream_t s)
{
    fill_kernel<<<(ncell + BLOCK - 1) / BLOCK, BLOCK, 0, s>>>(rho, ncell, 0.0);   // also the integer 0
    hipError_t e = hipGetLastError();
    if (e == hipSuccess) e = launch_rho_deposit(dims, split, runs, run, seg_max, nspill, rho, s);
    if (e == hipSuccess && det) {
        rho_from_fixed_kernel<<<(ncell + BLOCK - 1) / BLOCK, BLOCK, 0, s>>>(runs, run, rho, ncell);
        e = hipGetLastError();
    }
    return e;
}

// One thread that waits about `us` microseconds on the device wall clock
// (at most 2^24 polls, whatever the clock does).  Queued ahead of a timed
// sequence, it holds the stream until the host has enqueued the whole
// sequence, so that the events between the kernels measure the kernels and
// not the host's launch latency.
__global__ void gate_kernel(long long ticks)
{
    const long long t0 = wall_clock64();
    for (int i = 0; i < (1 << 24); ++i)
        if (wall_clock64() - t0 >= ticks) break;
}

hipError_t launch_gate(int us, hipStream_t s)
{
    int dev = 0, khz = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e == hipSuccess) e = hipDeviceGetAttribute(&khz, hipDeviceAttributeWallClockRate, dev);
    if (e != hipSuccess) return e;
    if (khz <= 0) khz = 100000;
    gate_kernel<<<1, 1, 0, s>>>((long long)(us > 0 ? us : 0) * khz / 1000);
    return hipGetLastError();
}

}  // namespace sdmd
