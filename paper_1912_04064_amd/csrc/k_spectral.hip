// k_spectral.hip -- the spectral (PSATD) field phase of one step, for runs
// with one periodic region and power-of-two grids.
//
// The field kernel has already summed the patch tiles into the region's J
// (transfer (i) of section 2.2, and the current filter).  The 9 real
// components E, B, J are transformed two at a time: array p holds
// component 2p in its real and component 2p + 1 in its imaginary part
// (5 complex arrays, the last with Jz alone), so every transform carries
// two real fields.  Then:
//   fft x    region E^n, B^n, J (real) -> the 5 packed arrays, transformed
//            along x (one workgroup per batch of x lines, the lines held in
//            LDS: iterative radix-2, bit-reversed load; twiddles from a
//            table of the run);
//   fft y    (3D) along y;
//   line     along the last axis, lines with their mirror lines (all
//            other wavevector components negated) in LDS: forward transform,
//            then for each wavevector k and its mirror -k together: split
//            the packed pairs (the transform A of a real field has
//            A(-k) = conj A(k), so Z = A + iB gives A = (Z(k) + conj
//            Z(-k)) / 2 and B = (Z(k) - conj Z(-k)) / 2i), the exact step
//            (move each component to its staggered position, phase
//            e^{-i k.s}; advance E, B over dt with J held at J^{n+1/2},
//            equations below; move back), repack E, B in pairs, inverse
//            transform of the 3 E/B arrays; lines too long for the LDS
//            take the three steps as separate launches over the whole
//            grid instead;
//   ifft y   (3D) inverse along y;
//   ifft x   inverse along x -> real and imaginary parts / (nx ny nz) =
//            E^{n+1}, B^{n+1} and Bm^{n+1} = B^{n+1} in the other E/B
//            buffer; the post kernel exchanges the ghost layers as for the
//            Yee update.
// The update takes the real part of each inverse transform, that is, the
// Hermitian part (A'(k) + conj A'(-k)) / 2 of each stepped spectrum.  On the
// Yee lattice the step maps conj A(k) at -k to the conjugate of its result
// at k for every wavevector, the Nyquist planes included: each lattice
// wavenumber k~_a enters multiplied by a half-cell shift e^{-+i k_a d_a / 2}
// along the same axis, and where the sampled -pi/d stands for +pi/d both
// change sign together.  So the stepped spectra are Hermitian, the step at k
// gives the one at -k by conjugation, and the inverse transform of the
// repacked Z' = A' + iB' returns A' and B' as its real and imaginary parts.
// With the lattice wavenumber k~_a = 2 sin(k_a d_a / 2) / d_a, w = |k~|,
// kappa = k~ / w, C = cos(w dt), S = sin(w dt):
//   E' = C E + (1 - C) kappa (kappa.E) + i S kappa x B - (S/w) J
//        + kappa (kappa.J) (S/w - dt)
//   B' = C B - i S kappa x E + i ((1 - C)/w) kappa x J
// (w = 0: E' = E - dt J, B' = B): the exact solution of the Yee-lattice
// Maxwell equations over one step, so the discrete Gauss law kept by the
// Esirkepov deposition is kept here too.
#include "launch.h"
#include "sdmd_dev.h"

namespace sdmd {

constexpr int FFT_MAX = SPEC_TW_LEN;   // longest transform line

// twiddle tables e^{-2 pi i k / N}, k < N/2, of N = 2, 4, .., FFT_MAX one
// after the other (the table of N starts at N/2 - 1): shared by every
// transform of the run from HBM (the L1 and L2 caches hold them), so the
// line kernel's LDS holds the data alone
__global__ void spec_twiddle_kernel(double2 *tw)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= FFT_MAX - 1) return;
    int N = 2;
    while (N - 1 <= i) N *= 2;
    const int k = i - (N / 2 - 1);
    double sn, cs;
    sincospi((double)(-2 * k) / (double)N, &sn, &cs);
    tw[i] = make_double2(cs, sn);
}

hipError_t launch_spec_twiddles(double2 *tw, hipStream_t s)
{
    spec_twiddle_kernel<<<(FFT_MAX + BLOCK - 1) / BLOCK, BLOCK, 0, s>>>(tw);
    return hipGetLastError();
}

__device__ __forceinline__ double2 cmul(double2 a, double2 b)
{
    return make_double2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}

// staggering of E (0..2), B (3..5), J (6..8): 1 = half-integer position
__device__ __forceinline__ int stag(int comp, int a)
{
    const int c = comp % 3;
    if (comp < 3 || comp >= 6) return c == a ? 1 : 0;   // E, J: along their own axis
    return c == a ? 0 : 1;                               // B: across the other two
}

// the region component behind grid array c (0..8: E, B, J) at parity par
__device__ __forceinline__ int src_comp(int c, int par)
{
    return c < 3 ? f_E(par) + c : (c < 6 ? f_B(par) + c - 3 : F_J + c - 6);
}

// Radix-2 stages on `lines` lines of N values in LDS (twiddles tw[k] =
// e^{-2 pi i k / N}, k < N/2).  A pass takes the 2^R values that R
// consecutive stages touch into registers (R = 3, then 2 or 1 for the
// last stages), so a transform of 2^m points takes ceil(m / 3)
// barrier-separated passes instead of m.
__device__ __forceinline__ double2 cadd(double2 a, double2 b) { return make_double2(a.x + b.x, a.y + b.y); }
__device__ __forceinline__ double2 csub(double2 a, double2 b) { return make_double2(a.x - b.x, a.y - b.y); }
__device__ __forceinline__ double2 conjd(double2 a) { return make_double2(a.x, -a.y); }

// One pass of R stages whose first (DIT) or last (DIF) stage has half-length
// h = 2^logh, on lines of N = 2^logn values: the values at b + k h, k <
// 2^R, b = block * 2^R h + pos, pos < h.  DIT stage s pairs k and k + 2^s
// (bit s of k clear) with the twiddle of the pair's offset pos + (k mod
// 2^s) h in its block of 2^{s+1} h; DIF runs the stages in the opposite
// order with (u + v, (u - v) conj(w)).  All sizes are powers of two, so the
// index arithmetic is shifts and masks.
template <int R, bool DIF, int NTH = BLOCK>
__device__ __forceinline__ void fft_pass(double2 *buf, const double2 *tw, int logn, int lines, int logh)
{
    constexpr int K = 1 << R;
    const int lg = logn - R;   // log2 of the groups of a line
    const int h = 1 << logh;
    for (int t = threadIdx.x; t < (lines << lg); t += NTH) {
        const int c = t >> lg, q = t & ((1 << lg) - 1), blk = q >> logh, pos = q & (h - 1);
        const int b = (c << logn) + (blk << (R + logh)) + pos;
        double2 v[K];
#pragma unroll
        for (int k = 0; k < K; ++k) v[k] = buf[b + k * h];
#pragma unroll
        for (int ss = 0; ss < R; ++ss) {
            const int s = DIF ? R - 1 - ss : ss;
            const int sh = logn - 1 - logh - s;   // the table step N / 2^{s+1} h
#pragma unroll
            for (int k = 0; k < K; ++k) {
                if (k & (1 << s)) continue;
                const int k2 = k + (1 << s);
                const double2 w = tw[(pos + ((k & ((1 << s) - 1)) << logh)) << sh];
                if constexpr (DIF) {
                    const double2 u = v[k], x = v[k2];
                    v[k] = cadd(u, x);
                    v[k2] = cmul(csub(u, x), conjd(w));
                } else {
                    const double2 x = cmul(v[k2], w);
                    v[k2] = csub(v[k], x);
                    v[k] = cadd(v[k], x);
                }
            }
        }
#pragma unroll
        for (int k = 0; k < K; ++k) buf[b + k * h] = v[k];
    }
    __syncthreads();
}

// decimation in time, bit-reversed input -> natural output
template <int NTH = BLOCK>
__device__ __forceinline__ void fft_dit(double2 *buf, const double2 *tw, int logn, int lines)
{
    int logh = 0;   // half-length of the first stage of the next pass
    for (; logh + 3 <= logn; logh += 3) fft_pass<3, false, NTH>(buf, tw, logn, lines, logh);
    if (logh + 2 <= logn) {
        fft_pass<2, false, NTH>(buf, tw, logn, lines, logh);
        logh += 2;
    }
    if (logh + 1 <= logn) fft_pass<1, false, NTH>(buf, tw, logn, lines, logh);
}

// decimation in frequency with the conjugate twiddles (the inverse of the
// forward table), natural input -> bit-reversed output
template <int NTH = BLOCK>
__device__ __forceinline__ void ifft_dif(double2 *buf, const double2 *tw, int logn, int lines)
{
    int loglen = logn;   // block length of the first stage of the next pass
    for (; loglen >= 3; loglen -= 3) fft_pass<3, true, NTH>(buf, tw, logn, lines, loglen - 3);
    if (loglen >= 2) {
        fft_pass<2, true, NTH>(buf, tw, logn, lines, loglen - 2);
        loglen -= 2;
    }
    if (loglen >= 1) fft_pass<1, true, NTH>(buf, tw, logn, lines, loglen - 1);
}

// 1D transforms of length N = n[axis] along `axis` of components [c0, c0+nc)
// of the packed grid arrays; sign -1 forward, +1 inverse (unscaled).  A workgroup
// transforms NL = max(1, FFT_BATCH / N) lines held in LDS (iterative
// radix-2, bit-reversed load; an inverse transform conjugates its input and
// its output).  Lines along y or z are taken NL adjacent in x, so every row
// of the batch is a contiguous read.  Grid: x = batch of lines, y = packed
// array.
constexpr int FFT_BATCH = 2048;   // complex values per workgroup: 32 KB of LDS
constexpr int SPEC_FFT_THREADS = 2 * BLOCK;   // three workgroups per CU (24 wavefronts; 20 at 256 threads)

__host__ __device__ inline int fft_lines_per_group(int N, int axis, const int n[3])
{
    int nl = N >= FFT_BATCH ? 1 : FFT_BATCH / N;
    const int avail = axis == 0 ? n[1] * n[2] : n[0];
    while (nl > avail) nl >>= 1;
    return nl;
}

// IN_REGION: the lines of packed array c are read from the region's real
// components 2c and 2c + 1 of E^n, B^n, J (the first forward transform);
// OUT_REGION: the real and imaginary parts, divided by the number of cells,
// are written to components 2c and 2c + 1 of the region's E^{n+1}, B^{n+1}
// and Bm (the last inverse transform).
template <bool IN_REGION, bool OUT_REGION>
__global__ __launch_bounds__(SPEC_FFT_THREADS) void spec_fft_kernel(const RunDev *__restrict__ runs, int run, int par, int axis,
                                                         int c0, int sign)
{
    extern __shared__ double2 sm[];
    const RunDev &rd = runs[run];
    if (rd.ctl->remaining[par] == 0) return;
    const int n0 = rd.n[0], n1 = rd.n[1], n2 = rd.n[2];
    const long long ncell = (long long)n0 * n1 * n2;
    const int N = rd.n[axis];
    if (N > FFT_MAX) return;
    const int NL = fft_lines_per_group(N, axis, rd.n);
    const long long groups = ncell / N / NL;
    const long long gidx = blockIdx.x;
    if (gidx >= groups) return;
    double2 *buf = sm;
    const double2 *tw = rd.spec_tw + (N / 2 - 1);
    // the grid sizes are powers of two: index arithmetic in shifts and masks
    const int logn = __builtin_ctz(N), lognl = __builtin_ctz(NL), logn0 = __builtin_ctz(n0),
              logn1 = __builtin_ctz(n1);
    // first line of the group and the offset between its lines
    long long o, stride, lstep;
    if (axis == 0) {
        o = (gidx * NL) << logn0;
        stride = 1;
        lstep = n0;
    } else if (axis == 1) {
        const long long first = gidx * NL;                      // lines enumerate (x, z), x fastest
        o = (first & (n0 - 1)) + ((first >> logn0) << (logn0 + logn1));
        stride = n0;
        lstep = 1;
    } else {
        o = gidx * NL;                                          // lines enumerate (x, y), x fastest
        stride = (long long)n0 * n1;
        lstep = 1;
    }
    const int comp = c0 + blockIdx.y;
    double2 *a = rd.spec + (long long)comp * ncell + o;
    // element j of x line l of the batch -> region element (the region's
    // interior is the grid; the region reads and writes are along x only)
    const long long line0 = gidx * NL;
    auto relem = [&](int l, int j) {
        const long long line = line0 + l;
        return rindex(rd, 0, (int)(line & (n1 - 1)), (int)(line >> logn1)) + j;
    };
    auto place = [&](int e, int &l, int &j) {
        if (axis == 0) {
            j = e & (N - 1);
            l = e >> logn;
        } else {
            l = e & (NL - 1);
            j = e >> lognl;
        }
    };
    const int tid = threadIdx.x;
    const int tot = NL * N;
    for (int e = tid; e < tot; e += SPEC_FFT_THREADS) {
        int l, j;
        place(e, l, j);
        const int r = logn ? (int)(__brev((unsigned)j) >> (32 - logn)) : 0;
        if constexpr (IN_REGION) {
            const long long q = relem(l, j);
            buf[(l << logn) + r] = make_double2(rcomp(rd, 0, src_comp(2 * comp, par))[q],
                                                2 * comp + 1 < 9 ? rcomp(rd, 0, src_comp(2 * comp + 1, par))[q] : 0.0);
        } else {
            const double2 v = a[l * lstep + j * stride];
            buf[(l << logn) + r] = sign > 0 ? conjd(v) : v;
        }
    }
    __syncthreads();
    fft_dit<SPEC_FFT_THREADS>(buf, tw, logn, NL);   // the inverse as conj(forward(conj(x)))
    const double scale = 1.0 / (double)ncell;   // a power of two: exact
    for (int e = tid; e < tot; e += SPEC_FFT_THREADS) {
        int l, j;
        place(e, l, j);
        if constexpr (OUT_REGION) {
            const long long p = relem(l, j);
            const double2 z = conjd(buf[(l << logn) + j]);   // written by an inverse transform only
            const double v[2] = {z.x * scale, z.y * scale};
#pragma unroll
            for (int h = 0; h < 2; ++h) {
                const int c = 2 * comp + h;
                if (c < 3) {
                    rcomp(rd, 0, f_E(1 - par) + c)[p] = v[h];
                } else {
                    rcomp(rd, 0, f_B(1 - par) + c - 3)[p] = v[h];
                    rcomp(rd, 0, F_BM + c - 3)[p] = v[h];
                }
            }
        } else {
            const double2 v = buf[(l << logn) + j];
            a[l * lstep + j * stride] = sign > 0 ? conjd(v) : v;
        }
    }
}

// The exact step of one wavevector: F[0..8] = E, B, J at grid index idx
// (as transformed, at the grid positions); on return F[0..5] hold E^{n+1},
// B^{n+1} at the grid positions.
__device__ __forceinline__ void kspace_step(const RunDev &rd, const int idx[3], double2 F[9])
{
    // fields at their physical (staggered) positions: a component shifted
    // by half a cell along axis a picks up e^{-i k_a d_a / 2}; the same
    // sine gives the lattice wavenumber
    double kt[3] = {0, 0, 0};
    double2 hs[3] = {make_double2(1, 0), make_double2(1, 0), make_double2(1, 0)};
    for (int a = 0; a < rd.dims; ++a) {
        const int m = idx[a] < (rd.n[a] + 1) / 2 ? idx[a] : idx[a] - rd.n[a];   // signed frequency
        const double k = 2.0 * M_PI * (double)m / rd.L[a];
        double sn, cs;
        sincos(0.5 * k * rd.d[a], &sn, &cs);
        kt[a] = 2.0 * sn / rd.d[a];
        hs[a] = make_double2(cs, sn);                           // e^{+i k_a d_a / 2}
    }
    auto shift = [&](int c) {                                   // e^{+i k.s_c}
        double2 z = make_double2(1, 0);
        for (int a = 0; a < rd.dims; ++a)
            if (stag(c, a)) z = cmul(z, hs[a]);
        return z;
    };
#pragma unroll
    for (int c = 0; c < 9; ++c) {
        const double2 z = shift(c);
        F[c] = cmul(F[c], make_double2(z.x, -z.y));
    }
    const double dt = rd.dt;
    const double w = sqrt(kt[0] * kt[0] + kt[1] * kt[1] + kt[2] * kt[2]);
    double2 En[3], Bn[3];
    if (w == 0.0) {
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            En[c] = make_double2(F[c].x - dt * F[6 + c].x, F[c].y - dt * F[6 + c].y);
            Bn[c] = F[3 + c];
        }
    } else {
        const double iw = 1.0 / w;
        const double kap[3] = {kt[0] * iw, kt[1] * iw, kt[2] * iw};
        double S, C;
        sincos(w * dt, &S, &C);
        const double Sw = S * iw, C1w = (1.0 - C) * iw;
        double2 kE = make_double2(0, 0), kJ = make_double2(0, 0);
#pragma unroll
        for (int a = 0; a < 3; ++a) {
            kE.x += kap[a] * F[a].x;
            kE.y += kap[a] * F[a].y;
            kJ.x += kap[a] * F[6 + a].x;
            kJ.y += kap[a] * F[6 + a].y;
        }
        auto crossc = [&](int b0, int c) -> double2 {   // (kappa x F[b0..b0+2])_c
            const int c1 = (c + 1) % 3, c2 = (c + 2) % 3;
            return make_double2(kap[c1] * F[b0 + c2].x - kap[c2] * F[b0 + c1].x,
                                kap[c1] * F[b0 + c2].y - kap[c2] * F[b0 + c1].y);
        };
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            const double2 xB = crossc(3, c), xE = crossc(0, c), xJ = crossc(6, c);
            // i * z = (-z.y, z.x)
            En[c].x = C * F[c].x + (1.0 - C) * kap[c] * kE.x - S * xB.y - Sw * F[6 + c].x + kap[c] * kJ.x * (Sw - dt);
            En[c].y = C * F[c].y + (1.0 - C) * kap[c] * kE.y + S * xB.x - Sw * F[6 + c].y + kap[c] * kJ.y * (Sw - dt);
            Bn[c].x = C * F[3 + c].x + S * xE.y - C1w * xJ.y;
            Bn[c].y = C * F[3 + c].y - S * xE.x + C1w * xJ.x;
        }
    }
    // back to the grid positions
#pragma unroll
    for (int c = 0; c < 6; ++c) F[c] = cmul(c < 3 ? En[c] : Bn[c - 3], shift(c));
}

// The step of wavevector k (grid index idx) and, by conjugation, of its
// mirror -k: pa, pb point at the packed arrays' values at k and -k, ps
// apart.  Splits the 5 pairs into the 9 spectra at k, steps them and writes
// the 3 repacked E/B pairs at k and at -k (at a wavevector that is its own
// mirror, the spectra of the real fields are real).
__device__ __forceinline__ void spec_pair_step(const RunDev &rd, double2 *pa, double2 *pb, long long ps,
                                               const int idx[3])
{
    double2 F[9];
#pragma unroll
    for (int p = 0; p < SPEC_ARRAYS; ++p) {
        const double2 z = pa[p * ps], zm = conjd(pb[p * ps]);
        F[2 * p] = make_double2(0.5 * (z.x + zm.x), 0.5 * (z.y + zm.y));
        if (2 * p + 1 < 9) F[2 * p + 1] = make_double2(0.5 * (z.y - zm.y), -0.5 * (z.x - zm.x));
    }
    kspace_step(rd, idx, F);
    const bool self = pa == pb;
#pragma unroll
    for (int p = 0; p < 3; ++p) {
        double2 u = F[2 * p], v = F[2 * p + 1];
        if (self) u.y = v.y = 0.0;
        pa[p * ps] = make_double2(u.x - v.y, u.y + v.x);                 // u + i v
        if (!self) pb[p * ps] = make_double2(u.x + v.y, v.x - u.y);      // conj u + i conj v
    }
}

// the mirror index (-i mod n) on every axis
__device__ __forceinline__ void mirror_index(const RunDev &rd, const int idx[3], int m[3])
{
#pragma unroll
    for (int a = 0; a < 3; ++a) m[a] = (rd.n[a] - idx[a]) & (rd.n[a] - 1);
}

// exact step of every wavevector of the grid (lines too long for
// spec_line_kernel): one thread per wavevector pair, taken by the one of
// the two with the lower linear index
__global__ __launch_bounds__(BLOCK) void spec_kspace_kernel(const RunDev *__restrict__ runs, int run, int par)
{
    const RunDev &rd = runs[run];
    if (rd.ctl->remaining[par] == 0) return;
    const long long ncell = (long long)rd.n[0] * rd.n[1] * rd.n[2];
    const long long gid = (long long)blockIdx.x * BLOCK + threadIdx.x;
    if (gid >= ncell) return;
    const int l0 = __builtin_ctz(rd.n[0]), l1 = __builtin_ctz(rd.n[1]);   // powers of two
    const int idx[3] = {(int)(gid & (rd.n[0] - 1)), (int)((gid >> l0) & (rd.n[1] - 1)), (int)(gid >> (l0 + l1))};
    int idxm[3];
    mirror_index(rd, idx, idxm);
    const long long gm = idxm[0] + (long long)rd.n[0] * (idxm[1] + (long long)rd.n[1] * idxm[2]);
    if (gm < gid) return;
    spec_pair_step(rd, rd.spec + gid, rd.spec + gm, ncell, idx);
}

// Four lines along the last axis in LDS, all 5 packed arrays, as two
// units of a line and its mirror line (or of two lines that are their own
// mirrors: x and, in 3D, y each 0 or n/2).  Forward transform (bit-reversed
// load, decimation in time), the paired step of each wavevector, inverse
// transform of the 3 E/B arrays (decimation in frequency: natural order in,
// bit-reversed order out, read back bit-reversed on the store).  Most
// workgroups take the lines x, x + 1 of a row and their mirrors -x - 1, -x
// of the mirror row, so every grid row is read as two contiguous pairs of
// values.  The workgroups are dealt to the XCDs in contiguous bands
// (workgroup l runs on XCD l % 8), so those that share the grid's cache
// lines run on one XCD.
constexpr int SPEC_LINE_MAX = 256;   // nodes of the last axis the line kernel takes
constexpr int SPEC_LINE_THREADS = 2 * BLOCK;

// the self-mirror or mirror unit of the columns x = 0, n0/2 in row y (lines
// x + n0 y; 2D: n1 = 1, y = 0): rows 0 and n1/2 pair the lines of the two
// columns that are their own mirrors; row y < n1/2 pairs (0, y) with (0, -y),
// row y > n1/2 pairs (n0/2, y - n1/2) with its mirror
__device__ __forceinline__ bool column_unit(int y, int dims, int n0, int n1, int &a, int &b)
{
    const int hx = n0 / 2, hy = n1 / 2;
    if (dims == 2) {
        a = 0;
        b = hx;
        return true;
    }
    if (y == 0 || y == hy) {
        const int x = y == 0 ? 0 : hx;
        a = x;
        b = x + n0 * hy;
        return true;
    }
    const int x = y < hy ? 0 : hx, yy = y < hy ? y : y - hy;
    a = x + n0 * yy;
    b = x + n0 * (n1 - yy);
    return false;
}

// line group g: lines L[0..3] and, per unit, its two buffer lines and
// whether they are their own mirrors.  With A = n0/4 - 1 groups of adjacent
// pairs per row: group y A + i takes (x, y), (x + 1, y), (-x - 1, -y),
// (-x, -y) for x = 2i + 1 (units: lines 0 and 3, 1 and 2); the last n1
// groups take row y's line (n0/2 - 1, y) with its mirror and the column
// unit of row y (units: lines 0 and 1, 2 and 3).
__device__ __forceinline__ void line_group(int g, int dims, int n0, int n1, int L[4], int ul[2][2], bool self[2])
{
    const int rows = dims == 3 ? n1 : 1, A = n0 / 4 - 1;
    if (g < A * rows) {
        const int y = g / A, x = 2 * (g % A) + 1, my = (n1 - y) & (n1 - 1);
        L[0] = x + n0 * y;
        L[1] = L[0] + 1;
        L[2] = (n0 - x - 1) + n0 * my;
        L[3] = L[2] + 1;
        ul[0][0] = 0; ul[0][1] = 3;
        ul[1][0] = 1; ul[1][1] = 2;
        self[0] = self[1] = false;
        return;
    }
    const int y = g - A * rows, my = (n1 - y) & (n1 - 1);
    L[0] = (n0 / 2 - 1) + n0 * y;
    L[1] = (n0 / 2 + 1) + n0 * my;
    self[0] = false;
    self[1] = column_unit(y, dims, n0, n1, L[2], L[3]);
    ul[0][0] = 0; ul[0][1] = 1;
    ul[1][0] = 2; ul[1][1] = 3;
}

__global__ __launch_bounds__(SPEC_LINE_THREADS, 4) void spec_line_kernel(const RunDev *__restrict__ runs, int run,
                                                                      int par)
{
    constexpr int NTH = SPEC_LINE_THREADS;
    __shared__ double2 buf[4 * SPEC_ARRAYS * SPEC_LINE_MAX];
    const RunDev &rd = runs[run];
    if (rd.ctl->remaining[par] == 0) return;
    const int dims = rd.dims, ax = dims - 1;
    const int n0 = rd.n[0], n1 = rd.n[1];
    const long long ncell = (long long)n0 * n1 * rd.n[2];
    const int N = rd.n[ax];
    const long long nlines = ncell / N, ngroups = nlines / 4;
    const long long band = (ngroups + 7) / 8;
    const long long grp = (long long)(blockIdx.x & 7) * band + (blockIdx.x >> 3);
    if ((blockIdx.x >> 3) >= band || grp >= ngroups) return;
    int L[4], ul[2][2];   // lines of the plane: at most 2048 x 2048
    bool self[2];
    line_group((int)grp, dims, n0, n1, L, ul, self);
    const long long stride = nlines;   // the last axis is the slowest: its lines are every nlines-th element
    // layout: array-major, then line, then node: the 3 E/B arrays first
    const double2 *tw = rd.spec_tw + (N / 2 - 1);   // forward twiddles; the inverse uses their conjugates
    const int logn = __builtin_ctz(N), logn0 = __builtin_ctz(n0);   // powers of two
    const int tid = threadIdx.x;
    for (int e = tid; e < 4 * SPEC_ARRAYS * N; e += NTH) {
        const int l = e & 3, j = (e >> 2) & (N - 1), p = e >> (logn + 2);
        const int r = logn ? (int)(__brev((unsigned)j) >> (32 - logn)) : 0;
        buf[(4 * p + l) * N + r] = rd.spec[p * ncell + L[l] + j * stride];
    }
    __syncthreads();
    fft_dit<NTH>(buf, tw, logn, 4 * SPEC_ARRAYS);   // forward, bit-reversed input
    // the paired steps, unit by unit: (line a, j) with (line b, -j), or
    // within each self-mirror line j with -j for j <= N/2
    const int half = N / 2 + 1;
    const int nt0 = self[0] ? 2 * half : N, ntask = nt0 + (self[1] ? 2 * half : N);
    for (int t = tid; t < ntask; t += NTH) {
        const int u = t < nt0 ? 0 : 1, tu = t - (u ? nt0 : 0);
        const int w = self[u] ? tu / half : 0;   // which line of a self unit
        const int l = ul[u][w], j = self[u] ? tu - w * half : tu;
        const int lm = self[u] ? l : ul[u][1], jm = (N - j) & (N - 1);
        const int ln = L[l];
        const int idx[3] = {ln & (n0 - 1), dims == 3 ? ln >> logn0 : j, dims == 3 ? j : 0};
        spec_pair_step(rd, buf + l * N + j, buf + lm * N + jm, 4 * N, idx);
    }
    __syncthreads();
    ifft_dif<NTH>(buf, tw, logn, 4 * 3);   // inverse of the E/B arrays, bit-reversed output
    for (int e = tid; e < 4 * 3 * N; e += NTH) {
        const int l = e & 3, j = (e >> 2) & (N - 1), p = e >> (logn + 2);
        const int r = logn ? (int)(__brev((unsigned)j) >> (32 - logn)) : 0;
        rd.spec[p * ncell + L[l] + j * stride] = buf[(4 * p + l) * N + r];
    }
}

hipError_t launch_spectral(const RunDev *runs, int run, int dims, const int n[3], int par, hipStream_t s)
{
    const long long ncell = (long long)n[0] * n[1] * n[2];
    const int last = dims - 1;
    auto fft = [&](auto kern, int a, int ncomp, int sign) {
        const int nl = fft_lines_per_group(n[a], a, n);
        const size_t lds = (size_t)nl * n[a] * sizeof(double2);
        kern<<<dim3((unsigned)(ncell / n[a] / nl), ncomp), SPEC_FFT_THREADS, lds, s>>>(runs, run, par, a, 0, sign);
    };
    // forward along x, reading the region's fields; then the middle axis (3D)
    fft(spec_fft_kernel<true, false>, 0, SPEC_ARRAYS, -1);
    for (int a = 1; a < last; ++a) fft(spec_fft_kernel<false, false>, a, SPEC_ARRAYS, -1);
    if (n[last] <= SPEC_LINE_MAX) {
        // four lines per workgroup (n[0], and n[1] in 3D, are powers of two
        // of at least one patch of 4 cells)
        const long long ngroups = ncell / n[last] / 4;
        spec_line_kernel<<<(unsigned)(8 * ((ngroups + 7) / 8)), SPEC_LINE_THREADS, 0, s>>>(runs, run, par);
    } else {
        fft(spec_fft_kernel<false, false>, last, SPEC_ARRAYS, -1);
        spec_kspace_kernel<<<(unsigned)((ncell + BLOCK - 1) / BLOCK), BLOCK, 0, s>>>(runs, run, par);
        fft(spec_fft_kernel<false, false>, last, 3, +1);
    }
    // inverse along the middle axis (3D), then along x into the region
    for (int a = last - 1; a >= 1; --a) fft(spec_fft_kernel<false, false>, a, 3, +1);
    fft(spec_fft_kernel<false, true>, 0, 3, +1);
    return hipGetLastError();
}

}  // namespace sdmd
