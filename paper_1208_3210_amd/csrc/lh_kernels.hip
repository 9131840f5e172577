// lh_kernels.hip -- gfx950 kernels of the Lindhard hot path and their launchers.
//
// Pass schedule of one exec (Sec. 3: Eq. (9) evaluated through the real-space
// functions of Eq. (10) and the convolution theorem):
//   P1  spectral builder (Eq. (5)) fused with the row real-to-complex FFT over kx
//   P2  column FFT over ky                      -> B(r, e_j), Eq. (10)
//   P3  energy-window product: S(r, m) = sum_j conj(B(r, j)) B(r, j + m) over
//       occupied j and unoccupied j + m (the omega integral of Eq. (9)),
//       written in place over the slices it has consumed
//   P4  inverse column FFT over ry
//   P5  inverse row complex-to-real FFT over rx, scale -d / Nk^2, orbital form
//       factor |M(Q)|^2 (Eqs. (2)-(3)) and extended-zone writes
// RPA path (Sec. 4): P5 keeps every lag of the first zone, then the
// Kramers-Kronig and chi / (1 - U chi) epilogues.
#include "lh_fft.h"
#include "lh_internal.h"
#include "lh_regfft.h"

#include <map>
#include <mutex>

namespace lh {

constexpr double kPi = 3.14159265358979323846;
constexpr int kThreads = 256;

// ---------------------------------------------------------------- setup
__global__ void __launch_bounds__(kThreads) k_band_tb(double *__restrict__ eps, int nkx, int logNx, int nky,
                                                     double t, double tp, double tpp, int kz)
{
    const long nk = (long)nkx * nky;
    const long k = (long)blockIdx.x * kThreads + threadIdx.x;
    if (k >= nk) return;
    // folded indices make eps(kx, ky) = eps(-kx, ky) = eps(kx, -ky) bit for bit
    // (any grid size: the row index by division)
    const int kx0 = (int)(k % nkx), ky0 = (int)(k / nkx);
    const int ix = min(kx0, nkx - kx0);
    const int iy = min(ky0, nky - ky0);
    // k_zones kz: the grid spans kz zones, k = 2 pi kz (ix / nkx, iy / nky)
    const double cx = cospi(2.0 * kz * ix / nkx), cy = cospi(2.0 * kz * iy / nky);
    const double c2x = cospi(4.0 * kz * ix / nkx), c2y = cospi(4.0 * kz * iy / nky);
    eps[k] = -2.0 * t * (cx + cy) - 4.0 * tp * cx * cy - 2.0 * tpp * (c2x + c2y);
}

// Partial sums of the occupation n(mu) and of dn/dmu over a fixed grid-stride
// partition (deterministic for a fixed grid).
__global__ void __launch_bounds__(kThreads) k_occ_partial(const double *__restrict__ eps, long nk, double mu,
                                                         double gamma, double *__restrict__ part)
{
    __shared__ double s0[kThreads], s1[kThreads];
    double a = 0.0, b = 0.0;
    const double ig = 1.0 / kPi;
    for (long k = (long)blockIdx.x * kThreads + threadIdx.x; k < nk; k += (long)gridDim.x * kThreads) {
        const double x = mu - eps[k];
        a += 0.5 + atan(x / gamma) * ig;
        b += (gamma * ig) / (x * x + gamma * gamma);
    }
    s0[threadIdx.x] = a;
    s1[threadIdx.x] = b;
    __syncthreads();
    for (int h = kThreads / 2; h > 0; h >>= 1) {
        if ((int)threadIdx.x < h) {
            s0[threadIdx.x] += s0[threadIdx.x + h];
            s1[threadIdx.x] += s1[threadIdx.x + h];
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        part[blockIdx.x] = s0[0];
        part[gridDim.x + blockIdx.x] = s1[0];
    }
}

__global__ void __launch_bounds__(kThreads) k_occ_final(const double *__restrict__ part, int nb, long nk,
                                                       double *__restrict__ out2)
{
    __shared__ double s0[kThreads], s1[kThreads];
    double a = 0.0, b = 0.0;
    for (int i = threadIdx.x; i < nb; i += kThreads) {
        a += part[i];
        b += part[nb + i];
    }
    s0[threadIdx.x] = a;
    s1[threadIdx.x] = b;
    __syncthreads();
    for (int h = kThreads / 2; h > 0; h >>= 1) {
        if ((int)threadIdx.x < h) {
            s0[threadIdx.x] += s0[threadIdx.x + h];
            s1[threadIdx.x] += s1[threadIdx.x + h];
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        out2[0] = 2.0 * s0[0] / (double)nk;
        out2[1] = 2.0 * s1[0] / (double)nk;
    }
}

__global__ void __launch_bounds__(kThreads) k_xi_shift(double *__restrict__ eps, long nk, double mu)
{
    const long k = (long)blockIdx.x * kThreads + threadIdx.x;
    if (k < nk) eps[k] = eps[k] - mu;
}

// tw[s] = exp(-2 pi i s / n), evaluated in FP64 and rounded once to T.
template <typename T>
__global__ void __launch_bounds__(kThreads) k_twiddle(cx<T> *__restrict__ tw, int n)
{
    const int s = blockIdx.x * kThreads + threadIdx.x;
    if (s >= n) return;
    double sv, cv;
    sincospi(-2.0 * (double)s / (double)n, &sv, &cv);
    tw[s] = mk<T>((T)cv, (T)sv);
}

// Per extended column (or row) X: (exp(-s Q^2), Q^2), Q = 2 pi h with
// h = kz (X - zones n/2) / n reciprocal-lattice units (a momentum grid of n
// points spanning kz zones has a step of kz / n).
__global__ void __launch_bounds__(kThreads) k_fftab(double2 *__restrict__ tab, int n, int zones, double s, int kz)
{
    const int X = blockIdx.x * kThreads + threadIdx.x;
    if (X >= n * zones) return;
    const double h = (double)kz * (double)(X - (zones * n) / 2) / (double)n;
    const double Q = 2.0 * kPi * h;
    const double Q2 = Q * Q;
    tab[X] = make_double2(exp(-s * Q2), Q2);
}

// Kramers-Kronig weights of the alternate-point rule (Sec. 4):
// w(i, j) = (2/pi) 2j / (j^2 - i^2) for j - i odd, 1 <= j < neps, else 0.
__device__ __forceinline__ double kk_weight(long i, int j)
{
    if (j < 1 || !(((long)j - i) & 1)) return 0.0;
    const double di = (double)i, dj = (double)j;
    return (2.0 / kPi) * 2.0 * dj / (dj * dj - di * di);
}
// Energy of position jp (0 <= jp < 16 nch) in the sequence a tile of lags of
// parity par sums over: in each chunk of 32 energies the 16 of the other parity.
__device__ __forceinline__ int kk_energy(int jp, int par) { return 32 * (jp >> 4) + (1 - par) + 2 * (jp & 15); }
// Weights per tile t of 16 lags (rows (lag, slot), lag < 0: padding), per
// energy position jp and per row r: w[(t * 16 nch + jp) * 16 + r].
__global__ void __launch_bounds__(kThreads) k_kkw(double *__restrict__ w, const int2 *__restrict__ rows, int ntiles,
                                                 int nch, int neps)
{
    const long n = (long)ntiles * 16 * nch * 16;
    const long idx = (long)blockIdx.x * kThreads + threadIdx.x;
    if (idx >= n) return;
    const int r = (int)(idx & 15), t = (int)(idx / (16L * nch * 16));
    const int jp = (int)((idx >> 4) % (16L * nch));
    const int lag = rows[t * 16 + r].x, par = rows[t * 16].x & 1;
    const int j = kk_energy(jp, par);
    w[idx] = (lag >= 0 && j < neps) ? kk_weight(lag, j) : 0.0;
}

// 16 bytes of consecutive elements (one vector load or store per lane).
template <typename T>
struct Vec16 {
    T v[16 / sizeof(T)];
};
typedef unsigned lh_u4 __attribute__((ext_vector_type(4)));

// Blocks are dispatched round-robin over the 8 XCDs (each with its own L2).
// Map launch index b to a logical tile so that consecutive logical tiles run
// on the same XCD: tiles sharing cache lines then meet in the same L2.
__device__ __forceinline__ unsigned xcd_tile(unsigned b, unsigned nblocks)
{
    const unsigned per = nblocks >> 3;          // full rounds of 8
    if (b >= (per << 3)) return b;              // ragged tail keeps its index
    return (b & 7) * per + (b >> 3);
}

// Lorentzian of Eq. (5) from the (already rounded) argument d = e_j - xi_k:
// (gamma/pi) / (d^2 + gamma^2).  FP32 uses the hardware reciprocal (1 ulp).
__device__ __forceinline__ float lorentz(float d, float gp, float g2)
{
    return gp * __builtin_amdgcn_rcpf(d * d + g2);
}
__device__ __forceinline__ double lorentz(double d, double gp, double g2) { return gp / (d * d + g2); }

// |M(Q)|^2 = F(Q)^2 at extended (X, Y), Eq. (3) for the Gaussian d orbital.
__device__ __forceinline__ double form_factor_sq(const double2 fx, const double2 fy, double s)
{
    const double q2 = fx.y + fy.y;
    const double dq = fx.y - fy.y;
    const double F = fx.x * fy.x * (1.0 - 2.0 * s * q2 + s * s * dq * dq);
    return F * F;
}

// FP32: an FFT twiddle table of n values copied into LDS at dst (stored with
// tw_swz), so that the transform passes read it there rather than waiting on
// the cache for every pass; returns the table to use.  FP64 keeps the global table (it would
// double the LDS of the blocks that use it).  Every thread of the block calls
// it (it ends with a barrier when it copies).
template <typename T>
constexpr bool kTwLds = sizeof(T) == 4;  // the kernels that copy their twiddles into LDS (FP32)
template <typename T>
__device__ __forceinline__ const cx<T> *tw_to_lds(const cx<T> *tw, cx<T> *dst, int n, int tid, int nthr)
{
    if constexpr (kTwLds<T>) {
        for (int i = tid; i < n; i += nthr) dst[tw_swz(i)] = tw[i];  // the layout RegFFT<..., true> reads
        __syncthreads();
        return dst;
    } else {
        return tw;
    }
}
// LDS bytes of such a table
template <typename T>
constexpr size_t tw_lds_bytes(int n)
{
    return sizeof(T) == 4 ? (size_t)n * sizeof(cx<T>) : 0;
}

// Row passes (the even path's builder and both paths' last row passes)
// in FP32 use the padded-layout engine (padding period 32) when a line spans
// whole waves (at least 64 threads); FP64 keeps its twiddles in global memory
// and the swizzled engine.
constexpr int kRowPB = 5;
template <typename T, int LOGN, int LOGE>
constexpr bool row_padded()
{
    return sizeof(T) == 4 && LOGN - LOGE >= 6 && LOGN <= 12;
}
// LDS elements between the lines of a row pass
template <typename T, int LOGN, int LOGE>
constexpr int row_line_stride()
{
    if constexpr (row_padded<T, LOGN, LOGE>())
        return RegFFTP<T, LOGN, false, LOGE, kRowPB>::LINE;
    else
        return 1 << LOGN;
}
// LDS slot of element x of a row-pass line
template <typename T, int LOGN, int LOGE>
__device__ __forceinline__ int row_slot(int x)
{
    if constexpr (row_padded<T, LOGN, LOGE>())
        return RegFFTP<T, LOGN, false, LOGE, kRowPB>::pad(x);
    else
        return x;
}
// LDS bytes of a row pass with R lines: the lines, then (FP32) the twiddles
template <typename T, int LOGN, int LOGE>
size_t row_lds_bytes(int R)
{
    if constexpr (row_padded<T, LOGN, LOGE>())
        return (size_t)(R * row_line_stride<T, LOGN, LOGE>() + RegFFTP<T, LOGN, false, LOGE, kRowPB>::TWN) *
               sizeof(cx<T>);
    else
        return (size_t)(R + (sizeof(T) == 4 ? 1 : 0)) * (1 << LOGN) * sizeof(cx<T>);
}

// ---------------------------------------------------------------- P1
// One block: R rows (ky) of the spectral function for jc consecutive energy
// slices; G = L/E threads per row.  Row kx of length nkx is packed as
// z[n] = A(2n) + i A(2n+1) and transformed with the register FFT of length
// L = nkx/2, then split into X[k], k = 0..L (real-to-complex) and written to
// the column-tiled spectral array.  e_j - xi_k is formed in FP64; the
// Lorentzian and the transform run in T.
template <typename T, int LOGL, bool W>
__global__ void __launch_bounds__(kThreads) k_p1(const double *__restrict__ xi, Geo g, double emin, double deps,
                                                double gamma, const cx<T> *__restrict__ twx,
                                                cx<T> *__restrict__ spec, const T *__restrict__ rho, int acc)
{
    using F = RegFFT<T, LOGL, false, ilog2_c(kP1Elems), kTwLds<T>>;
    constexpr int L = F::N, E = F::E, G = F::G;
    extern __shared__ __align__(16) unsigned char smem_raw[];
    cx<T> *lds = reinterpret_cast<cx<T> *>(smem_raw);
    const int R = g.p1_R, logR = g.p1_logR;
    const int tid = threadIdx.x;
    const int row = tid / G, gg = tid % G;
    const int ky0 = blockIdx.x * R;
    const int jbeg = g.jA + blockIdx.y * g.p1_jc;
    const int jend = min(g.jB, jbeg + g.p1_jc);
    cx<T> *buf = lds + row * L;
    const cx<T> *tw = tw_to_lds<T>(twx, lds + R * L, 2 * L, tid, R * G);

    double xa[E], xb[E];
    T ra[W ? E : 1], rb[W ? E : 1];  // momentum-density weights (W)
    {
        const double2 *xr = reinterpret_cast<const double2 *>(xi + (size_t)(ky0 + row) * g.nkx);
#pragma unroll
        for (int s = 0; s < E; ++s) {
            const double2 x2 = xr[gg + s * G];
            xa[s] = x2.x;
            xb[s] = x2.y;
            if constexpr (W) {
                ra[s] = rho[(size_t)(ky0 + row) * g.nkx + 2 * (gg + s * G)];
                rb[s] = rho[(size_t)(ky0 + row) * g.nkx + 2 * (gg + s * G) + 1];
            }
        }
    }
    const T gp = (T)(gamma / kPi), g2 = (T)(gamma * gamma);
    const int C = g.C, logC = g.logC;
    const int nout = g.NT * (R << logC);

    for (int j = jbeg; j < jend; ++j) {
        const double ej = emin + (j + 0.5) * deps;
        cx<T> v[E];
#pragma unroll
        for (int s = 0; s < E; ++s) {
            const T d0 = (T)(ej - xa[s]), d1 = (T)(ej - xb[s]);
            if constexpr (W)
                v[s] = mk<T>(lorentz(d0, gp, g2) * ra[s], lorentz(d1, gp, g2) * rb[s]);
            else
                v[s] = mk<T>(lorentz(d0, gp, g2), lorentz(d1, gp, g2));
        }
        F::run(v, buf, tw, 1, gg, lds_xor_gfast<L, G>(row));
#pragma unroll
        for (int s = 0; s < E; ++s) buf[swz(gg + s * G)] = v[s];
        __syncthreads();
        cx<T> *dst = spec + (size_t)(j - g.jA) * g.slice_elems;
        for (int it = tid; it < nout; it += R * G) {
            const int c = it & (C - 1);
            const int r = (it >> logC) & (R - 1);
            const int tile = it >> (logC + logR);
            const int k = tile * C + c;
            cx<T> X = mk<T>((T)0, (T)0);
            if (k <= L) {
                const cx<T> Zk = lds[r * L + swz(k & (L - 1))];
                const cx<T> ZL = cconj(lds[r * L + swz((L - k) & (L - 1))]);
                const cx<T> Ev = cscale(cadd(Zk, ZL), (T)0.5);
                const cx<T> D = cscale(csub(Zk, ZL), (T)0.5);
                const cx<T> w = tw[kTwLds<T> ? tw_swz(k) : k];
                X = cadd(Ev, cmul(mk<T>(w.y, -w.x), D));
            }
            cx<T> *o = dst + ((size_t)tile * g.nky + ky0 + r) * C + c;
            *o = acc ? cadd(*o, X) : X;  // acc: add this band to the earlier ones
        }
        __syncthreads();
    }
}

// ---------------------------------------------------------------- P2 / P4
// Column pass: each line is one column of a tile (nky values, C columns per
// tile row).  Threads are ordered line-fastest so that one load instruction of
// a wave covers whole 32-byte tile rows; data go straight from HBM into the
// register FFT and back.  TPB tiles per block keep small transforms at 256
// threads.  Transformed in place.
template <typename T, int LOGN, bool INV>
__global__ void __launch_bounds__(col_threads(LOGN)) k_col(cx<T> *__restrict__ spec, Geo g,
                                                          const cx<T> *__restrict__ twy)
{
    using F = RegFFT<T, LOGN, INV, 4, kTwLds<T>>;
    constexpr int N = F::N, E = F::E, G = F::G;
    constexpr int C = sizeof(T) == 4 ? 4 : 2;
    constexpr int TPB = (G * C >= 256) ? 1 : 256 / (G * C);
    constexpr int NL = TPB * C;
    extern __shared__ __align__(16) unsigned char smem_raw[];
    cx<T> *lds = reinterpret_cast<cx<T> *>(smem_raw);
    const int tid = threadIdx.x;
    const int line = tid % NL, gg = tid / NL;
    const int tb = line / C, c = line % C;
    const int tile = blockIdx.x * TPB + tb;  // tiles of every kz plane (three dimensions)
    const bool active = tile < g.NT * g.nkz;
    const cx<T> *tw = tw_to_lds<T>(twy, lds + NL * N, N, tid, NL * G);
    cx<T> *base = spec + (size_t)blockIdx.y * g.slice_elems + (size_t)(active ? tile : 0) * N * C;
    cx<T> v[E];
#pragma unroll
    for (int s = 0; s < E; ++s) v[s] = active ? base[(gg + s * G) * C + c] : mk<T>((T)0, (T)0);
    F::run(v, lds + line * N, tw, 0, gg, lds_xor_interleaved<T, N>(line, NL));
    if (active) {
#pragma unroll
        for (int s = 0; s < E; ++s) base[(gg + s * G) * C + c] = v[s];
    }
}

// Third-axis pass (three-dimensional grids): each line runs along kz through
// the planes of one slice (stride plane_elems); the lines are the (tile, ky,
// c) positions of a plane, C consecutive c per group so that the loads of a
// wave cover whole 32-byte tile rows.  Transformed in place.
template <typename T, int LOGN, bool INV>
__global__ void __launch_bounds__(512) k_zcol(cx<T> *__restrict__ spec, Geo g, const cx<T> *__restrict__ twz)
{
    using F = RegFFT<T, LOGN, INV, 4, kTwLds<T>>;
    constexpr int N = F::N, E = F::E, G = F::G;
    constexpr int C = sizeof(T) == 4 ? 4 : 2;
    constexpr int TPB = (G * C >= 256) ? 1 : 256 / (G * C);
    constexpr int NL = TPB * C;
    extern __shared__ __align__(16) unsigned char smem_raw[];
    cx<T> *lds = reinterpret_cast<cx<T> *>(smem_raw);
    const int tid = threadIdx.x;
    const int line = tid % NL, gg = tid / NL;
    const int grp = blockIdx.x * TPB + line / C, c = line % C;
    const bool active = grp < g.NT * g.nky;
    const cx<T> *tw = tw_to_lds<T>(twz, lds + NL * N, N, tid, NL * G);
    cx<T> *base = spec + (size_t)blockIdx.y * g.slice_elems + (size_t)(active ? grp : 0) * C + c;
    cx<T> v[E];
#pragma unroll
    for (int s = 0; s < E; ++s) v[s] = active ? base[(size_t)(gg + s * G) * g.plane_elems] : mk<T>((T)0, (T)0);
    F::run(v, lds + line * N, tw, 0, gg, lds_xor_interleaved<T, N>(line, NL));
    if (active) {
#pragma unroll
        for (int s = 0; s < E; ++s) base[(size_t)(gg + s * G) * g.plane_elems] = v[s];
    }
}

// ---------------------------------------------------------------- P3
template <typename T>
__device__ __forceinline__ void two_sum(T &s, T &e, T b)
{
    const T a = s;
    const T t = a + b;
    const T bb = t - a;
    e += (a - (t - bb)) + (b - bb);
    s = t;
}

// One block: TR = RY * C real-space points (RY rows of one column tile) with
// every slice they need staged in LDS as buf[slice][point].  Each wave takes
// blocks of 8 consecutive lags; its 64 lanes are TR points x SU = 64/TR
// sub-ranges of the occupied-energy sum, so all lanes of a wave run the same
// trip count.  Lane partial sums are combined with shuffles.
// COMP: blocks of 8 products are summed in T and folded into a two-sum
// (hi, lo) accumulator; the SU partials are merged with two-sum as well.
template <typename T, bool COMP>
__global__ void __launch_bounds__(kThreads) k_p3(cx<T> *__restrict__ spec, Geo g)
{
    extern __shared__ __align__(16) unsigned char smem_raw[];
    cx<T> *buf = reinterpret_cast<cx<T> *>(smem_raw);
    const int TR = g.p3_TR, logTR = g.p3_logTR;
    const int tid = threadIdx.x;
    const size_t off = ((size_t)blockIdx.x * g.nky + (size_t)blockIdx.y * g.p3_RY) << g.logC;
    const int ne = g.nS;
    for (int it0 = tid; it0 < (ne << logTR); it0 += 8 * kThreads) {
        cx<T> v[8];
#pragma unroll
        for (int k = 0; k < 8; ++k) {
            const int it = it0 + k * kThreads;
            const int s = it >> logTR, rp = it & (TR - 1);
            v[k] = spec[it < (ne << logTR) ? (size_t)s * g.slice_elems + off + rp : 0];
        }
#pragma unroll
        for (int k = 0; k < 8; ++k)
            if (it0 + k * kThreads < (ne << logTR)) buf[it0 + k * kThreads] = v[k];
    }
    __syncthreads();

    const int j0 = g.j0 - g.jA;
    const int lane = tid & 63, wave = tid >> 6;
    const int rp = lane & (TR - 1);
    const int su = lane >> logTR;
    const int SU = 64 >> logTR;
    const int nB = (g.nL + 7) >> 3;
    const cx<T> zero = mk<T>((T)0, (T)0);

    auto ldH = [&](int jj) -> cx<T> {
        const int jc = jj < ne ? jj : ne - 1;
        const cx<T> v = buf[(jc << logTR) + rp];
        return (jj >= j0 && jj < ne) ? v : zero;
    };

    for (int b = wave; b < nB; b += kThreads / 64) {
        const int mf = g.m_lo + 8 * b;
        const int jlo = max(0, j0 - (mf + 7));
        const int jhi = min(j0, ne - mf);
        cx<T> hi[8], lo[8];
#pragma unroll
        for (int i = 0; i < 8; ++i) {
            hi[i] = zero;
            lo[i] = zero;
        }
        if (jlo < jhi) {
            const int Lj = jhi - jlo;
            const int cl = (Lj + SU - 1) / SU;
            const int js = jlo + su * cl;
            const int je = min(jhi, js + cl);
            const int nit = (cl + 7) & ~7;
            const int hb = js + mf;
            cx<T> w[8];
#pragma unroll
            for (int s = 0; s < 8; ++s) w[s] = ldH(hb + s);
            for (int u0 = 0; u0 < nit; u0 += 8) {
                cx<T> tmp[8];
#pragma unroll
                for (int i = 0; i < 8; ++i) tmp[i] = zero;
#pragma unroll
                for (int u = 0; u < 8; ++u) {
                    const int j = js + u0 + u;
                    const int jc = j < ne ? j : ne - 1;
                    cx<T> p = buf[(jc << logTR) + rp];
                    if (j >= je) p = zero;
#pragma unroll
                    for (int i = 0; i < 8; ++i) {
                        const cx<T> h = w[(u + i) & 7];
                        // conj(p) * h
                        tmp[i].x += p.x * h.x + p.y * h.y;
                        tmp[i].y += p.x * h.y - p.y * h.x;
                    }
                    w[u] = ldH(hb + u0 + u + 8);
                }
#pragma unroll
                for (int i = 0; i < 8; ++i) {
                    if (COMP) {
                        two_sum(hi[i].x, lo[i].x, tmp[i].x);
                        two_sum(hi[i].y, lo[i].y, tmp[i].y);
                    } else {
                        hi[i].x += tmp[i].x;
                        hi[i].y += tmp[i].y;
                    }
                }
            }
        }
        for (int o = TR; o < 64; o <<= 1) {
#pragma unroll
            for (int i = 0; i < 8; ++i) {
                const T ohx = __shfl_xor(hi[i].x, o, 64), ohy = __shfl_xor(hi[i].y, o, 64);
                if (COMP) {
                    const T olx = __shfl_xor(lo[i].x, o, 64), oly = __shfl_xor(lo[i].y, o, 64);
                    two_sum(hi[i].x, lo[i].x, ohx);
                    two_sum(hi[i].y, lo[i].y, ohy);
                    lo[i].x += olx;
                    lo[i].y += oly;
                } else {
                    hi[i].x += ohx;
                    hi[i].y += ohy;
                }
            }
        }
        if (su == 0) {
#pragma unroll
            for (int i = 0; i < 8; ++i) {
                const int m = mf + i;
                if (m <= g.m_hi)
                    spec[(size_t)(m - g.m_lo) * g.slice_elems + off + rp] =
                        COMP ? mk<T>(hi[i].x + lo[i].x, hi[i].y + lo[i].y) : hi[i];
            }
        }
    }
}

// Energy-window product by FFT along the energy axis.  For one real-space
// point let P_j = B(r, j) for occupied j and H_j = B(r, j) for unoccupied j
// (zero elsewhere).  Because every occupied index lies below every unoccupied
// one, the circular correlation of length N >= (number of slices) equals the
// linear one for 0 <= m < N, so
//   S(r, m) = sum_j conj(P_j) H_{j+m} = IFFT_N( conj(FFT_N P) * FFT_N H )(m) / N.
// One block: TR real-space points (RY rows of one column tile), G threads per
// point; the slices are staged through LDS, which is then reused as the FFT
// line buffers.  Written in place over the slices, as the direct form.
template <typename T, int LOGN>
__global__ void __launch_bounds__(512) k_p3f(cx<T> *__restrict__ spec, Geo g, const cx<T> *__restrict__ twe)
{
    using FF = RegFFT<T, LOGN, false, 4, kTwLds<T>>;
    using FI = RegFFT<T, LOGN, true, 4, kTwLds<T>>;
    constexpr int N = FF::N, E = FF::E, G = FF::G;
    extern __shared__ __align__(16) unsigned char smem_raw[];
    cx<T> *lds = reinterpret_cast<cx<T> *>(smem_raw);  // [N][TR], then [TR][N]
    const int TR = g.p3f_TR, logTR = g.p3f_logTR;
    const int tid = threadIdx.x;
    const int rp = tid & (TR - 1), gg = tid >> logTR;
    const size_t off = ((size_t)blockIdx.x * g.nky + (size_t)blockIdx.y * (TR >> g.logC)) << g.logC;
    const int ne = g.nS;
    const int j0 = g.j0 - g.jA;
    const int nthr = TR * G;
    const cx<T> *tw = tw_to_lds<T>(twe, lds + TR * N, N, tid, nthr);
    for (int it0 = tid; it0 < (ne << logTR); it0 += 8 * nthr) {
        cx<T> v[8];
#pragma unroll
        for (int k = 0; k < 8; ++k) {
            const int it = it0 + k * nthr;
            const int sl = it >> logTR, p = it & (TR - 1);
            v[k] = spec[it < (ne << logTR) ? (size_t)sl * g.slice_elems + off + p : 0];
        }
#pragma unroll
        for (int k = 0; k < 8; ++k)
            if (it0 + k * nthr < (ne << logTR)) lds[it0 + k * nthr] = v[k];
    }
    __syncthreads();
    const cx<T> zero = mk<T>((T)0, (T)0);
    cx<T> vp[E], vh[E];
#pragma unroll
    for (int s = 0; s < E; ++s) {
        const int j = gg + s * G;
        const cx<T> b = j < ne ? lds[(j << logTR) + rp] : zero;
        vp[s] = j < j0 ? b : zero;
        vh[s] = j >= j0 ? b : zero;
    }
    __syncthreads();
    cx<T> *buf = lds + rp * N;
    const int lxe = lds_xor_interleaved<T, N>(rp, TR);
    FF::run(vp, buf, tw, 0, gg, lxe);
    FF::run(vh, buf, tw, 0, gg, lxe);
#pragma unroll
    for (int s = 0; s < E; ++s) {
        const cx<T> a = vp[s], b = vh[s];
        vh[s] = mk<T>(a.x * b.x + a.y * b.y, a.x * b.y - a.y * b.x);  // conj(a) b
    }
    FI::run(vh, buf, tw, 0, gg, lxe);
    const T inv = (T)(1.0 / N);
#pragma unroll
    for (int s = 0; s < E; ++s) {
        const int m = gg + s * G;
        if (m >= g.m_lo && m <= g.m_hi)
            spec[(size_t)(m - g.m_lo) * g.slice_elems + off + rp] = cscale(vh[s], inv);
    }
}

// ---------------------------------------------------------------- P5
// One block: R rows (qy) of one output plane, G threads per row.
// Complex-to-real inverse over rx from the half spectrum X[0..L]:
// Z'[k] = (X[k] + X*[L-k]) + i e^{+2 pi i k/nkx} (X[k] - X*[L-k]); the inverse
// register FFT of length L gives x[2n] + i x[2n+1] (no 1/N), written as pairs.
// MODE 0: plane = requested omega; writes the extended, form-factor weighted
//         map out[plane][Y][X] (zeros for an empty window).
// MODE 1: plane = window slot; writes the first-zone map out[m][qy][qx].
template <typename T, int LOGL, int MODE>
__global__ void __launch_bounds__(kThreads) k_p5(const cx<T> *__restrict__ spec, Geo g,
                                                const cx<T> *__restrict__ twx, const PlaneSrc *__restrict__ psrc,
                                                double scale, int zx, int zy, int ff, double ffs,
                                                const double2 *__restrict__ ffx, const double2 *__restrict__ ffy,
                                                T *__restrict__ out, int out_nx, int out_ny,
                                                const T *__restrict__ m2, int acc)
{
    using F = RegFFT<T, LOGL, true, 4, kTwLds<T>>;
    using FP = RegFFTP<T, LOGL, true, 4, kRowPB>;
    constexpr bool PADDED = row_padded<T, LOGL, 4>();
    constexpr int L = F::N, E = F::E, G = F::G;
    // line stride: L + 1 staged values, then the transform's line (padded: LINE > L + 1)
    constexpr int LS = PADDED ? row_line_stride<T, LOGL, 4>() : L + 1;
    extern __shared__ __align__(16) unsigned char smem_raw[];
    cx<T> *lds = reinterpret_cast<cx<T> *>(smem_raw);  // [R][LS]
    const int R = g.p5_R, logR = g.p5_logR;
    const int nthr = R * G;
    const int tid = threadIdx.x;
    const int row = tid / G, gg = tid % G;
    const int plane = blockIdx.y;
    const int qy0 = blockIdx.x * R;
    const PlaneSrc ps = MODE == 0 ? psrc[plane] : PlaneSrc{plane, -1, 1.0, 0.0};
    const int slot = ps.a;
    const int nkx = g.nkx, nky = g.nky;

    if (MODE == 0 && slot < 0) {
        if (acc) return;  // adds nothing
        for (int rz = 0; rz < R * zy; ++rz) {
            const int r = rz % R, zi = rz / R;
            const int Y = zi * nky + ((qy0 + r + zy * nky / 2) & (nky - 1));
            T *orow = out + ((size_t)plane * out_ny + Y) * out_nx;
            for (int X = tid; X < out_nx; X += nthr) orow[X] = (T)0;
        }
        return;
    }
    // the transform's twiddles (tw) and the split's exp(-2 pi i k / nkx), k < L
    // (tws): with the padded engine the per-pass tables, then the split table
    // in natural order (made visible by the barrier after the staging loop);
    // otherwise one swizzled table of nkx values serving both
    const cx<T> *tw, *tws;
    if constexpr (PADDED) {
        cx<T> *twp = lds + R * LS, *twsl = twp + FP::TWN;
        FP::fill_twiddles(twp, twx, tid, nthr, 1);
        for (int i = tid; i < L; i += nthr) twsl[i] = twx[i];
        tw = twp;
        tws = twsl;
    } else {
        tw = tw_to_lds<T>(twx, lds + R * (L + 1), 2 * L, tid, nthr);
        tws = tw;
    }

    const int C = g.C, logC = g.logC;
    const cx<T> *src = spec + (size_t)slot * g.slice_elems;
    // an omega between two lags: wa S[a] + wb S[b] (wb = 0 reads S[a] twice)
    const bool blend = ps.b >= 0 || ps.wa != 1.0;
    const cx<T> *src2 = spec + (size_t)(ps.b >= 0 ? ps.b : slot) * g.slice_elems;
    const T wa = (T)ps.wa, wb = (T)ps.wb;
    const int nin = g.NT * (R << logC);
    for (int it0 = tid; it0 < nin; it0 += 8 * nthr) {
        cx<T> v[8];
#pragma unroll
        for (int k = 0; k < 8; ++k) {
            const int it = it0 + k * nthr;
            const int c = it & (C - 1);
            const int r = (it >> logC) & (R - 1);
            const int tile = it >> (logC + logR);
            const size_t o = it < nin ? ((size_t)tile * nky + qy0 + r) * C + c : 0;
            v[k] = src[o];
            if (blend) {
                const cx<T> y = src2[o];
                v[k] = mk<T>(wa * v[k].x + wb * y.x, wa * v[k].y + wb * y.y);
            }
        }
#pragma unroll
        for (int k = 0; k < 8; ++k) {
            const int it = it0 + k * nthr;
            const int c = it & (C - 1);
            const int r = (it >> logC) & (R - 1);
            const int kk = (it >> (logC + logR)) * C + c;
            if (it < nin && kk <= L) lds[r * LS + kk] = v[k];
        }
    }
    __syncthreads();
    cx<T> *xb = lds + row * LS;
    cx<T> v[E];
#pragma unroll
    for (int s = 0; s < E; ++s) {
        const int k = gg + s * G;
        const cx<T> Xk = xb[k];
        const cx<T> XL = cconj(xb[L - k]);
        const cx<T> A = cadd(Xk, XL);
        const cx<T> D = csub(Xk, XL);
        const cx<T> wk = PADDED ? tws[k] : tws[kTwLds<T> ? tw_swz(k) : k];
        const cx<T> wD = cmul(cconj(wk), D);  // e^{+2 pi i k / nkx} D
        v[s] = cadd(A, mk<T>(-wD.y, wD.x));      // A + i w D
    }
    __syncthreads();
    if constexpr (PADDED)
        FP::run(v, xb, tw, gg);
    else
        F::run(v, xb, tw, 1, gg, lds_xor_gfast<L, G>(row));

    const T sc = (T)scale;
    const int qy = qy0 + row;
    if (MODE == 0) {
        for (int zi = 0; zi < zy; ++zi) {
            const int Y = zi * nky + ((qy + zy * nky / 2) & (nky - 1));
            T *orow = out + ((size_t)plane * out_ny + Y) * out_nx;
            const double2 fy = ff ? ffy[Y] : make_double2(1.0, 0.0);
            for (int zj = 0; zj < zx; ++zj) {
#pragma unroll
                for (int s = 0; s < E; ++s) {
                    const int u = 2 * (gg + s * G);
                    const int X = zj * nkx + ((u + nkx / 2) & (nkx - 1));
                    T a = v[s].x * sc, b = v[s].y * sc;
                    if (ff) {
                        a = (T)((double)a * form_factor_sq(ffx[X], fy, ffs));
                        b = (T)((double)b * form_factor_sq(ffx[X + 1], fy, ffs));
                    }
                    if (m2) {
                        // a band pair's |M(Q)|^2 map, the pairs summed in the output
                        const cx<T> mm = *reinterpret_cast<const cx<T> *>(m2 + (size_t)Y * out_nx + X);
                        a = (T)((double)a * (double)mm.x);
                        b = (T)((double)b * (double)mm.y);
                        if (acc) {
                            const cx<T> o = *reinterpret_cast<const cx<T> *>(orow + X);
                            a += o.x;
                            b += o.y;
                        }
                    }
                    *reinterpret_cast<cx<T> *>(orow + X) = mk<T>(a, b);
                }
            }
        }
    } else {
        // first-zone rows of lag m; out_ny rows per lag (nkz planes of nky rows in 3D)
        const int m = g.m_lo + slot;
        T *orow = out + ((size_t)m * out_ny + qy) * nkx;
#pragma unroll
        for (int s = 0; s < E; ++s) {
            const int u = 2 * (gg + s * G);
            *reinterpret_cast<cx<T> *>(orow + u) = mk<T>(v[s].x * sc, v[s].y * sc);
        }
    }
}

// ====================================================================== even
// Mirror-symmetric band: A(kx,ky) = A(-kx,ky) = A(kx,-ky), so every transform
// maps real even sequences to real even sequences.  Two real even lines are
// packed as one complex line z = a + i b; its full-length FFT is X_a + i X_b
// with X_a, X_b real, so the real and imaginary parts separate exactly.  Only
// rx in [0, nkx/2] and ry in [0, nky/2] are stored (see Geo).

// P1 (even): R row pairs (ky = 2p, 2p+1, ky <= nky/2) for jc slices.
// FP32: at least four waves per SIMD (with the momentum-density weights the
// kernel otherwise takes one register more than four waves allow); FP64 would
// spill under that bound.
template <typename T, int LOGNX, bool W>
__device__ __forceinline__ void e1_body(const double *__restrict__ xi, const Geo &g, double emin, double deps,
                                                double gamma, const cx<T> *__restrict__ twx, T *__restrict__ spec,
                                                const T *__restrict__ rho, int acc)
{
    constexpr int LOGE = ilog2_c(e1_elems(LOGNX));
    using F = RegFFT<T, LOGNX, false, LOGE, kTwLds<T>>;
    using FP = RegFFTP<T, LOGNX, false, LOGE, kRowPB>;
    constexpr bool PADDED = row_padded<T, LOGNX, LOGE>();
    constexpr int N = F::N, E = F::E, G = F::G;
    constexpr int LS = row_line_stride<T, LOGNX, LOGE>();
    extern __shared__ __align__(16) unsigned char smem_raw[];
    cx<T> *lds = reinterpret_cast<cx<T> *>(smem_raw);  // [R][LS]
    const int R = g.e1_R;
    const int tid = threadIdx.x;
    const int line = tid / G, gg = tid % G;
    const int p0 = blockIdx.x * R;
    const int kya = min(2 * (p0 + line), g.Hy - 1), kyb = min(2 * (p0 + line) + 1, g.Hy - 1);
    const int jbeg = g.jA + blockIdx.y * g.e1_jc;
    const int jend = min(g.jB, jbeg + g.e1_jc);
    cx<T> *buf = lds + line * LS;
    // FP32: the twiddle table lives in LDS after the line buffers
    const cx<T> *tw = twx;
    if (sizeof(T) == 4) {
        cx<T> *twl = lds + R * LS;
        if constexpr (PADDED)
            FP::fill_twiddles(twl, twx, tid, R * G);
        else
            for (int i = tid; i < N; i += R * G) twl[tw_swz(i)] = twx[i];
        tw = twl;
        __syncthreads();
    }
    double xa[E], xb[E];
    T ra[W ? E : 1], rb[W ? E : 1];  // momentum-density weights (W)
#pragma unroll
    for (int s = 0; s < E; ++s) {
        xa[s] = xi[(size_t)kya * N + gg + s * G];
        xb[s] = xi[(size_t)kyb * N + gg + s * G];
        if constexpr (W) {
            ra[s] = rho[(size_t)kya * N + gg + s * G];
            rb[s] = rho[(size_t)kyb * N + gg + s * G];
        }
    }
    const T gp = (T)(gamma / kPi), g2 = (T)(gamma * gamma);
    const int Ce = g.Ce, H = N / 2;
    const int rows = 2 * R, logRows = 1 + __builtin_ctz(R);
    constexpr int VEC = 16 / sizeof(T), HV = 32 / 16, logHV = 1;  // 16-byte pieces of a 32-byte tile row
    const int nvec = g.NTe * rows * HV;
    // Output items (VEC consecutive rx of one output row, 16 bytes; items
    // ordered half-row, row, tile so that a block writes whole tiles).  A
    // thread's items are the same in every slice, so they are decoded once:
    // LDS slot of the first value, byte offset in the slice, which row of the
    // packed pair, and whether all VEC values lie in [0, nkx/2] (only the last
    // tile's items do not).  nvec / (R G) <= 2 E / Ce + 4 E / N.
    constexpr int MAXIT = 2 * E / (32 / (int)sizeof(T)) + 4 * E / N + 1;
    int islot[MAXIT], ioff[MAXIT], irx[MAXIT];
    bool iodd[MAXIT], ifull[MAXIT];
#pragma unroll
    for (int k = 0; k < MAXIT; ++k) {
        const int it = tid + k * R * G;
        const int h = it & (HV - 1);
        const int r = (it >> logHV) & (rows - 1);
        const int tile = (it >> logHV) >> logRows;
        const int ky = 2 * p0 + r;
        const int rx0 = tile * Ce + h * VEC;
        const bool ok = it < nvec && ky < g.Hy;
        irx[k] = rx0;
        iodd[k] = (r & 1) != 0;
        ifull[k] = rx0 + VEC - 1 <= H;
        // rx0 is a multiple of VEC: no padding slot falls between the VEC values
        islot[k] = (r >> 1) * LS + row_slot<T, LOGNX, LOGE>(min(rx0, H));
        ioff[k] = ok ? ((tile * g.HyS + ky) * Ce + h * VEC) * (int)sizeof(T) : -1;
    }
    for (int j = jbeg; j < jend; ++j) {
        const double ej = emin + (j + 0.5) * deps;
        cx<T> v[E];
#pragma unroll
        for (int s = 0; s < E; ++s) {
            const T d0 = (T)(ej - xa[s]), d1 = (T)(ej - xb[s]);
            if constexpr (W)
                v[s] = mk<T>(lorentz(d0, gp, g2) * ra[s], lorentz(d1, gp, g2) * rb[s]);
            else
                v[s] = mk<T>(lorentz(d0, gp, g2), lorentz(d1, gp, g2));
        }
        if constexpr (PADDED) {
            FP::run(v, buf, tw, gg);
            // only rx in [0, nkx/2] is stored (s G is a multiple of the padding period)
            cx<T> *ob = buf + FP::pad(gg);
#pragma unroll
            for (int s = 0; s <= E / 2; ++s)
                if (gg + s * G <= H) ob[FP::pad(s * G)] = v[s];
        } else {
            F::run(v, buf, tw, 0, gg, lds_xor_gfast<N, G>(line));
#pragma unroll
            for (int s = 0; s <= E / 2; ++s)
                if (gg + s * G <= H) buf[gg + s * G] = v[s];
        }
        __syncthreads();
        // 32-bit offsets into the slice through a buffer descriptor
        const __amdgpu_buffer_rsrc_t rs = __builtin_amdgcn_make_buffer_rsrc(
            (void *)(spec + (size_t)(j - g.jA) * g.slice_e), 0, (int)(g.slice_e * sizeof(T)), 0x00020000);
#pragma unroll
        for (int k = 0; k < MAXIT; ++k) {
            if (ioff[k] < 0) continue;
            const cx<T> *zp = lds + islot[k];
            Vec16<T> o;
            if (ifull[k]) {
#pragma unroll
                for (int i = 0; i < VEC; ++i) o.v[i] = iodd[k] ? zp[i].y : zp[i].x;
            } else {
                // the last tile: the values past nkx/2 are zero (zp holds rx0 <= nkx/2)
#pragma unroll
                for (int i = 0; i < VEC; ++i) o.v[i] = irx[k] + i <= H ? (iodd[k] ? zp[i].y : zp[i].x) : (T)0;
            }
            const int off = ioff[k];
            if (acc) {  // add this band to the earlier ones
                const Vec16<T> old = __builtin_bit_cast(Vec16<T>, __builtin_amdgcn_raw_buffer_load_b128(rs, off, 0, 0));
#pragma unroll
                for (int i = 0; i < VEC; ++i) o.v[i] += old.v[i];
            }
            __builtin_amdgcn_raw_buffer_store_b128(__builtin_bit_cast(lh_u4, o), rs, off, 0, 0);
        }
        __syncthreads();
    }
}

template <typename T, int LOGNX, bool W>
__global__ void __launch_bounds__(kThreads, (sizeof(T) == 4 && LOGNX < 12) ? 4 : 1) k_e1(const double *__restrict__ xi, Geo g, double emin, double deps,
                                                double gamma, const cx<T> *__restrict__ twx, T *__restrict__ spec,
                                                const T *__restrict__ rho, int acc)
{
    e1_body<T, LOGNX, W>(xi, g, emin, deps, gamma, twx, spec, rho, acc);
}
// Batched P1: instance blockIdx.z of the descriptors (band 0, no accumulation)
template <typename T, int LOGNX, bool W>
__global__ void __launch_bounds__(kThreads, (sizeof(T) == 4 && LOGNX < 12) ? 4 : 1) k_e1_batch(const EvenInst *__restrict__ in)
{
    const EvenInst &d = in[blockIdx.z];
    const Geo g = d.g;
    if ((int)blockIdx.y * g.e1_jc >= g.nS) return;
    e1_body<T, LOGNX, W>(d.xi, g, d.emin, d.deps, d.gamma, (const cx<T> *)d.twx, (T *)d.spec, (const T *)d.rho, 0);
}

// Column pass (even), forward or inverse: each line is a pair of adjacent
// real columns of a tile (read as one complex value per row); rows above
// nky/2 are the mirror of the stored ones.  Transformed in place.
template <typename T, int LOGN, bool INV>
__device__ __forceinline__ void ecol_body(T *__restrict__ spec, const Geo &g,
                                                           const cx<T> *__restrict__ twy)
{
    using F = RegFFT<T, LOGN, INV, ilog2_c(kEcolElems), kTwLds<T>>;
    constexpr int N = F::N, E = F::E, G = F::G;
    constexpr int C = sizeof(T) == 4 ? 4 : 2;  // complex pairs per tile row
    constexpr int TPB = (G * C >= 256) ? 1 : 256 / (G * C);
    constexpr int NL = TPB * C;
    extern __shared__ __align__(16) unsigned char smem_raw[];
    cx<T> *lds = reinterpret_cast<cx<T> *>(smem_raw);
    const int tid = threadIdx.x;
    const int line = tid % NL, gg = tid / NL;
    const int tb = line / C, c = line % C;
    const int tile = blockIdx.x * TPB + tb;
    const bool active = tile < g.NTe;
    const int Hy = g.Hy;
    // twiddles first: the barrier that ends the copy then does not wait for
    // the column loads as well
    const cx<T> *tw = tw_to_lds<T>(twy, lds + NL * N, N, tid, NL * G);
    cx<T> *base = reinterpret_cast<cx<T> *>(spec + (size_t)blockIdx.y * g.slice_e +
                                            (size_t)(active ? tile : 0) * g.HyS * (2 * C));
    cx<T> v[E];
#pragma unroll
    for (int s = 0; s < E; ++s) {
        const int ky = gg + s * G;
        const int row = ky <= N / 2 ? ky : N - ky;
        v[s] = active ? base[row * C + c] : mk<T>((T)0, (T)0);
    }
    F::run(v, lds + line * N, tw, 0, gg, lds_xor_interleaved<T, N>(line, NL));
    if (active) {
#pragma unroll
        for (int s = 0; s < E; ++s) {
            const int ry = gg + s * G;
            if (ry < Hy) base[ry * C + c] = v[s];
        }
    }
}

template <typename T, int LOGN, bool INV>
__global__ void __launch_bounds__(col_threads(LOGN)) k_ecol(T *__restrict__ spec, Geo g,
                                                           const cx<T> *__restrict__ twy)
{
    ecol_body<T, LOGN, INV>(spec, g, twy);
}
// Batched column pass: instance blockIdx.z, its nS (forward) or nL (inverse) slices
template <typename T, int LOGN, bool INV>
__global__ void __launch_bounds__(col_threads(LOGN)) k_ecol_batch(const EvenInst *__restrict__ in)
{
    const EvenInst &d = in[blockIdx.z];
    const Geo g = d.g;
    if ((int)blockIdx.y >= (INV ? g.nL : g.nS)) return;
    ecol_body<T, LOGN, INV>((T *)d.spec, g, (const cx<T> *)d.twy);
}

// Energy window (even, direct): S(r, m) = sum_j B(r, j) B(r, j + m), real.
// With P'[a] = B(j0 - 1 - a) (occupied, reversed) and H'[x] = B(j0 + x)
// (unoccupied), S(m) = sum_{a=0}^{m-1} P'[a] H'[m-1-a]: a linear convolution.
// Both arrays are staged in LDS with zero padding.  One block: TR consecutive
// points of the flattened slice; lanes are TR points x SU = 64/TR sub-ranges
// of a (lengths 1 mod 4, so the SU lane groups read different LDS bank
// quarters; only the last chunk of a sub-range is masked); each wave takes
// blocks of 16 lags held in registers with a 16-value sliding window of H'
// (16 FMAs per two LDS reads).  Products are summed in T over 32 steps; the
// block sums are accumulated in FP64 (compensating the FP32 partial sums) and
// the lane partials are merged in FP64.  COMP selects nothing else today: the
// FP64 instantiation sums in FP64 throughout.
template <typename T, bool COMP, int TR>
__device__ __forceinline__ void e3_body(T *__restrict__ spec, const Geo &g)
{
    constexpr int SU = 64 / TR;
    constexpr int HP = 16 * SU + 32;
    extern __shared__ __align__(16) unsigned char smem_raw[];
    T *lds = reinterpret_cast<T *>(smem_raw);
    const int PL = g.e3_PL, HL = g.m_lo + 16 * ((g.nL + 15) >> 4) - 1;
    T *Pz = lds;                    // [PL][TR]
    T *Hz = lds + (size_t)PL * TR;  // [HP + HL][TR], row (HP + x)
    const int tid = threadIdx.x;
    const size_t p0 = (size_t)xcd_tile(blockIdx.x, gridDim.x) * TR;
    const int ne = g.nS, j0 = g.j0 - g.jA;
    const size_t sl = g.slice_e;
    // Stage P' and H' with batches of independent loads (clamped addresses,
    // select afterwards) so that the loads of one thread overlap.
    {
        constexpr int UNR = 8;
        const int nP = PL * TR, nH = (HP + HL) * TR;
        for (int it0 = tid; it0 < nP + nH; it0 += UNR * kThreads) {
            T v[UNR];
#pragma unroll
            for (int k = 0; k < UNR; ++k) {
                const int it = it0 + k * kThreads;
                const bool inP = it < nP;
                const int row = inP ? it / TR : (it - nP) / TR;
                const int p = it % TR;
                const size_t pt = p0 + p;
                int js;
                bool ok;
                if (inP) {
                    js = j0 - 1 - row;
                    ok = row < j0;
                } else {
                    js = j0 + row - HP;
                    ok = row >= HP && js < ne;
                }
                ok = ok && it < nP + nH && pt < sl;
                const size_t src = ok ? (size_t)js * sl + pt : 0;
                const T x = spec[src];
                v[k] = ok ? x : (T)0;
            }
#pragma unroll
            for (int k = 0; k < UNR; ++k) {
                const int it = it0 + k * kThreads;
                if (it < nP + nH) lds[it] = v[k];
            }
        }
    }
    __syncthreads();
    const int lane = tid & 63, wave = tid >> 6;
    const int p = lane % TR;
    const int su = lane / TR;
    const int nB = (g.nL + 15) >> 4;
    for (int b = wave; b < nB; b += kThreads / 64) {
        const int mf = g.m_lo + 16 * b;
        const int Atot = min(mf + 15, j0);
        double acc[16];
#pragma unroll
        for (int i = 0; i < 16; ++i) acc[i] = 0.0;
        if (Atot > 0) {
            // sub-range length cl = 1 (mod 4) puts the SU lane groups on
            // different LDS bank quarters; the last chunk is masked
            int cl = (Atot + SU - 1) / SU;
            if (SU > 1) cl += (1 - cl) & 3;
            const int nfull = cl >> 4;
            const int as = su * cl;
            // window slot (i - u) & 15 holds H'[mf - 1 - a + i], a = as + step
            const T *pp = Pz + as * TR + p;
            const T *hp = Hz + (HP + mf - 1 - as) * TR + p;
            T w[16];
#pragma unroll
            for (int i = 0; i < 16; ++i) w[i] = hp[i * TR];
            T tmp[16];
#pragma unroll
            for (int i = 0; i < 16; ++i) tmp[i] = (T)0;
            for (int c = 0; c <= nfull; ++c) {
                const int rem = c < nfull ? 16 : cl - 16 * nfull;  // wave-uniform
                if (rem == 0) break;
                hp -= 16 * TR;
                if (rem == 16) {
#pragma unroll
                    for (int u = 0; u < 16; ++u) {
                        const T pv = pp[u * TR];
#pragma unroll
                        for (int i = 0; i < 16; ++i) tmp[i] += pv * w[(i - u) & 15];
                        w[(15 - u) & 15] = hp[(15 - u) * TR];
                    }
                } else {
#pragma unroll
                    for (int u = 0; u < 16; ++u) {
                        const T pv = u < rem ? pp[u * TR] : (T)0;
#pragma unroll
                        for (int i = 0; i < 16; ++i) tmp[i] += pv * w[(i - u) & 15];
                        w[(15 - u) & 15] = hp[(15 - u) * TR];
                    }
                }
                pp += 16 * TR;
                if ((c & 1) || c + 1 >= nfull + (cl > 16 * nfull ? 1 : 0)) {
#pragma unroll
                    for (int i = 0; i < 16; ++i) {
                        acc[i] += (double)tmp[i];
                        tmp[i] = (T)0;
                    }
                }
            }
        }
        for (int o = TR; o < 64; o <<= 1) {
#pragma unroll
            for (int i = 0; i < 16; ++i) acc[i] += __shfl_xor(acc[i], o, 64);
        }
        if (su == 0 && p0 + p < sl) {
#pragma unroll
            for (int i = 0; i < 16; ++i) {
                const int m = mf + i;
                if (m <= g.m_hi) spec[(size_t)(m - g.m_lo) * sl + p0 + p] = (T)acc[i];
            }
        }
    }
}

template <typename T, bool COMP, int TR>
__global__ void __launch_bounds__(kThreads) k_e3(T *__restrict__ spec, Geo g)
{
    e3_body<T, COMP, TR>(spec, g);
}
// Batched direct window: instance blockIdx.z
template <typename T, bool COMP, int TR>
__global__ void __launch_bounds__(kThreads) k_e3_batch(const EvenInst *__restrict__ in)
{
    const EvenInst &d = in[blockIdx.z];
    const Geo g = d.g;
    e3_body<T, COMP, TR>((T *)d.spec, g);
}

// Energy window (even) on the matrix cores.  The same convolution
// S(m) = sum_a P'[a] H'[m-1-a] as k_e3, blocked by 16: with m = m0 + 16 c + i
// (c = 0..15 output column, i = 0..15 row) and a = 16 n + k, the block pair
// (c, n) only depends on e = c - n through the Toeplitz block
// T_e[i][k] = H'[m0 - 1 + 16 e + i - k], so for every e one 16x16x16 product
// T_e * [P'_0 ... P'_15] (four 16x16x4 MFMAs, columns n) gives the terms of
// column c = n + e: the result is moved e columns to the right with DPP row
// shifts (zeros shifted in, columns pushed past 15 dropped) and added to the
// accumulator.  The P' operand is loaded once per point; each MFMA reads one
// Toeplitz operand from LDS.  FP32: partial sums of four e (64 products) are
// accumulated in FP64; FP64: everything in FP64.
//
// Operand layouts (16x16x4): A lane l = (row l%16, k l/16); B lane l =
// (k l/16, column l%16); D lane l, register r = (row 4(l/16)+r, column l%16)
// for FP32 and (row 4r+l/16, column l%16) for FP64.
//
// Tiles of TR consecutive points; each point staged point-major, stride PS
// (congruent to 64 / TR modulo 64, so that the staging writes of one wave hit
// 64 different banks): [PA values P'[a], zero for a >= nA][32 zeros]
// [nHe values H'[x]][32 zeros].  Lags and occupied energies beyond 256 are
// handled in groups of 256 (NMG, NAG).  Each wave takes TR/4 points; results
// go through an LDS tile [256 lags][TR + 1] so that the in-place stores of S
// are coalesced.  Blocks are persistent and load the next tile into
// registers while the current one is on the matrix cores.
typedef float lh_f4 __attribute__((ext_vector_type(4)));
typedef double lh_d4 __attribute__((ext_vector_type(4)));

template <typename T>
struct MfmaVec;
template <>
struct MfmaVec<float> {
    using V = lh_f4;
};
template <>
struct MfmaVec<double> {
    using V = lh_d4;
};

__device__ __forceinline__ lh_f4 mfma16x16x4(float a, float b, lh_f4 c)
{
    return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
}
__device__ __forceinline__ lh_d4 mfma16x16x4(double a, double b, lh_d4 c)
{
    return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
}

// Value of column c - E of the same 16-lane row (0 where that is outside the row).
template <int E>
__device__ __forceinline__ int col_shift_i(int v)
{
    constexpr int ctl = E > 0 ? 0x110 + E : 0x100 - E;  // row_shr:E, row_shl:-E
    return __builtin_amdgcn_update_dpp(0, v, ctl, 0xF, 0xF, true);
}
template <int E>
__device__ __forceinline__ float col_shift(float v)
{
    if constexpr (E == 0)
        return v;
    else
        return __int_as_float(col_shift_i<E>(__float_as_int(v)));
}
template <int E>
__device__ __forceinline__ double col_shift(double v)
{
    if constexpr (E == 0) {
        return v;
    } else {
        const long long b = __double_as_longlong(v);
        const int lo = col_shift_i<E>((int)(b & 0xffffffffLL));
        const int hi = col_shift_i<E>((int)(b >> 32));
        return __longlong_as_double((long long)(unsigned)lo | ((long long)hi << 32));
    }
}

// Row of the 16x16 result held in register r by lane group k4 = lane / 16.
template <typename T>
__device__ __forceinline__ int mfma_row(int r, int k4)
{
    return sizeof(T) == 4 ? 4 * k4 + r : 4 * r + k4;
}

// x + T_E [P'_0 .. P'_15]: four 16x16x4 products accumulated on x.
template <typename T, int E>
__device__ __forceinline__ typename MfmaVec<T>::V e3m_prod(const T *hb, const T (&b)[4], typename MfmaVec<T>::V x)
{
    x = mfma16x16x4(hb[16 * E], b[0], x);
    x = mfma16x16x4(hb[16 * E - 4], b[1], x);
    x = mfma16x16x4(hb[16 * E - 8], b[2], x);
    x = mfma16x16x4(hb[16 * E - 12], b[3], x);
    return x;
}

template <int S, typename V>
__device__ __forceinline__ V vshift(V x)
{
#pragma unroll
    for (int r = 0; r < 4; ++r) x[r] = col_shift<S>(x[r]);
    return x;
}

// Horner chains over groups of four e: the products of a group are summed in
// the precision of the MFMA (64 products per FP32 partial sum) and each group
// is folded once into the FP64 accumulator.  A chain runs from the largest e
// of its group down, with one-column right shifts in between and a final
// right shift by the smallest e; every shift moves the same way, so what
// leaves the 16-column row has left the lag block for good.
// Four Horner chains at once (e from EA, EA + 4, EA + 8 and EA + 12 downwards,
// N steps each), their products interleaved so that the matrix ops of one
// chain run while the others wait for their results to be shifted.
template <typename T, int EA>
__device__ __forceinline__ void e3m_prod4(const T *hb, const T (&b)[4], typename MfmaVec<T>::V (&x)[4])
{
#pragma unroll
    for (int s = 0; s < 4; ++s)
#pragma unroll
        for (int c = 0; c < 4; ++c) x[c] = mfma16x16x4(hb[16 * (EA + 4 * c) - 4 * s], b[s], x[c]);
}
template <typename T, int EA, int N>
__device__ __forceinline__ void e3m_chain4(const T *hb, const T (&b)[4], typename MfmaVec<T>::V (&x)[4])
{
    e3m_prod4<T, EA>(hb, b, x);
    if constexpr (N > 1) {
#pragma unroll
        for (int c = 0; c < 4; ++c) x[c] = vshift<1>(x[c]);
        e3m_chain4<T, EA - 1, N - 1>(hb, b, x);
    }
}

// Every e in [0, 15] (the whole range is known to be needed): the groups
// [0, 3], [4, 7], [8, 11], [12, 15] as four interleaved chains, each group's
// FP32 (or FP64) partial sum folded once into the FP64 accumulator.
template <typename T>
__device__ __forceinline__ void e3m_all(const T *hb, const T (&b)[4], double (&acc)[4])
{
    typename MfmaVec<T>::V x[4] = {{0, 0, 0, 0}, {0, 0, 0, 0}, {0, 0, 0, 0}, {0, 0, 0, 0}};
    e3m_chain4<T, 3, 4>(hb, b, x);
    x[1] = vshift<4>(x[1]);
    x[2] = vshift<8>(x[2]);
    x[3] = vshift<12>(x[3]);
#pragma unroll
    for (int r = 0; r < 4; ++r) acc[r] += ((double)x[0][r] + (double)x[1][r]) + ((double)x[2][r] + (double)x[3][r]);
}

// One e alone, folded at once (the general ranges of e3m_some).
template <typename T, int E>
__device__ __forceinline__ void e3m_one(const T *hb, const T (&b)[4], double (&acc)[4])
{
    typename MfmaVec<T>::V x = {0, 0, 0, 0};
    x = vshift<E>(e3m_prod<T, E>(hb, b, x));
#pragma unroll
    for (int r = 0; r < 4; ++r) acc[r] += (double)x[r];
}

// Only the e in [e_lo, e_hi] (wave-uniform bounds within [-15, 15]).
template <typename T, int E = -15>
__device__ __forceinline__ void e3m_some(const T *hb, const T (&b)[4], int e_lo, int e_hi, double (&acc)[4])
{
    if constexpr (E <= 15) {
        if (E >= e_lo && E <= e_hi) e3m_one<T, E>(hb, b, acc);
        e3m_some<T, E + 1>(hb, b, e_lo, e_hi, acc);
    }
}

// Staging geometry of one thread: P' rows a < nA, H' rows x < nHe (at row
// PA + 32 + x), byte offset qb of its points within the tile row, slice
// stride sb bytes.
struct E3mStage {
    int PA, nA, nHe;
    unsigned qb, sb;
};
struct E3mRsrc {
    __amdgpu_buffer_rsrc_t P, H;
};

// Buffer descriptors of one tile (first point p0): P' rows a at slice
// j0 - 1 - a counted from base slice j0 - nA, H' rows x at slice j0 + x; each
// range ends with the last element of its slices.
template <typename T>
__device__ __forceinline__ E3mRsrc e3m_rsrc(T *spec, size_t sl, int j0, int nA, int nHe, size_t p0)
{
    const size_t nP = (size_t)nA * sl, nH = (size_t)nHe * sl;
    E3mRsrc r;
    r.P = __builtin_amdgcn_make_buffer_rsrc((void *)(spec + (size_t)(j0 - nA) * sl + p0), 0,
                                            (int)(nP > p0 ? (nP - p0) * sizeof(T) : 0), 0x00020000);
    r.H = __builtin_amdgcn_make_buffer_rsrc((void *)(spec + (size_t)j0 * sl + p0), 0,
                                            (int)(nH > p0 ? (nH - p0) * sizeof(T) : 0), 0x00020000);
    return r;
}

// Staged row rr of this thread's points (0 for the zero rows: out-of-range
// offset; the P' / H' choice is wave-uniform).
template <typename T>
__device__ __forceinline__ Vec16<T> e3m_bload(const E3mRsrc &rs, const E3mStage &st, int rr)
{
    const bool wP = __builtin_amdgcn_readfirstlane(rr) < st.PA;
    const int x = rr - st.PA - 32;
    unsigned off;
    if (wP)
        off = rr < st.nA ? (unsigned)(st.nA - 1 - rr) * st.sb + st.qb : 0xFFFFFFF0u;
    else
        off = (x >= 0 && x < st.nHe) ? (unsigned)x * st.sb + st.qb : 0xFFFFFFF0u;
    const lh_u4 w = __builtin_amdgcn_raw_buffer_load_b128(wP ? rs.P : rs.H, (int)off, 0, 0);
    return __builtin_bit_cast(Vec16<T>, w);
}

// Write a staged row of this thread's points into the point-major LDS layout.
template <typename T>
__device__ __forceinline__ void e3m_put(T *lds, int PS, int pq, int rows, int rr, const Vec16<T> &v)
{
    if (rr < rows) {
#pragma unroll
        for (int i = 0; i < (int)(16 / sizeof(T)); ++i) lds[(pq + i) * PS + rr] = v.v[i];
    }
}

// Scalar staging (plain global loads, any size): point pst, slice stride sl.
struct E3mStageS {
    int PA, nA, nHe, pst;
};

// One staged row with a plain global load (any size).
template <typename T>
__device__ __forceinline__ T e3m_gload(const T *col, bool pv, const E3mStageS &st, int j0, int rows, size_t sl,
                                       int rr)
{
    int js;
    bool ok;
    if (rr < st.PA) {
        js = j0 - 1 - rr;
        ok = rr < st.nA;
    } else {
        const int xx = rr - st.PA - 32;
        js = j0 + xx;
        ok = xx >= 0 && xx < st.nHe;
    }
    ok = ok && rr < rows && pv;
    const T xv = col[ok ? (size_t)js * sl : 0];
    return ok ? xv : (T)0;
}

template <typename T, int TR>
__global__ void __launch_bounds__(kThreads, 4) k_e3m(T *__restrict__ spec, Geo g, int ntiles)
{
    static_assert(TR >= 4 && (TR & (TR - 1)) == 0, "TR: power of two >= 4");
    constexpr int PPW = TR / 4;  // points per wave
    constexpr int TS = TR + 1;   // row stride of the output tile
    extern __shared__ __align__(16) unsigned char smem_raw[];
    T *lds = reinterpret_cast<T *>(smem_raw);
    const int PA = g.e3m_PA, nA = g.e3m_nA, nHe = g.e3m_nHe, PS = g.e3m_PS;
    const int NAG = g.e3m_NAG, NMG = g.e3m_NMG;
    const int rows = PA + nHe + 64;
    const int tid = threadIdx.x;
    const int j0 = g.j0 - g.jA;
    const size_t sl = g.slice_e;
    // Persistent blocks: the blocks of one XCD (launch index mod 8) walk one
    // contiguous range of tiles, so neighbouring tiles meet in that XCD's L2.
    const int xcd = blockIdx.x & 7, bi = blockIdx.x >> 3, bx = gridDim.x >> 3;
    const int per = (ntiles + 7) >> 3;
    const int t_end = min(ntiles, (xcd + 1) * per);
    int t = xcd * per + bi;
    if (t >= t_end) return;

    // Staging with buffer loads (both slice ranges below 4 GiB): each lane
    // loads VEC consecutive points (16 bytes) of one row, LR lanes per row,
    // rows r0 + k RP (the 64 / LR rows of one wave at one k never straddle
    // the P' / H' boundary, a multiple of 256); rows of zeros get an
    // out-of-range offset and read 0.  Otherwise plain global loads, one
    // point per lane.
    constexpr int VEC = 16 / sizeof(T);
    static_assert(TR >= VEC, "a tile row holds at least one 16-byte load");
    constexpr int LR = TR / VEC, RP = kThreads / LR;
    constexpr int NPF = (TR == 16 && sizeof(T) == 4) ? 10 : 6;  // 16-byte registers of the next tile
    const int q = tid % LR, r0 = tid / LR;
    const bool buf = g.e3m_buf != 0;
    const E3mStage st{PA, nA, nHe, (unsigned)(q * 16), (unsigned)(sl * sizeof(T))};
    auto stage_sync = [&](size_t p0) {
        if (buf) {
            constexpr int UNR = 4;
            const E3mRsrc rs = e3m_rsrc(spec, sl, j0, nA, nHe, p0);
            for (int rb = r0; rb < rows; rb += UNR * RP) {
                Vec16<T> v[UNR];
#pragma unroll
                for (int k = 0; k < UNR; ++k) v[k] = e3m_bload<T>(rs, st, rb + k * RP);
#pragma unroll
                for (int k = 0; k < UNR; ++k) e3m_put<T>(lds, PS, q * VEC, rows, rb + k * RP, v[k]);
            }
        } else {
            constexpr int UNR = 8, RS = kThreads / TR;
            const int pst = tid % TR, r0s = tid / TR;
            const E3mStageS sts{PA, nA, nHe, pst};
            const bool pv = p0 + pst < sl;
            const T *col = spec + (pv ? p0 + pst : 0);
            for (int rb = r0s; rb < rows; rb += UNR * RS) {
                T v[UNR];
#pragma unroll
                for (int k = 0; k < UNR; ++k) v[k] = e3m_gload<T>(col, pv, sts, j0, rows, sl, rb + k * RS);
#pragma unroll
                for (int k = 0; k < UNR; ++k)
                    if (rb + k * RS < rows) lds[pst * PS + rb + k * RS] = v[k];
            }
        }
    };
    Vec16<T> pf[NPF];

    const int lane = tid & 63, wave = tid >> 6;
    const int c16 = lane & 15, k4 = lane >> 4;
    const bool overlay = NMG == 1;  // the output tile reuses the staging area
    const bool prefetch = buf && overlay && rows <= NPF * RP;
    T *tile = overlay ? lds : lds + (size_t)TR * PS;

    if (prefetch) {
        const E3mRsrc rs = e3m_rsrc(spec, sl, j0, nA, nHe, (size_t)t * TR);
#pragma unroll
        for (int k = 0; k < NPF; ++k) pf[k] = e3m_bload<T>(rs, st, r0 + k * RP);
#pragma unroll
        for (int k = 0; k < NPF; ++k) e3m_put<T>(lds, PS, q * VEC, rows, r0 + k * RP, pf[k]);
    } else {
        stage_sync((size_t)t * TR);
    }
    __syncthreads();
    for (;;) {
        const size_t p0 = (size_t)t * TR;
        const int tn = t + bx;
        const bool more = tn < t_end;
        if (prefetch && more) {  // in flight during the products
            const E3mRsrc rs = e3m_rsrc(spec, sl, j0, nA, nHe, (size_t)tn * TR);
            // The row offsets do not change from tile to tile; hiding r0 from
            // the optimiser keeps it from holding all NPF of them in registers
            // for the whole kernel (they are cheap to recompute).
            int r0v = r0;
            asm volatile("" : "+v"(r0v));
#pragma unroll
            for (int k = 0; k < NPF; ++k) pf[k] = e3m_bload<T>(rs, st, r0v + k * RP);
        }
        for (int gm = 0; gm < NMG; ++gm) {
            T res[PPW][4];
#pragma unroll
            for (int pi = 0; pi < PPW; ++pi) {
                const int P = (wave + 4 * pi) * PS;
                double acc[4] = {0.0, 0.0, 0.0, 0.0};
                for (int ga = 0; ga < NAG; ++ga) {
                    T b[4];
#pragma unroll
                    for (int s4 = 0; s4 < 4; ++s4) b[s4] = lds[P + 256 * ga + 16 * c16 + 4 * s4 + k4];
                    const int D0 = g.m_lo - 1 + 256 * (gm - ga);
                    // e with some H' index D0 + 16 e + [-15, 15] inside [0, nHe)
                    const int e_lo = max(-15, -((D0 + 15) >> 4));
                    const int e_hi = min(15, (nHe + 14 - D0) >> 4);
                    const T *hb = lds + (P + PA + 32 + D0 + c16 - k4);
                    if (e_lo == 0 && e_hi == 15)
                        e3m_all<T>(hb, b, acc);
                    else
                        e3m_some<T>(hb, b, e_lo, e_hi, acc);
                }
                if (overlay) {
#pragma unroll
                    for (int r = 0; r < 4; ++r) res[pi][r] = (T)acc[r];
                } else {
#pragma unroll
                    for (int r = 0; r < 4; ++r)
                        tile[(16 * c16 + mfma_row<T>(r, k4)) * TS + wave + 4 * pi] = (T)acc[r];
                }
            }
            __syncthreads();
            if (overlay) {
#pragma unroll
                for (int pi = 0; pi < PPW; ++pi)
#pragma unroll
                    for (int r = 0; r < 4; ++r)
                        tile[(16 * c16 + mfma_row<T>(r, k4)) * TS + wave + 4 * pi] = res[pi][r];
                __syncthreads();
            }
            const int mb = g.m_lo + 256 * gm;
            for (int it = tid; it < 256 * LR; it += kThreads) {
                const int row = it / LR, pq = (it % LR) * VEC;
                const int m = mb + row;
                if (m > g.m_hi) continue;
                const size_t pb = p0 + pq;
                T *dst = spec + (size_t)(m - g.m_lo) * sl + pb;
                if (pb + VEC <= sl) {
                    Vec16<T> v;
#pragma unroll
                    for (int i = 0; i < VEC; ++i) v.v[i] = tile[row * TS + pq + i];
                    *reinterpret_cast<lh_u4 *>(dst) = __builtin_bit_cast(lh_u4, v);
                } else {
                    for (int i = 0; i < VEC; ++i)
                        if (pb + i < sl) dst[i] = tile[row * TS + pq + i];
                }
            }
            __syncthreads();
        }
        if (!more) break;
        t = tn;
        if (prefetch) {
#pragma unroll
            for (int k = 0; k < NPF; ++k) e3m_put<T>(lds, PS, q * VEC, rows, r0 + k * RP, pf[k]);
        } else
            stage_sync((size_t)t * TR);
        __syncthreads();
    }
}

// P5 (even): R row pairs (qy = 2p, 2p+1 <= nky/2) of one plane.  Each line is
// the full even row rebuilt from rx in [0, nkx/2]; its FFT gives the two real
// rows C(qx, qy) for every qx, written to rows qy and nky - qy of each zone.
// MODE 0: extended, form-factor weighted output planes; MODE 1: first-zone
// planes (natural order) for the RPA path.
template <typename T, int LOGNX, int MODE>
__device__ __forceinline__ void e5_body(const T *__restrict__ spec, const Geo &g, const cx<T> *__restrict__ twx,
                                                const PlaneSrc *__restrict__ psrc, double scale, int zx, int zy,
                                                int ff, double ffs, const double2 *__restrict__ ffx,
                                                const double2 *__restrict__ ffy, T *__restrict__ out, int out_nx,
                                                int out_ny, const T *__restrict__ m2, int acc)
{
    using F = RegFFT<T, LOGNX, true, 4, kTwLds<T>>;
    using FP = RegFFTP<T, LOGNX, true, 4, kRowPB>;
    constexpr bool PADDED = row_padded<T, LOGNX, 4>();
    constexpr int N = F::N, E = F::E, G = F::G;
    constexpr int LS = row_line_stride<T, LOGNX, 4>();
    extern __shared__ __align__(16) unsigned char smem_raw[];
    cx<T> *lds = reinterpret_cast<cx<T> *>(smem_raw);  // [R][LS] complex; staging [2R][N/2+1] reals
    T *stage = reinterpret_cast<T *>(smem_raw);
    const int R = g.e5_R;
    const int tid = threadIdx.x, nthr = R * G;
    const int line = tid / G, gg = tid % G;
    const int plane = blockIdx.y;
    const int p0 = blockIdx.x * R;
    const PlaneSrc ps = MODE == 0 ? psrc[plane] : PlaneSrc{plane, -1, 1.0, 0.0};
    const int slot = ps.a;
    const int nkx = g.nkx, nky = g.nky, Hy = g.Hy, H = N / 2, SW = H + 1;
    const int rows = 2 * R, logRows = 1 + __builtin_ctz(R);

    if (MODE == 0 && slot < 0) {
        if (acc) return;  // adds nothing
        for (int rz = 0; rz < rows * 2 * zy; ++rz) {
            const int r = rz % rows, mir = (rz / rows) & 1, zi = rz / (2 * rows);
            const int qy0 = 2 * p0 + r;
            if (qy0 >= Hy) continue;
            const int qy = mir ? (nky - qy0) & (nky - 1) : qy0;
            const int Y = zi * nky + ((qy + zy * nky / 2) & (nky - 1));
            T *orow = out + ((size_t)plane * out_ny + Y) * out_nx;
            for (int X = tid; X < out_nx; X += nthr) orow[X] = (T)0;
        }
        return;
    }
    const int Ce = g.Ce;
    const T *src = spec + (size_t)slot * g.slice_e;
    // an omega between two lags: wa S[a] + wb S[b] (wb = 0 reads S[a] twice)
    const bool blend = ps.b >= 0 || ps.wa != 1.0;
    const T *src2 = spec + (size_t)(ps.b >= 0 ? ps.b : slot) * g.slice_e;
    const T wa = (T)ps.wa, wb = (T)ps.wb;
    constexpr int VEC = 16 / sizeof(T), HV = 2, logHV = 1;  // 16-byte pieces of a 32-byte tile row
    const int nvec = g.NTe * rows * HV;
    const cx<T> *tw = twx;
    if (sizeof(T) == 4) {
        // after the staging area (2R (N/2 + 1) reals < R LS complex)
        cx<T> *twl = lds + R * LS;
        if constexpr (PADDED)
            FP::fill_twiddles(twl, twx, tid, nthr);
        else
            for (int i = tid; i < N; i += nthr) twl[tw_swz(i)] = twx[i];
        tw = twl;  // made visible by the barrier after the staging loop
    }
    // 16-byte loads (items ordered half-row, row, tile), independent in
    // batches of 4 so that they overlap
    for (int it0 = tid; it0 < nvec; it0 += 4 * nthr) {
        Vec16<T> v[4];
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            const int it = it0 + k * nthr;
            const int h = it & (HV - 1);
            const int r = (it >> logHV) & (rows - 1);
            const int tile = (it >> logHV) >> logRows;
            const int qy = 2 * p0 + r;
            const bool ok = it < nvec && qy < Hy;
            const size_t o = ok ? ((size_t)tile * g.HyS + qy) * Ce + h * VEC : 0;
            v[k] = __builtin_bit_cast(Vec16<T>, *reinterpret_cast<const lh_u4 *>(src + o));
            if (blend) {
                const Vec16<T> y = __builtin_bit_cast(Vec16<T>, *reinterpret_cast<const lh_u4 *>(src2 + o));
#pragma unroll
                for (int i = 0; i < VEC; ++i) v[k].v[i] = wa * v[k].v[i] + wb * y.v[i];
            }
        }
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            const int it = it0 + k * nthr;
            const int h = it & (HV - 1);
            const int r = (it >> logHV) & (rows - 1);
            const int rx0 = ((it >> logHV) >> logRows) * Ce + h * VEC;
            const int qy = 2 * p0 + r;
            if (it < nvec) {
#pragma unroll
                for (int i = 0; i < VEC; ++i)
                    if (rx0 + i <= H) stage[r * SW + rx0 + i] = qy < Hy ? v[k].v[i] : (T)0;
            }
        }
    }
    __syncthreads();
    cx<T> v[E];
#pragma unroll
    for (int s = 0; s < E; ++s) {
        const int rx = gg + s * G;
        const int rr = rx <= H ? rx : N - rx;
        v[s] = mk<T>(stage[(2 * line) * SW + rr], stage[(2 * line + 1) * SW + rr]);
    }
    __syncthreads();
    if constexpr (PADDED)
        FP::run(v, lds + line * LS, tw, gg);
    else
        F::run(v, lds + line * N, tw, 0, gg, lds_xor_gfast<N, G>(line));

    const T sc = (T)scale;
    for (int half = 0; half < 2; ++half) {
        const int qy0 = 2 * (p0 + line) + half;
        if (qy0 >= Hy) continue;
        for (int mir = 0; mir < 2; ++mir) {
            const int qy = mir ? (nky - qy0) & (nky - 1) : qy0;
            if (mir && qy == qy0) continue;
            if (MODE == 0) {
                for (int zi = 0; zi < zy; ++zi) {
                    const int Y = zi * nky + ((qy + zy * nky / 2) & (nky - 1));
                    T *orow = out + ((size_t)plane * out_ny + Y) * out_nx;
                    const double2 fy = ff ? ffy[Y] : make_double2(1.0, 0.0);
                    for (int zj = 0; zj < zx; ++zj) {
#pragma unroll
                        for (int s = 0; s < E; ++s) {
                            const int qx = gg + s * G;
                            const int X = zj * nkx + ((qx + nkx / 2) & (nkx - 1));
                            T val = (half ? v[s].y : v[s].x) * sc;
                            if (ff) val = (T)((double)val * form_factor_sq(ffx[X], fy, ffs));
                            if (m2) {
                                // a band pair's |M(Q)|^2 map, the pairs summed in the output
                                val = (T)((double)val * (double)m2[(size_t)Y * out_nx + X]);
                                if (acc) val += orow[X];
                            }
                            orow[X] = val;
                        }
                    }
                }
            } else {
                const int m = g.m_lo + slot;
                T *orow = out + ((size_t)m * out_ny + qy) * nkx;
#pragma unroll
                for (int s = 0; s < E; ++s) orow[gg + s * G] = (half ? v[s].y : v[s].x) * sc;
            }
        }
    }
}

template <typename T, int LOGNX, int MODE>
__global__ void __launch_bounds__(kE5MaxThreads) k_e5(const T *__restrict__ spec, Geo g, const cx<T> *__restrict__ twx,
                                                const PlaneSrc *__restrict__ psrc, double scale, int zx, int zy,
                                                int ff, double ffs, const double2 *__restrict__ ffx,
                                                const double2 *__restrict__ ffy, T *__restrict__ out, int out_nx,
                                                int out_ny, const T *__restrict__ m2, int acc)
{
    e5_body<T, LOGNX, MODE>(spec, g, twx, psrc, scale, zx, zy, ff, ffs, ffx, ffy, out, out_nx, out_ny, m2, acc);
}
// Batched P5 (extended output planes): instance blockIdx.z, its omegas
template <typename T, int LOGNX, int MODE>
__global__ void __launch_bounds__(kE5MaxThreads) k_e5_batch(const EvenInst *__restrict__ in)
{
    const EvenInst &d = in[blockIdx.z];
    const Geo g = d.g;
    if ((int)blockIdx.y >= d.nomega) return;
    e5_body<T, LOGNX, MODE>((const T *)d.spec, g, (const cx<T> *)d.twx, d.psrc, d.scale, d.zx, d.zy, d.ff, d.ffs,
                            d.ffx, d.ffy, (T *)d.out, d.onx, d.ony, (const T *)nullptr, 0);
}

// First-zone value at lag m (0 outside 1 <= m < neps), and the blend
// (1 - f) value(m) + f value(m + 1) in FP64 for an omega between two lags.
template <typename T>
__device__ __forceinline__ T lag_value(const T *__restrict__ im1, size_t nk, size_t q, int neps, long m)
{
    const bool in = m >= 1 && m < neps;
    const T x = im1[(size_t)(in ? m : 1) * nk + q];
    return in ? x : (T)0;
}
template <typename T>
__device__ __forceinline__ double lag_blend(const T *__restrict__ im1, size_t nk, size_t q, int neps, long m,
                                            double f)
{
    return (1.0 - f) * (double)lag_value(im1, nk, q, neps, m) + f * (double)lag_value(im1, nk, q, neps, m + 1);
}

// Extended, form-factor weighted map from the first-zone planes (RPA path).
template <typename T>
__global__ void __launch_bounds__(kThreads) k_extend(const T *__restrict__ im1, int nkx, int nky, int nkz, int neps,
                                                    const int *__restrict__ lags, const double *__restrict__ fracs,
                                                    int nw, int zx, int zy, int ff, double ffs,
                                                    const double2 *__restrict__ ffx, const double2 *__restrict__ ffy,
                                                    T *__restrict__ out, int out_nx, int out_ny)
{
    // one thread per first-zone point (u, v) and group of four planes: the
    // first-zone values are read once and written to every zone image.  In
    // three dimensions v runs over nkz planes of nky rows (natural order);
    // plane z goes to the output block (z + nkz/2) mod nkz of zy * nky rows.
    const int u = blockIdx.x * kThreads + threadIdx.x;
    const int v = blockIdx.y;
    const int w0 = blockIdx.z * 4;
    if (u >= nkx) return;
    const size_t nk = (size_t)nkx * nky * nkz, q = (size_t)v * nkx + u;
    T vals[4];
#pragma unroll
    for (int i = 0; i < 4; ++i) {
        const int w = min(w0 + i, nw - 1);
        const double f = fracs[w];
        vals[i] = f > 0.0 ? (T)lag_blend(im1, nk, q, neps, lags[w], f) : lag_value(im1, nk, q, neps, lags[w]);
    }
    const size_t plane = (size_t)out_nx * out_ny;
    // (any grid size: modulo rather than masks)
    const int vy = v % nky, vz = v / nky;
    const int Yz = ((vz + nkz / 2) % nkz) * zy * nky;  // first row of the output block
    const int xu = (u + (zx * nkx) / 2) % nkx, yv = (vy + (zy * nky) / 2) % nky;
    for (int zi = 0; zi < zy; ++zi) {
        const int Yb = zi * nky + yv, Y = Yz + Yb;
        for (int zj = 0; zj < zx; ++zj) {
            const int X = zj * nkx + xu;
            const double m2 = ff ? form_factor_sq(ffx[X], ffy[Yb], ffs) : 1.0;
            const size_t o0 = (size_t)Y * out_nx + X;
#pragma unroll
            for (int i = 0; i < 4; ++i)
                if (w0 + i < nw) out[(size_t)(w0 + i) * plane + o0] = ff ? (T)((double)vals[i] * m2) : vals[i];
        }
    }
}

// Kramers-Kronig on the matrix cores: re1[slot][q] = sum_j w(lag, j) im1[j][q]
// for every needed lag, with FP64 products and sums (v_mfma_f64_16x16x4f64).
// The weights vanish unless j - lag is odd, so the lags come in tiles of 16
// of one parity and a tile sums over the 16 energies of the other parity in
// each chunk of 32.  Block: WV waves (one lag tile each; eight when there are
// more than four tiles, so that Im is read once for up to 128 lags) and 128 q;
// the chunk of Im (32 energies x 128 q) is staged through LDS and shared by
// the tiles, the next chunk's loads in flight while the current one is summed.
// Per step of 4 energies a wave loads its 16 x 4 weights (one double per
// lane, contiguous) and issues eight MFMAs, one per 16 q.
//   MFMA operands: lane l holds A[l % 16][l / 16] (lag row, energy) and
//   B[l / 16][l % 16] (energy, q); result register r of lane l is the sum for
//   lag row 4 r + l / 16 and q column l % 16.
typedef double lh_d4 __attribute__((ext_vector_type(4)));
constexpr int kKkQ = 128;            // q per block
constexpr int kKkStride = kKkQ + 8;  // LDS row stride (energies two apart land 16 banks apart)
template <typename T, int WV>
__global__ void __launch_bounds__(64 * WV) k_kkm(const T *__restrict__ im1, int nk, int neps,
                                                const double *__restrict__ w, const int2 *__restrict__ rows,
                                                int ntiles, int nch, T *__restrict__ re1)
{
    __shared__ __align__(16) T tile[32 * kKkStride];
    constexpr int NT = 64 * WV;                     // threads
    constexpr int VEC = 16 / sizeof(T);             // values per 16-byte load
    constexpr int NV = 32 * kKkQ / VEC / NT;        // loads per thread per chunk
    const int tid = threadIdx.x, lane = tid & 63;
    const int t = blockIdx.y * WV + (tid >> 6);    // this wave's lag tile
    const bool active = t < ntiles;
    const long q0 = (long)blockIdx.x * kKkQ;
    const int par = active ? (rows[t * 16].x & 1) : 0;
    const int J = 16 * nch;
    // staging: load v of a chunk covers energy row e = idx / (kKkQ / VEC), q group
    // 16-byte loads while every energy row starts on a 16-byte boundary (a
    // grid of any size may not: then element by element)
    const bool vec = nk % VEC == 0;
    auto load = [&](int c, Vec16<T> *v) {
#pragma unroll
        for (int k = 0; k < NV; ++k) {
            const int idx = tid + k * NT, e = idx / (kKkQ / VEC), qv = (idx % (kKkQ / VEC)) * VEC;
            const int j = 32 * c + e;
            if (vec && j < neps && q0 + qv < nk) {
                v[k] = *reinterpret_cast<const Vec16<T> *>(im1 + (size_t)j * nk + q0 + qv);
            } else {
#pragma unroll
                for (int u = 0; u < VEC; ++u)
                    v[k].v[u] = j < neps && q0 + qv + u < nk ? im1[(size_t)j * nk + q0 + qv + u] : (T)0;
            }
        }
    };
    auto store = [&](const Vec16<T> *v) {
#pragma unroll
        for (int k = 0; k < NV; ++k) {
            const int idx = tid + k * NT, e = idx / (kKkQ / VEC), qv = (idx % (kKkQ / VEC)) * VEC;
            *reinterpret_cast<Vec16<T> *>(&tile[e * kKkStride + qv]) = v[k];
        }
    };
    lh_d4 acc[8];
#pragma unroll
    for (int i = 0; i < 8; ++i) acc[i] = lh_d4{0.0, 0.0, 0.0, 0.0};
    Vec16<T> v[NV];
    double a[4];
    load(0, v);
    const double *wt = w + (size_t)(active ? t : 0) * J * 16 + lane;
#pragma unroll
    for (int s = 0; s < 4; ++s) a[s] = active ? wt[(size_t)(4 * s) * 16] : 0.0;
    // energy row of this lane's B operand within a chunk, step s: (1 - par) + 2 (4 s + lane / 16)
    const int erow = (1 - par) + 2 * (lane >> 4), qcol = lane & 15;
    for (int c = 0; c < nch; ++c) {
        __syncthreads();
        store(v);
        __syncthreads();
        double an[4];
        if (c + 1 < nch) {
            load(c + 1, v);
#pragma unroll
            for (int s = 0; s < 4; ++s) an[s] = active ? wt[(size_t)(16 * (c + 1) + 4 * s) * 16] : 0.0;
        }
        if (active) {
#pragma unroll
            for (int s = 0; s < 4; ++s) {
                const T *brow = tile + (erow + 8 * s) * kKkStride + qcol;
#pragma unroll
                for (int qt = 0; qt < 8; ++qt)
                    acc[qt] = __builtin_amdgcn_mfma_f64_16x16x4f64(a[s], (double)brow[16 * qt], acc[qt], 0, 0, 0);
            }
        }
        if (c + 1 < nch)
#pragma unroll
            for (int s = 0; s < 4; ++s) a[s] = an[s];
    }
    if (!active) return;
#pragma unroll
    for (int r = 0; r < 4; ++r) {
        const int slot = rows[t * 16 + 4 * r + (lane >> 4)].y;
        if (slot < 0) continue;
        T *dst = re1 + (size_t)slot * nk + q0 + qcol;
#pragma unroll
        for (int qt = 0; qt < 8; ++qt)
            if (q0 + 16 * qt + qcol < nk) dst[16 * qt] = (T)acc[qt][r];
    }
}

// RPA epilogue on the extended map: chi = |M|^2 (Re + i Im),
// chi_RPA = chi / (1 - V chi) with a contact (vkind 0) or Coulomb (vkind 1)
// interaction, FP64 arithmetic, rounded once to T.
template <typename T>
__global__ void __launch_bounds__(kThreads) k_rpa(const T *__restrict__ im1, const T *__restrict__ re1, int nkx,
                                                 int nky, int neps, const int *__restrict__ lags,
                                                 const double *__restrict__ fracs,
                                                 const int *__restrict__ kkslot, int nw, int zx,
                                                 int zy, int ff, double ffs, const double2 *__restrict__ ffx,
                                                 const double2 *__restrict__ ffy, int vkind, double V, int kzn,
                                                 T *__restrict__ re_out, T *__restrict__ imr, T *__restrict__ rer,
                                                 int out_nx, int out_ny, int nkz)
{
    // one thread per first-zone point (u, v) and group of four planes: the
    // first-zone Im / Re are read once and every zone image is written (in
    // three dimensions as in k_extend: v over nkz planes of nky rows)
    const int u = blockIdx.x * kThreads + threadIdx.x;
    const int v = blockIdx.y;
    const int w0 = blockIdx.z * 4;
    if (u >= nkx) return;
    const size_t q = (size_t)v * nkx + u, nk = (size_t)nkx * nky * nkz;
    double imv[4], rev[4];
#pragma unroll
    for (int i = 0; i < 4; ++i) {
        const int w = min(w0 + i, nw - 1);
        const double f = fracs[w];
        imv[i] = f > 0.0 ? (double)(T)lag_blend(im1, nk, q, neps, lags[w], f)
                         : (double)lag_value(im1, nk, q, neps, lags[w]);
        // Re chi at the omega: its lag's plane, or the blend of two lags
        const int sa = kkslot[2 * w], sb = kkslot[2 * w + 1];
        const double ra = (double)re1[(size_t)sa * nk + q];
        rev[i] = f > 0.0 && sb >= 0 ? (double)(T)((1.0 - f) * ra + f * (double)re1[(size_t)sb * nk + q]) : ra;
    }
    const size_t plane = (size_t)out_nx * out_ny;
    const int vy = v % nky, vz = v / nky;
    const int Zc = (vz + nkz / 2) % nkz, Yz = Zc * zy * nky;
    // kz in reciprocal-lattice units of the third axis (0 in two dimensions)
    const double hz = (double)(Zc - nkz / 2) / nkz;
    const int xu = (u + (zx * nkx) / 2) % nkx, yv = (vy + (zy * nky) / 2) % nky;
    for (int zi = 0; zi < zy; ++zi) {
        const int Yb = zi * nky + yv, Y = Yz + Yb;
        for (int zj = 0; zj < zx; ++zj) {
            const int X = zj * nkx + xu;
            // interaction: contact U = V, or Coulomb V / |Q|^2 with
            // Q = 2 pi (h, l, hz) in units of 1/a (h, l the reciprocal-lattice
            // coordinates of X, Y: a grid spanning kzn zones has a step of
            // kzn / n; hz that of the kz plane, lattice constant a along z
            // too); at Q = 0 chi_RPA -> -1/V -> 0
            double U = V;
            bool q0 = false;
            if (vkind == 1) {
                const double h = (double)kzn * (X - (zx * nkx) / 2) / nkx, l = (double)kzn * (Yb - (zy * nky) / 2) / nky;
                const double q2 = (2.0 * kPi) * (2.0 * kPi) * (h * h + l * l + hz * hz);
                q0 = q2 == 0.0;
                U = q0 ? 0.0 : V / q2;
            }
            const double m2 = ff ? form_factor_sq(ffx[X], ffy[Yb], ffs) : 1.0;
            const size_t o0 = (size_t)Y * out_nx + X;
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                if (w0 + i >= nw) break;
                double im = imv[i], re = rev[i];
                if (ff) {
                    im = (double)(T)(im * m2);
                    re = (double)(T)(re * m2);
                }
                const double a = 1.0 - U * re, b = U * im;
                const double inv = 1.0 / (a * a + b * b);
                const size_t o = (size_t)(w0 + i) * plane + o0;
                if (re_out) re_out[o] = (T)re;
                if (imr) imr[o] = q0 ? (T)0 : (T)(im * inv);
                if (rer) rer[o] = q0 ? (T)0 : (T)((re * a - U * im * im) * inv);
            }
        }
    }
}

// Dynamical structure factor from Im chi (Eq. (1)): S = -(1/pi) Im chi /
// (1 - exp(-omega / kT)) with omega = m d of each output plane; kT = 0 is the
// zero-temperature limit (factor 1 for omega > 0); omega = 0 gives 0.  VEC
// consecutive elements per thread (16-byte accesses) when both arrays allow.
template <typename T, int VEC>
__global__ void __launch_bounds__(kThreads) k_sqw(const T *__restrict__ im, T *__restrict__ s,
                                                 const int *__restrict__ lags, const double *__restrict__ fracs,
                                                 double deps, double kT, size_t plane)
{
    const int w = blockIdx.y;
    const double om = fracs[w] > 0.0 ? (lags[w] + fracs[w]) * deps : lags[w] * deps;
    double f;
    if (kT > 0.0)
        f = om == 0.0 ? 0.0 : 1.0 / (-expm1(-om / kT));
    else
        f = om > 0.0 ? 1.0 : 0.0;
    const double c = -(1.0 / kPi) * f;
    const size_t base = (size_t)w * plane;
    const size_t nv = plane / VEC;
    for (size_t i = (size_t)blockIdx.x * kThreads + threadIdx.x; i < nv; i += (size_t)gridDim.x * kThreads) {
        if constexpr (VEC > 1) {
            Vec16<T> v = __builtin_bit_cast(Vec16<T>, *reinterpret_cast<const lh_u4 *>(im + base + i * VEC));
#pragma unroll
            for (int k = 0; k < VEC; ++k) v.v[k] = (T)(c * (double)v.v[k]);
            *reinterpret_cast<lh_u4 *>(s + base + i * VEC) = __builtin_bit_cast(lh_u4, v);
        } else {
            s[base + i] = (T)(c * (double)im[base + i]);
        }
    }
}

// Average of every output plane over its (X, Y) points in FP64, in a fixed
// order (no atomics): kQavgBlocks partial sums per plane, then one thread
// per plane adds them up.
template <typename T>
__global__ void __launch_bounds__(kThreads) k_qavg_part(const T *__restrict__ im, size_t plane,
                                                       double *__restrict__ part)
{
    __shared__ double red[kThreads];
    const int w = blockIdx.y;
    const T *src = im + (size_t)w * plane;
    double acc = 0.0;
    for (size_t i = (size_t)blockIdx.x * kThreads + threadIdx.x; i < plane; i += (size_t)kQavgBlocks * kThreads)
        acc += (double)src[i];
    red[threadIdx.x] = acc;
    __syncthreads();
    for (int s2 = kThreads / 2; s2 > 0; s2 >>= 1) {
        if ((int)threadIdx.x < s2) red[threadIdx.x] += red[threadIdx.x + s2];
        __syncthreads();
    }
    if (threadIdx.x == 0) part[(size_t)w * kQavgBlocks + blockIdx.x] = red[0];
}

__global__ void __launch_bounds__(kThreads) k_qavg_final(const double *__restrict__ part, int nw, double inv,
                                                        double *__restrict__ out)
{
    const int w = blockIdx.x * kThreads + threadIdx.x;
    if (w >= nw) return;
    double s2 = 0.0;
    for (int b = 0; b < kQavgBlocks; ++b) s2 += part[(size_t)w * kQavgBlocks + b];
    out[w] = s2 * inv;
}

// Peak search over the output planes: for every (X, Y) the plane index with
// the largest -Im (the first one on ties), compared in the array's precision.
template <typename T>
__global__ void __launch_bounds__(kThreads) k_peak(const T *__restrict__ im, int32_t *__restrict__ idx, size_t plane,
                                                  int nw)
{
    const size_t p = (size_t)blockIdx.x * kThreads + threadIdx.x;
    if (p >= plane) return;
    T best = im[p];
    int32_t bw = 0;
    for (int w = 1; w < nw; ++w) {
        const T x = im[(size_t)w * plane + p];
        if (x < best) {
            best = x;
            bw = w;
        }
    }
    idx[p] = bw;
}

// ---------------------------------------------------------------- cuts
// Every output plane at caller-chosen extended points (a path such as the
// high-symmetry lines of Fig. 2(a)): out[w][p] = im[w][Y_p][X_p], with xy the
// (X, Y) pairs (checked against the grid on the host).
template <typename T>
__global__ void __launch_bounds__(kThreads) k_cut(const T *__restrict__ im, size_t plane, int out_nx,
                                                 const int *__restrict__ xy, int npts, T *__restrict__ out)
{
    const int p = blockIdx.x * kThreads + threadIdx.x;
    const int w = blockIdx.y;
    if (p >= npts) return;
    out[(size_t)w * npts + p] = im[(size_t)w * plane + (size_t)xy[2 * p + 1] * out_nx + xy[2 * p]];
}

// Zone-by-zone envelope of one plane along a cut from the extended-grid
// centre (Fig. 5): direction 0 runs along [100] (X = Xc + s, Y = Yc), 1 along
// [110] (X = Xc + s, Y = Yc + s).  With zones nk grid steps wide, segment 0
// is s in [0, nk/2) (the central zone up to its boundary) and segment k >= 1
// is s in [nk/2 + (k-1) nk, nk/2 + k nk) (the k-th zone along the cut).  Each segment contributes the point of its
// largest -Im chi (decided in the array's precision, the first on ties),
// normalised by the largest of them; then the one-parameter Lorentzian
// 1 / (1 + (q / k0)^2) is fitted by least squares over u = 1 / k0^2: a scan of
// F(u) = sum_k (y_k - 1/(1 + q_k^2 u))^2 over kEnvScan log-spaced u in
// [kEnvUlo, kEnvUhi], then bisection on dF/du inside the best scan cell.
// res: [k0, c_max, nseg, then (X, Y, q, y) per segment]; one block.
constexpr int kEnvScan = 4096;
constexpr double kEnvUlo = 1e-8, kEnvUhi = 1e8;

__device__ __forceinline__ double env_F(const double *q, const double *y, int n, double u)
{
    double f = 0.0;
    for (int k = 0; k < n; ++k) {
        const double r = y[k] - 1.0 / (1.0 + q[k] * q[k] * u);
        f += r * r;
    }
    return f;
}
__device__ __forceinline__ double env_dF(const double *q, const double *y, int n, double u)
{
    double f = 0.0;
    for (int k = 0; k < n; ++k) {
        const double q2 = q[k] * q[k], g = 1.0 / (1.0 + q2 * u);
        f += (y[k] - g) * q2 * g * g;
    }
    return 2.0 * f;
}

template <typename T>
__global__ void __launch_bounds__(kThreads) k_envelope(const T *__restrict__ im, int out_nx, int Xc, int Yc, int nk,
                                                      int dir, int nseg, double qstep, double *__restrict__ res)
{
    __shared__ T bv[kThreads];
    __shared__ int bs[kThreads];
    __shared__ double fv[kThreads];
    __shared__ int fi[kThreads];
    __shared__ double sq[LINDHARD_ENVELOPE_MAX], sy[LINDHARD_ENVELOPE_MAX];
    __shared__ int ss[LINDHARD_ENVELOPE_MAX];
    const int tid = threadIdx.x;
    for (int k = 0; k < nseg; ++k) {
        const int lo = k == 0 ? 0 : nk / 2 + (k - 1) * nk, hi = k == 0 ? nk / 2 : lo + nk;
        T best = (T)0;
        int bi = INT_MAX;
        for (int s = lo + tid; s < hi; s += kThreads) {  // increasing s: ties keep the first
            const T c = -im[(size_t)(dir ? Yc + s : Yc) * out_nx + Xc + s];
            if (bi == INT_MAX || c > best) {
                best = c;
                bi = s;
            }
        }
        bv[tid] = best;
        bs[tid] = bi;
        __syncthreads();
        for (int o = kThreads / 2; o > 0; o >>= 1) {
            if (tid < o) {
                const T vo = bv[tid + o];
                const int io = bs[tid + o];
                if (io != INT_MAX && (bs[tid] == INT_MAX || vo > bv[tid] || (vo == bv[tid] && io < bs[tid]))) {
                    bv[tid] = vo;
                    bs[tid] = io;
                }
            }
            __syncthreads();
        }
        if (tid == 0) {
            ss[k] = bs[0];
            sy[k] = (double)bv[0];
            sq[k] = qstep * (double)bs[0];
        }
        __syncthreads();
    }
    if (tid == 0) {
        double cmax = sy[0];
        for (int k = 1; k < nseg; ++k) cmax = sy[k] > cmax ? sy[k] : cmax;
        for (int k = 0; k < nseg; ++k) sy[k] = sy[k] / cmax;
        res[1] = cmax;
        res[2] = (double)nseg;
        for (int k = 0; k < nseg; ++k) {
            res[3 + 4 * k] = (double)(Xc + ss[k]);
            res[4 + 4 * k] = (double)(dir ? Yc + ss[k] : Yc);
            res[5 + 4 * k] = sq[k];
            res[6 + 4 * k] = sy[k];
        }
    }
    __syncthreads();
    // scan of F over log u
    const double sl = log(kEnvUlo), sh = log(kEnvUhi), ds = (sh - sl) / (kEnvScan - 1);
    double fb = 0.0;
    int ib = INT_MAX;
    for (int i = tid; i < kEnvScan; i += kThreads) {
        const double f = env_F(sq, sy, nseg, exp(sl + i * ds));
        if (ib == INT_MAX || f < fb) {
            fb = f;
            ib = i;
        }
    }
    fv[tid] = fb;
    fi[tid] = ib;
    __syncthreads();
    for (int o = kThreads / 2; o > 0; o >>= 1) {
        if (tid < o) {
            const double vo = fv[tid + o];
            const int io = fi[tid + o];
            if (vo < fv[tid] || (vo == fv[tid] && io < fi[tid])) {
                fv[tid] = vo;
                fi[tid] = io;
            }
        }
        __syncthreads();
    }
    if (tid == 0) {
        const int i = fi[0];
        double a = sl + (i > 0 ? i - 1 : 0) * ds, b = sl + (i < kEnvScan - 1 ? i + 1 : i) * ds;
        double sx = sl + i * ds;
        if (env_dF(sq, sy, nseg, exp(a)) < 0.0 && env_dF(sq, sy, nseg, exp(b)) > 0.0) {
            for (int it = 0; it < 200; ++it) {
                const double m = 0.5 * (a + b);
                if (m <= a || m >= b) break;
                if (env_dF(sq, sy, nseg, exp(m)) < 0.0)
                    a = m;
                else
                    b = m;
            }
            sx = 0.5 * (a + b);
        }
        res[0] = exp(-0.5 * sx);
    }
}

// ====================================================== grids of any size
// A transform of length N that is not a power of two runs as Bluestein's
// chirp convolution: with b_n = exp(i pi n^2 / N), the forward transform is
// X_k = conj(b_k) sum_n (x_n conj(b_n)) b_(k-n), a circular convolution of
// length M = 2^logM >= 2N - 2 done with two register FFTs of length M (the
// chirp is even in k - n, so the lags -(N-1) and N-1 may share one place).  The
// tables of one axis (built in FP64 on the host, rounded once): chirp b_n
// (n < N) and the spectra hf = FFT_M(B) / M, hi = FFT_M(conj B) / M of the
// chirp sequence B (B_m = b_m, B_(M-m) = b_m, zero between) for the forward
// and the inverse transform.
struct BsTab {
    const void *b, *hf, *hi, *tw;  // cx<T>[N], cx<T>[M], cx<T>[M], cx<T>[M] (FFT twiddles of length M)
    int n;
};

// Launch index -> work index such that grp consecutive work items (which
// share cache lines) run on one XCD: blocks are dispatched round-robin over the
// 8 XCDs, launch index b on XCD b mod 8.  The grid is padded to a multiple of
// 8 grp blocks; the caller skips work indices past its range.
__device__ __forceinline__ int xcd_group(int b, int grp)
{
    const int xcd = b & 7, i = b >> 3;
    return ((i / grp) * 8 + xcd) * grp + i % grp;
}

// A zero the optimiser cannot see through.  Added to a thread's position in
// a loop body it keeps the loads and LDS addresses that depend on it inside
// the loop, rather than hoisted out and held in registers across it.
__device__ __forceinline__ int opaque_zero()
{
    int z = 0;
    asm volatile("" : "+s"(z));
    return z;
}

// FP32 up to M = 4096: the FFT twiddles of an axis copied into LDS after the
// block's R line buffers (M values), so that every pass reads them from LDS
// rather than waiting on the cache.  FP64 and longer lines keep them in
// global memory (the table would take the block past 64 KB of LDS).
template <typename T, int LOGM>
__host__ __device__ constexpr bool bs_tw_lds()
{
    return sizeof(T) == 4 && LOGM <= 12;
}
// Every thread of the block calls it.
template <typename T, int M>
__device__ __forceinline__ BsTab bs_lds_twiddles(BsTab t, cx<T> *lds, int R, int tid, int nthr)
{
    if constexpr (bs_tw_lds<T, ilog2_c(M)>()) {
        cx<T> *twl = lds + R * M;
        const cx<T> *tw = (const cx<T> *)t.tw;
        for (int i = tid; i < M; i += nthr) twl[tw_swz(i)] = tw[i];
        __syncthreads();
        t.tw = twl;
    }
    return t;
}

// v[s] = x[g + s G] (zero for n >= N) -> the DFT of length N (INV: inverse,
// no 1/N) in the same places; TWS: t.tw is an LDS table stored with tw_swz.
// Every thread of the block calls it.
template <typename T, int LOGM, bool INV, bool TWS = false>
__device__ __forceinline__ void bs_line(cx<T> *v, cx<T> *buf, const BsTab &t, int g, int lx)
{
    using F = RegFFT<T, LOGM, false, 4, TWS>;
    using Fi = RegFFT<T, LOGM, true, 4, TWS>;
    constexpr int E = F::E, G = F::G;
    const cx<T> *b = (const cx<T> *)t.b, *h = (const cx<T> *)(INV ? t.hi : t.hf), *tw = (const cx<T> *)t.tw;
#pragma unroll
    for (int s = 0; s < E; ++s) {
        const int n = g + s * G;
        v[s] = n < t.n ? cmul(v[s], INV ? b[n] : cconj(b[n])) : mk<T>((T)0, (T)0);
    }
    F::run(v, buf, tw, 0, g, lx);
#pragma unroll
    for (int s = 0; s < E; ++s) v[s] = cmul(v[s], h[g + s * G]);
    __syncthreads();
    Fi::run(v, buf, tw, 0, g, lx);
#pragma unroll
    for (int s = 0; s < E; ++s) {
        const int k = g + s * G;
        if (k < t.n) v[s] = cmul(v[s], INV ? b[k] : cconj(b[k]));
    }
}

// P1, any size: R lines of one energy slice, each line two rows (ky = 2p,
// 2p + 1) packed as z = A(2p) + i A(2p + 1).  After bs_line the two spectra
// separate through the line's LDS buffer, X(2p)_k = (Z_k + conj Z_(N-k)) / 2,
// X(2p+1)_k = (Z_k - conj Z_(N-k)) / 2i; the rows are real, so only the
// columns kx <= nkx / 2 are kept (the others are conjugates), written to the
// column-tiled array (NT = ceil((nkx / 2 + 1) / C) tiles, padding columns 0).
// Two row pairs fill the 128-byte lines of a tile, so with one line per
// block the two blocks of a pair run on one XCD.  The twiddles stay in global
// memory here: this pass is bound by how many lines a CU holds, and a table in
// LDS would cost a third of them.
template <typename T, int LOGM, bool W>
__global__ void __launch_bounds__(512) k_bs_row(const double *__restrict__ xi, Geo g, double emin, double deps,
                                               double gamma, BsTab tx, cx<T> *__restrict__ spec,
                                               const T *__restrict__ rho)
{
    using F = RegFFT<T, LOGM, false>;
    constexpr int M = F::N, E = F::E, G = F::G;
    extern __shared__ __align__(16) unsigned char smem_raw[];
    cx<T> *lds = reinterpret_cast<cx<T> *>(smem_raw);
    const int R = g.bs_Rr;
    const int tid = threadIdx.x, line = tid / G, gg = tid % G;
    const int w = xcd_group(blockIdx.x, R >= 2 ? 1 : 2);
    if (w * R >= (g.nky + 1) / 2) return;  // padding block (block-uniform)
    const int p = w * R + line;              // row pair
    const int ka = min(2 * p, g.nky - 1), kb = min(2 * p + 1, g.nky - 1);
    const bool hasa = 2 * p < g.nky, hasb = 2 * p + 1 < g.nky;
    const int j = g.jA + blockIdx.y;
    const int nkx = g.nkx;
    const double ej = emin + (j + 0.5) * deps;
    const T gp = (T)(gamma / kPi), g2 = (T)(gamma * gamma);
    cx<T> v[E];
#pragma unroll
    for (int s = 0; s < E; ++s) {
        const int n = gg + s * G;
        T a = (T)0, b = (T)0;
        if (n < nkx) {
            a = lorentz((T)(ej - xi[(size_t)ka * nkx + n]), gp, g2);
            b = lorentz((T)(ej - xi[(size_t)kb * nkx + n]), gp, g2);
            if constexpr (W) {
                a *= rho[(size_t)ka * nkx + n];
                b *= rho[(size_t)kb * nkx + n];
            }
        }
        v[s] = mk<T>(hasa ? a : (T)0, hasb ? b : (T)0);
    }
    cx<T> *buf = lds + line * M;
    bs_line<T, LOGM, false>(v, buf, tx, gg, lds_xor_gfast<M, G>(line));
#pragma unroll
    for (int s = 0; s < E; ++s) {
        const int k = gg + s * G;
        if (k < nkx) buf[k] = v[s];
    }
    __syncthreads();
    cx<T> *dst = spec + (size_t)blockIdx.y * g.slice_elems;
    const int C = g.C, logC = g.logC, H = nkx / 2, ncol = g.NT * C;
    for (int k = gg; k < ncol; k += G) {
        cx<T> xa = mk<T>((T)0, (T)0), xb = xa;
        if (k <= H) {
            const cx<T> zk = buf[k], zn = cconj(buf[k == 0 ? 0 : nkx - k]);
            xa = cscale(cadd(zk, zn), (T)0.5);
            const cx<T> dd = csub(zk, zn);
            xb = mk<T>((T)0.5 * dd.y, (T)-0.5 * dd.x);  // (zk - zn) / 2i
        }
        const size_t o = ((size_t)(k >> logC) * g.nky) * C + (k & (C - 1));
        if (hasa) dst[o + (size_t)ka * C] = xa;
        if (hasb) dst[o + (size_t)kb * C] = xb;
    }
}

// Column pass, any size: lines along ky (stride C in a tile), one per
// column (tile, c), for bs_SJ slices; R lines per block, lane-interleaved so
// that a wave's loads cover neighbouring columns.  In FP32 the next slice's
// column is loaded while the current one is transformed.  When R < C the C / R blocks of one tile (whose 32-byte
// rows share 128-byte lines) run on one XCD.  Transformed in place.
template <typename T, int LOGM, bool INV>
__global__ void __launch_bounds__(512) k_bs_col(cx<T> *__restrict__ spec, Geo g, BsTab ty, int nslices)
{
    using F = RegFFT<T, LOGM, false>;
    constexpr int M = F::N, E = F::E, G = F::G;
    extern __shared__ __align__(16) unsigned char smem_raw[];
    cx<T> *lds = reinterpret_cast<cx<T> *>(smem_raw);
    const int R = g.bs_Rc;
    const int tid = threadIdx.x, line = tid % R, gg = tid / R;
    const int ncol = g.NT * g.C;
    const int w = xcd_group(blockIdx.x, R >= g.C ? 1 : g.C / R);
    if (w * R >= ncol) return;  // padding block (block-uniform)
    const int col = w * R + line;  // tile * C + c
    const bool active = col < ncol;
    const int tile = (active ? col : 0) >> g.logC, c = (active ? col : 0) & (g.C - 1);
    cx<T> *base0 = spec + (size_t)tile * g.nky * g.C + c;
    const int lx = lds_xor_interleaved<T, M>(line, R);
    const int j0 = blockIdx.y * g.bs_SJ, j1 = min(nslices, j0 + g.bs_SJ);
    const BsTab tl = bs_lds_twiddles<T, M>(ty, lds, R, tid, R * G);
    constexpr bool PF = sizeof(T) == 4;  // FP64 has no registers to spare for the prefetch
    cx<T> nx[E];
    auto load = [&](int j, int go) {
        const cx<T> *base = base0 + (size_t)j * g.slice_elems;
#pragma unroll
        for (int s = 0; s < E; ++s) {
            const int n = go + s * G;
            nx[s] = (active && n < g.nky) ? base[(size_t)n * g.C] : mk<T>((T)0, (T)0);
        }
    };
    if (PF) load(j0, gg);
    for (int j = j0; j < j1; ++j) {
        const int go = gg + opaque_zero();
        if (!PF) load(j, go);
        cx<T> v[E];
#pragma unroll
        for (int s = 0; s < E; ++s) v[s] = nx[s];
        if (PF && j + 1 < j1) load(j + 1, go);
        bs_line<T, LOGM, INV, bs_tw_lds<T, LOGM>()>(v, lds + line * M, tl, go, lx);
        if (active) {
            cx<T> *base = base0 + (size_t)j * g.slice_elems;
#pragma unroll
            for (int s = 0; s < E; ++s) {
                const int k = go + s * G;
                if (k < g.nky) base[(size_t)k * g.C] = v[s];
            }
        }
    }
}

// P5, any size: the inverse transform along kx of R lines of one output
// plane (wa S[a] + wb S[b] for an omega between two lags), each line the rows
// qy = 2p, 2p + 1 packed as z = S(2p) + i S(2p + 1): both rows have real
// transforms, so the real and imaginary parts of the result are the two
// output rows.  Columns rx > nkx / 2 are rebuilt as conj S(nkx - rx).  The
// rows are scaled and written Gamma-centred into every zone image:
// out[plane][zi nky + (qy + (zy nky)/2) mod nky][zj nkx + (qx + (zx nkx)/2)
// mod nkx], times the orbital |M(Q)|^2 if ff (MODE 0); MODE 1 (the RPA path)
// writes the first-zone map of window slot `plane` in natural order,
// out[m_lo + plane][qy][qx].
template <typename T, int LOGM, int MODE>
__global__ void __launch_bounds__(512) k_bs_p5(const cx<T> *__restrict__ spec, Geo g, BsTab tx,
                                              const PlaneSrc *__restrict__ psrc, double scale,
                                              T *__restrict__ out, int zx, int zy, int ff, double ffs,
                                              const double2 *__restrict__ ffx, const double2 *__restrict__ ffy)
{
    using F = RegFFT<T, LOGM, false>;
    constexpr int M = F::N, E = F::E, G = F::G;
    extern __shared__ __align__(16) unsigned char smem_raw[];
    cx<T> *lds = reinterpret_cast<cx<T> *>(smem_raw);
    const int R = g.bs_Rr;
    const int tid = threadIdx.x, line = tid / G, gg = tid % G;
    const int plane = blockIdx.y;
    const int w = xcd_group(blockIdx.x, R >= 2 ? 1 : 2);  // as in k_bs_row
    if (w * R >= (g.nky + 1) / 2) return;                  // padding block (block-uniform)
    const int p = w * R + line;
    const int qa = min(2 * p, g.nky - 1), qb = min(2 * p + 1, g.nky - 1);
    const bool hasa = 2 * p < g.nky, hasb = 2 * p + 1 < g.nky;
    const int nkx = g.nkx, nky = g.nky, H = nkx / 2;
    const PlaneSrc ps = MODE == 0 ? psrc[plane] : PlaneSrc{plane, -1, 1.0, 0.0};
    const int onx = MODE == 0 ? zx * nkx : nkx, ony = MODE == 0 ? zy * nky : nky;
    const int sx = MODE == 0 ? (zx * nkx) / 2 : 0, sy = MODE == 0 ? (zy * nky) / 2 : 0;
    const int nzx = MODE == 0 ? zx : 1, nzy = MODE == 0 ? zy : 1;
    const int oplane = MODE == 0 ? plane : g.m_lo + plane;
    // output rows of zone row zi: zi nky + (q + sy) mod nky
    const int ya = (qa + sy) % nky, yb = (qb + sy) % nky;
    if (ps.a < 0) {  // the plane is zero (block-uniform)
        for (int zi = 0; zi < nzy; ++zi) {
            T *ra = out + ((size_t)oplane * ony + zi * nky + ya) * onx;
            T *rb = out + ((size_t)oplane * ony + zi * nky + yb) * onx;
            for (int k = gg; k < onx; k += G) {
                if (hasa) ra[k] = (T)0;
                if (hasb) rb[k] = (T)0;
            }
        }
        return;
    }
    const BsTab tl = bs_lds_twiddles<T, M>(tx, lds, R, tid, R * G);
    const cx<T> *src = spec + (size_t)ps.a * g.slice_elems;
    const cx<T> *src2 = spec + (size_t)(ps.b >= 0 ? ps.b : ps.a) * g.slice_elems;
    const bool blend = ps.b >= 0 || ps.wa != 1.0;
    const T wa = (T)ps.wa, wb = (T)ps.wb;
    const int C = g.C, logC = g.logC;
    auto at = [&](int row, int k) {  // S(k, row) for k <= nkx / 2
        const size_t o = ((size_t)(k >> logC) * nky + row) * C + (k & (C - 1));
        cx<T> x = src[o];
        if (blend) {
            const cx<T> y = src2[o];
            x = mk<T>(wa * x.x + wb * y.x, wa * x.y + wb * y.y);
        }
        return x;
    };
    cx<T> v[E];
#pragma unroll
    for (int s = 0; s < E; ++s) {
        const int k = gg + s * G;
        cx<T> z = mk<T>((T)0, (T)0);
        if (k < nkx) {
            const bool lo = k <= H;
            const int kk = lo ? k : nkx - k;
            cx<T> sa = at(qa, kk), sb = at(qb, kk);
            if (!lo) {
                sa = cconj(sa);
                sb = cconj(sb);
            }
            if (!hasb) sb = mk<T>((T)0, (T)0);
            z = mk<T>(sa.x - sb.y, sa.y + sb.x);  // sa + i sb
        }
        v[s] = z;
    }
    bs_line<T, LOGM, true, bs_tw_lds<T, LOGM>()>(v, lds + line * M, tl, gg, lds_xor_gfast<M, G>(line));
    const T sc = (T)scale;
    const int xs = MODE == 0 ? sx : 0;
    for (int zi = 0; zi < nzy; ++zi) {
        const int Ya = zi * nky + ya, Yb = zi * nky + yb;
        T *ra = out + ((size_t)oplane * ony + (MODE == 0 ? Ya : qa)) * onx;
        T *rb = out + ((size_t)oplane * ony + (MODE == 0 ? Yb : qb)) * onx;
        const double2 fya = ff ? ffy[Ya] : make_double2(1.0, 0.0), fyb = ff ? ffy[Yb] : make_double2(1.0, 0.0);
        for (int zj = 0; zj < nzx; ++zj) {
#pragma unroll
            for (int s = 0; s < E; ++s) {
                const int k = gg + s * G;
                if (k < nkx) {
                    const int X = zj * nkx + (MODE == 0 ? (k + xs) % nkx : k);
                    T a = v[s].x * sc, b = v[s].y * sc;
                    if (MODE == 0 && ff) {
                        a = (T)((double)a * form_factor_sq(ffx[X], fya, ffs));
                        b = (T)((double)b * form_factor_sq(ffx[X], fyb, ffs));
                    }
                    if (hasa) ra[X] = a;
                    if (hasb) rb[X] = b;
                }
            }
        }
    }
}

// ---------------------------------------------------------------- launchers
static inline unsigned cdiv(long a, long b) { return (unsigned)((a + b - 1) / b); }
// n blocks padded for xcd_group with groups of grp
static inline unsigned xcd_grid(unsigned n, int grp) { return cdiv(n, 8L * grp) * 8u * (unsigned)grp; }

hipError_t launch_band(const Plan &pl, const double *d_table, hipStream_t st)
{
    const Geo &g = pl.g;
    const long nk = (long)g.nkx * g.nky;
    if (d_table) return hipMemcpyAsync(pl.xi, d_table, nk * sizeof(double), hipMemcpyDeviceToDevice, st);
    hipLaunchKernelGGL(k_band_tb, dim3(cdiv(nk, kThreads)), dim3(kThreads), 0, st, pl.xi, g.nkx, g.logNx, g.nky,
                       pl.p.t, pl.p.tp, pl.p.tpp, pl.p.k_zones);
    return hipGetLastError();
}

// Occupation of every band (electrons per site: the sum runs over all bands,
// the normalisation over the k points of one).
hipError_t launch_occ(const Plan &pl, double mu, double *d_out2, hipStream_t st)
{
    const long nk = (long)pl.g.nkx * pl.g.nky * pl.g.nkz, nall = nk * pl.nb;
    const int nb = (int)std::min<long>(kOccBlocks, cdiv(nall, kThreads));
    hipLaunchKernelGGL(k_occ_partial, dim3(nb), dim3(kThreads), 0, st, pl.xi, nall, mu, pl.p.gamma, pl.scratch);
    hipLaunchKernelGGL(k_occ_final, dim3(1), dim3(kThreads), 0, st, pl.scratch, nb, nk, d_out2);
    return hipGetLastError();
}

hipError_t launch_xi_shift(const Plan &pl, double mu, hipStream_t st)
{
    const long nall = (long)pl.g.nkx * pl.g.nky * pl.g.nkz * pl.nb;
    hipLaunchKernelGGL(k_xi_shift, dim3(cdiv(nall, kThreads)), dim3(kThreads), 0, st, pl.xi, nall, mu);
    return hipGetLastError();
}

template <typename T>
static hipError_t tables_t(const Plan &pl, hipStream_t st)
{
    const Geo &g = pl.g;
    hipLaunchKernelGGL(k_twiddle<T>, dim3(cdiv(g.nkx, kThreads)), dim3(kThreads), 0, st, (cx<T> *)pl.twx, g.nkx);
    hipLaunchKernelGGL(k_twiddle<T>, dim3(cdiv(g.nky, kThreads)), dim3(kThreads), 0, st, (cx<T> *)pl.twy, g.nky);
    hipLaunchKernelGGL(k_twiddle<T>, dim3(cdiv(g.nkz, kThreads)), dim3(kThreads), 0, st, (cx<T> *)pl.twz, g.nkz);
    hipLaunchKernelGGL(k_twiddle<T>, dim3(cdiv(1 << g.logNE, kThreads)), dim3(kThreads), 0, st, (cx<T> *)pl.twe,
                       1 << g.logNE);
    if (pl.p.ff_kind != LINDHARD_FF_NONE) {
        hipLaunchKernelGGL(k_fftab, dim3(cdiv(pl.out_nx, kThreads)), dim3(kThreads), 0, st, pl.ffx, g.nkx, pl.zx,
                           pl.ff_s, pl.p.k_zones);
        hipLaunchKernelGGL(k_fftab, dim3(cdiv(pl.out_ny, kThreads)), dim3(kThreads), 0, st, pl.ffy, g.nky, pl.zy,
                           pl.ff_s, pl.p.k_zones);
    }
    if (pl.p.want_rpa) {
        const long n = (long)pl.kk_ntiles * 16 * pl.kk_nch * 16;
        hipLaunchKernelGGL(k_kkw, dim3(cdiv(n, kThreads)), dim3(kThreads), 0, st, pl.kkw, pl.d_kkrow, pl.kk_ntiles,
                           pl.kk_nch, g.neps);
    }
    return hipGetLastError();
}

hipError_t launch_tables(const Plan &pl, hipStream_t st)
{
    return pl.g.fp64 ? tables_t<double>(pl, st) : tables_t<float>(pl, st);
}

// Launch helpers with the transform length as a template parameter.
template <typename T, int LOGL>
static void launch_p1(const Plan &pl, cx<T> *spec, int band, int z, int acc, hipStream_t st)
{
    const Geo &g = pl.g;
    using F = RegFFT<T, LOGL, false, ilog2_c(kP1Elems)>;
    const dim3 grid(g.nky / g.p1_R, cdiv(g.nS, g.p1_jc));
    const size_t lds = (size_t)g.p1_R * F::N * sizeof(cx<T>) + tw_lds_bytes<T>(2 * F::N);
    // band `band`, kz plane z of the table; the plane's spectrum at spec
    const size_t nk = (size_t)g.nkx * g.nky * g.nkz, off = band * nk + (size_t)z * g.nkx * g.nky;
    const double *xi = pl.xi + off;
    if (pl.rho)
        hipLaunchKernelGGL((k_p1<T, LOGL, true>), grid, dim3(g.p1_R * F::G), lds, st, xi, g, pl.p.emin, pl.deps,
                           pl.p.gamma, (const cx<T> *)pl.twx, spec, (const T *)pl.rho + off, acc);
    else
        hipLaunchKernelGGL((k_p1<T, LOGL, false>), grid, dim3(g.p1_R * F::G), lds, st, xi, g, pl.p.emin, pl.deps,
                           pl.p.gamma, (const cx<T> *)pl.twx, spec, (const T *)nullptr, acc);
}

template <typename T, int LOGN, bool INV>
static void launch_col(const Plan &pl, cx<T> *spec, int nslices, hipStream_t st)
{
    const Geo &g = pl.g;
    using F = RegFFT<T, LOGN, INV>;
    constexpr int C = sizeof(T) == 4 ? 4 : 2;
    constexpr int TPB = (F::G * C >= 256) ? 1 : 256 / (F::G * C);
    hipLaunchKernelGGL((k_col<T, LOGN, INV>), dim3(cdiv(g.NT * g.nkz, TPB), nslices), dim3(F::G * TPB * C),
                       (size_t)TPB * C * F::N * sizeof(cx<T>) + tw_lds_bytes<T>(F::N), st, spec, g,
                       (const cx<T> *)pl.twy);
}

template <typename T, int LOGN, bool INV>
static void launch_zcol(const Plan &pl, cx<T> *spec, int nslices, hipStream_t st)
{
    const Geo &g = pl.g;
    using F = RegFFT<T, LOGN, INV>;
    constexpr int C = sizeof(T) == 4 ? 4 : 2;
    constexpr int TPB = (F::G * C >= 256) ? 1 : 256 / (F::G * C);
    hipLaunchKernelGGL((k_zcol<T, LOGN, INV>), dim3(cdiv((long)g.NT * g.nky, TPB), nslices), dim3(F::G * TPB * C),
                       (size_t)TPB * C * F::N * sizeof(cx<T>) + tw_lds_bytes<T>(F::N), st, spec, g,
                       (const cx<T> *)pl.twz);
}

template <typename T, int LOGN>
static void launch_p3f(const Plan &pl, cx<T> *spec, hipStream_t st)
{
    const Geo &g = pl.g;
    using F = RegFFT<T, LOGN, false>;
    hipLaunchKernelGGL((k_p3f<T, LOGN>), dim3(g.NT * g.nkz, g.nky / (g.p3f_TR >> g.logC)), dim3(g.p3f_TR * F::G),
                       (size_t)g.p3f_TR * F::N * sizeof(cx<T>) + tw_lds_bytes<T>(F::N), st, spec, g,
                       (const cx<T> *)pl.twe);
}

template <typename T, int LOGL, int MODE>
static void launch_p5(const Plan &pl, const cx<T> *spec, int nplanes, T *out, int onx, int ony, hipStream_t st,
                      const T *m2 = nullptr, int acc = 0)
{
    const Geo &g = pl.g;
    using F = RegFFT<T, LOGL, true>;
    const int ff = pl.p.ff_kind != LINDHARD_FF_NONE;
    // the padded engine: lines, per-pass tables and the L split twiddles
    const size_t lds = row_padded<T, LOGL, 4>()
                           ? row_lds_bytes<T, LOGL, 4>(g.p5_R) + F::N * sizeof(cx<T>)
                           : (size_t)g.p5_R * (F::N + 1) * sizeof(cx<T>) + tw_lds_bytes<T>(2 * F::N);
    hipLaunchKernelGGL((k_p5<T, LOGL, MODE>), dim3(g.nky / g.p5_R, nplanes), dim3(g.p5_R * F::G), lds, st, spec, g,
                       (const cx<T> *)pl.twx, pl.d_src, pl.scale, pl.zx, pl.zy, ff, pl.ff_s, pl.ffx, pl.ffy, out, onx,
                       ony, m2, acc);
}

template <typename T, int LOGNX>
static void launch_e1(const Plan &pl, T *spec, int band, int acc, hipStream_t st)
{
    const Geo &g = pl.g;
    using F = RegFFT<T, LOGNX, false, ilog2_c(e1_elems(LOGNX))>;
    const int np = (g.Hy + 1) / 2;
    const dim3 grid(cdiv(np, g.e1_R), cdiv(g.nS, g.e1_jc));
    const size_t lds = row_lds_bytes<T, LOGNX, ilog2_c(e1_elems(LOGNX))>(g.e1_R);
    const size_t nk = (size_t)g.nkx * g.nky;
    const double *xi = pl.xi + band * nk;
    if (pl.rho)
        hipLaunchKernelGGL((k_e1<T, LOGNX, true>), grid, dim3(g.e1_R * F::G), lds, st, xi, g, pl.p.emin, pl.deps,
                           pl.p.gamma, (const cx<T> *)pl.twx, spec, (const T *)pl.rho + band * nk, acc);
    else
        hipLaunchKernelGGL((k_e1<T, LOGNX, false>), grid, dim3(g.e1_R * F::G), lds, st, xi, g, pl.p.emin,
                           pl.deps, pl.p.gamma, (const cx<T> *)pl.twx, spec, (const T *)nullptr, acc);
}

template <typename T, int LOGN, bool INV>
static void launch_ecol(const Plan &pl, T *spec, int nslices, hipStream_t st)
{
    const Geo &g = pl.g;
    using F = RegFFT<T, LOGN, INV, ilog2_c(kEcolElems)>;
    constexpr int C = sizeof(T) == 4 ? 4 : 2;
    constexpr int TPB = (F::G * C >= 256) ? 1 : 256 / (F::G * C);
    hipLaunchKernelGGL((k_ecol<T, LOGN, INV>), dim3(cdiv(g.NTe, TPB), nslices), dim3(F::G * TPB * C),
                       (size_t)TPB * C * F::N * sizeof(cx<T>) + tw_lds_bytes<T>(F::N), st, spec, g,
                       (const cx<T> *)pl.twy);
}

template <typename T, int LOGNX, int MODE>
static void launch_e5(const Plan &pl, const T *spec, int nplanes, T *out, int onx, int ony, hipStream_t st,
                      const T *m2 = nullptr, int acc = 0)
{
    const Geo &g = pl.g;
    using F = RegFFT<T, LOGNX, true>;
    const int ff = pl.p.ff_kind != LINDHARD_FF_NONE;
    const int np = (g.Hy + 1) / 2;
    const size_t lds = row_lds_bytes<T, LOGNX, 4>(g.e5_R);
    hipLaunchKernelGGL((k_e5<T, LOGNX, MODE>), dim3(cdiv(np, g.e5_R), nplanes), dim3(g.e5_R * F::G), lds, st,
                       spec, g,
                       (const cx<T> *)pl.twx, pl.d_src, pl.scale, pl.zx, pl.zy, ff, pl.ff_s, pl.ffx, pl.ffy, out,
                       onx, ony, m2, acc);
}

#define LH_SWITCH_LOG(v, CALL)                   \
    switch (v) {                                 \
    case 1: CALL(1); break;                      \
    case 2: CALL(2); break;                      \
    case 3: CALL(3); break;                      \
    case 4: CALL(4); break;                      \
    case 5: CALL(5); break;                      \
    case 6: CALL(6); break;                      \
    case 7: CALL(7); break;                      \
    case 8: CALL(8); break;                      \
    case 9: CALL(9); break;                      \
    case 10: CALL(10); break;                    \
    case 11: CALL(11); break;                    \
    default: return hipErrorInvalidValue;        \
    }

// The same for the transform lengths of the k axes (up to 4096 points).
#define LH_SWITCH_LOG12(v, CALL)                 \
    switch (v) {                                 \
    case 12: CALL(12); break;                    \
    default: LH_SWITCH_LOG(v, CALL)              \
    }

#define LH_HIP_TRY(x)                     \
    do {                                  \
        const hipError_t e_ = (x);        \
        if (e_ != hipSuccess) return e_;  \
    } while (0)

template <typename T>
static hipError_t window_t(const Plan &pl, hipStream_t st);

#define LH_SWITCH_LOGM(v, CALL)                  \
    switch (v) {                                 \
    case 3: CALL(3); break;                      \
    case 4: CALL(4); break;                      \
    case 5: CALL(5); break;                      \
    case 6: CALL(6); break;                      \
    case 7: CALL(7); break;                      \
    case 8: CALL(8); break;                      \
    case 9: CALL(9); break;                      \
    case 10: CALL(10); break;                    \
    case 11: CALL(11); break;                    \
    case 12: CALL(12); break;                    \
    case 13: CALL(13); break;                    \
    default: return hipErrorInvalidValue;        \
    }

// dst = a src (overwrite) or dst += a src, n values of T, the arithmetic in T.
template <typename T>
__global__ void __launch_bounds__(kThreads) k_lin(T *__restrict__ dst, const T *__restrict__ src, T a, int overwrite,
                                                 size_t n)
{
    for (size_t i = (size_t)blockIdx.x * kThreads + threadIdx.x; i < n; i += (size_t)gridDim.x * kThreads)
        dst[i] = overwrite ? a * src[i] : dst[i] + a * src[i];
}

template <typename T>
static hipError_t launch_lin(T *dst, const T *src, double a, bool overwrite, size_t n, hipStream_t st)
{
    if (n == 0) return hipSuccess;
    const unsigned blocks = (unsigned)std::min<size_t>((n + kThreads - 1) / kThreads, 8192);
    hipLaunchKernelGGL(k_lin<T>, dim3(blocks), dim3(kThreads), 0, st, dst, src, (T)a, overwrite ? 1 : 0, n);
    return hipGetLastError();
}

static BsTab bs_tab(const Plan &pl, bool y)
{
    void *const *t = y ? pl.bsy : pl.bsx;
    return BsTab{t[0], t[1], t[2], t[3], y ? pl.g.nky : pl.g.nkx};
}

template <typename T, int LOGM>
static void launch_bs_row(const Plan &pl, cx<T> *spec, hipStream_t st)
{
    const Geo &g = pl.g;
    using F = RegFFT<T, LOGM, false>;
    const dim3 grid(xcd_grid(cdiv((g.nky + 1) / 2, g.bs_Rr), g.bs_Rr >= 2 ? 1 : 2), g.nS);
    const size_t lds = (size_t)g.bs_Rr * F::N * sizeof(cx<T>);
    if (pl.rho)
        hipLaunchKernelGGL((k_bs_row<T, LOGM, true>), grid, dim3(g.bs_Rr * F::G), lds, st, pl.xi, g, pl.p.emin,
                           pl.deps, pl.p.gamma, bs_tab(pl, false), spec, (const T *)pl.rho);
    else
        hipLaunchKernelGGL((k_bs_row<T, LOGM, false>), grid, dim3(g.bs_Rr * F::G), lds, st, pl.xi, g, pl.p.emin,
                           pl.deps, pl.p.gamma, bs_tab(pl, false), spec, (const T *)nullptr);
}

template <typename T, int LOGM, bool INV>
static void launch_bs_col(const Plan &pl, cx<T> *spec, int nslices, hipStream_t st)
{
    const Geo &g = pl.g;
    using F = RegFFT<T, LOGM, false>;
    const dim3 grid(xcd_grid(cdiv((long)g.NT * g.C, g.bs_Rc), g.bs_Rc >= g.C ? 1 : g.C / g.bs_Rc),
                    cdiv(nslices, g.bs_SJ));
    const size_t lds = (size_t)(g.bs_Rc + (bs_tw_lds<T, LOGM>() ? 1 : 0)) * F::N * sizeof(cx<T>);
    hipLaunchKernelGGL((k_bs_col<T, LOGM, INV>), grid, dim3(g.bs_Rc * F::G), lds, st, spec, g, bs_tab(pl, true),
                       nslices);
}

template <typename T, int LOGM, int MODE>
static void launch_bs_p5(const Plan &pl, const cx<T> *spec, T *out, hipStream_t st)
{
    const Geo &g = pl.g;
    using F = RegFFT<T, LOGM, false>;
    const dim3 grid(xcd_grid(cdiv((g.nky + 1) / 2, g.bs_Rr), g.bs_Rr >= 2 ? 1 : 2), MODE == 0 ? pl.p.nomega : g.nL);
    const size_t lds = (size_t)(g.bs_Rr + (bs_tw_lds<T, LOGM>() ? 1 : 0)) * F::N * sizeof(cx<T>);
    const int ff = pl.p.ff_kind != LINDHARD_FF_NONE;
    hipLaunchKernelGGL((k_bs_p5<T, LOGM, MODE>), grid, dim3(g.bs_Rr * F::G), lds, st, spec, g, bs_tab(pl, false),
                       pl.d_src, pl.scale, out, pl.zx, pl.zy, ff, pl.ff_s, pl.ffx, pl.ffy);
}

// Grids of any size: Bluestein row and column passes around the same window.
template <typename T>
static hipError_t exec_bs(const Plan &pl, T *out, hipStream_t st, hipEvent_t *ev)
{
    const Geo &g = pl.g;
    cx<T> *spec = (cx<T> *)pl.spec;
    auto mark = [&](int i) {
        if (ev) (void)hipEventRecord(ev[i], st);
    };
    mark(0);
    if (g.nL > 0) {
#define LH_B1(LG) launch_bs_row<T, LG>(pl, spec, st)
        LH_SWITCH_LOGM(g.logMx, LH_B1)
#undef LH_B1
        mark(1);
#define LH_B2(LG) launch_bs_col<T, LG, false>(pl, spec, g.nS, st)
        LH_SWITCH_LOGM(g.logMy, LH_B2)
#undef LH_B2
        mark(2);
        LH_HIP_TRY(window_t<T>(pl, st));
        mark(3);
#define LH_B4(LG) launch_bs_col<T, LG, true>(pl, spec, g.nL, st)
        LH_SWITCH_LOGM(g.logMy, LH_B4)
#undef LH_B4
        mark(4);
    } else {
        mark(1);
        mark(2);
        mark(3);
        mark(4);
    }
    if (pl.p.want_rpa) {
        // the RPA path: first-zone maps of every lag, then the requested planes
        if (g.nL > 0) {
#define LH_B5(LG) launch_bs_p5<T, LG, 1>(pl, spec, (T *)pl.im1, st)
            LH_SWITCH_LOGM(g.logMx, LH_B5)
#undef LH_B5
        }
        const int ff = pl.p.ff_kind != LINDHARD_FF_NONE;
        hipLaunchKernelGGL(k_extend<T>, dim3(cdiv(g.nkx, kThreads), g.nky, cdiv(pl.p.nomega, 4)), dim3(kThreads), 0,
                           st, (const T *)pl.im1, g.nkx, g.nky, 1, g.neps, pl.d_lag, pl.d_frac, pl.p.nomega, pl.zx,
                           pl.zy, ff, pl.ff_s, pl.ffx, pl.ffy, out, pl.out_nx, pl.out_ny);
    } else {
#define LH_B5(LG) launch_bs_p5<T, LG, 0>(pl, spec, out, st)
        LH_SWITCH_LOGM(g.logMx, LH_B5)
#undef LH_B5
    }
    mark(5);
    return hipGetLastError();
}

// ev (optional, 6 events): recorded before P1 and after P1, P2, P3, P4, P5
// (with a band-pair sum, after the forward passes of every band, then at the
// end of the pair loop, which holds P3, P4 and P5 of every pair).
template <typename T>
static hipError_t exec_t(const Plan &pl, T *out, hipStream_t st, hipEvent_t *ev)
{
    const Geo &g = pl.g;
    if (g.bs) return exec_bs<T>(pl, out, st, ev);
    const int ff = pl.p.ff_kind != LINDHARD_FF_NONE;
    auto mark = [&](int i) {
        if (ev) (void)hipEventRecord(ev[i], st);
    };
    const size_t sb = g.even ? g.slice_e * sizeof(T) : g.slice_elems * sizeof(cx<T>);  // bytes per slice
    // P1 of one band into dst (acc: added to what dst holds)
    auto p1 = [&](void *dst, int band, int acc) -> hipError_t {
        if (g.even) {
#define LH_E1(LG) launch_e1<T, LG>(pl, (T *)dst, band, acc, st)
            LH_SWITCH_LOG12(g.logNx, LH_E1)
#undef LH_E1
        } else {
            for (int z = 0; z < g.nkz; ++z) {
                cx<T> *pz = (cx<T> *)dst + (size_t)z * g.plane_elems;
#define LH_P1(LG) launch_p1<T, LG>(pl, pz, band, z, acc, st)
                LH_SWITCH_LOG(g.logL, LH_P1)
#undef LH_P1
            }
        }
        return hipGetLastError();
    };
    // forward (P2) or inverse (P4) column pass over n slices of buf
    auto col = [&](void *buf, int n, bool inv) -> hipError_t {
        if (g.even) {
            if (inv) {
#define LH_E4(LG) launch_ecol<T, LG, true>(pl, (T *)buf, n, st)
                LH_SWITCH_LOG12(g.logNy, LH_E4)
#undef LH_E4
            } else {
#define LH_E2(LG) launch_ecol<T, LG, false>(pl, (T *)buf, n, st)
                LH_SWITCH_LOG12(g.logNy, LH_E2)
#undef LH_E2
            }
        } else {
            if (inv) {
                if (g.nkz > 1) {
#define LH_PZ(LG) launch_zcol<T, LG, true>(pl, (cx<T> *)buf, n, st)
                    LH_SWITCH_LOG(g.logNz, LH_PZ)
#undef LH_PZ
                }
#define LH_P4(LG) launch_col<T, LG, true>(pl, (cx<T> *)buf, n, st)
                LH_SWITCH_LOG12(g.logNy, LH_P4)
#undef LH_P4
            } else {
#define LH_P2(LG) launch_col<T, LG, false>(pl, (cx<T> *)buf, n, st)
                LH_SWITCH_LOG12(g.logNy, LH_P2)
#undef LH_P2
                if (g.nkz > 1) {
#define LH_PZ(LG) launch_zcol<T, LG, false>(pl, (cx<T> *)buf, n, st)
                    LH_SWITCH_LOG(g.logNz, LH_PZ)
#undef LH_PZ
                }
            }
        }
        return hipGetLastError();
    };
    // P5 from the window output in buf; m2: a band pair's |M(Q)|^2 map
    // (acc: the pair adds to the output)
    auto p5 = [&](void *buf, const T *m2 = nullptr, int acc = 0) -> hipError_t {
        const bool rpa = pl.p.want_rpa != 0;
        if (g.even) {
            T *spr = (T *)buf;
            if (rpa) {
#define LH_E5(LG) launch_e5<T, LG, 1>(pl, spr, g.nL, (T *)pl.im1, g.nkx, g.nky, st)
                LH_SWITCH_LOG12(g.logNx, LH_E5)
#undef LH_E5
            } else {
#define LH_E5(LG) launch_e5<T, LG, 0>(pl, spr, pl.p.nomega, out, pl.out_nx, pl.out_ny, st, m2, acc)
                LH_SWITCH_LOG12(g.logNx, LH_E5)
#undef LH_E5
            }
        } else {
            const cx<T> *spec = (const cx<T> *)buf;
            if (rpa) {
                // first-zone planes [lag][kz][ky][kx] (natural order)
                for (int z = 0; z < g.nkz; ++z) {
                    const cx<T> *sz = spec + (size_t)z * g.plane_elems;
                    T *iz = (T *)pl.im1 + (size_t)z * g.nky * g.nkx;
#define LH_P5(LG) launch_p5<T, LG, 1>(pl, sz, g.nL, iz, g.nkx, g.nky * g.nkz, st)
                    LH_SWITCH_LOG(g.logL, LH_P5)
#undef LH_P5
                }
            } else {
                // kz plane z of the spectrum -> output block Z = (z + nkz/2) mod nkz
                // of zones_y * nky rows
                for (int z = 0; z < g.nkz; ++z) {
                    const cx<T> *sz = spec + (size_t)z * g.plane_elems;
                    T *oz = out + (size_t)((z + g.nkz / 2) & (g.nkz - 1)) * pl.zy * g.nky * pl.out_nx;
#define LH_P5(LG) launch_p5<T, LG, 0>(pl, sz, pl.p.nomega, oz, pl.out_nx, pl.out_ny, st, m2, acc)
                    LH_SWITCH_LOG(g.logL, LH_P5)
#undef LH_P5
                }
            }
        }
        return hipGetLastError();
    };
    const size_t plane_out = (size_t)pl.out_nx * pl.out_ny;
    mark(0);
    if (g.nL > 0 && !pl.pairs && !(pl.has_m2 && pl.nb > 1)) {
        for (int b = 0; b < pl.nb; ++b) LH_HIP_TRY(p1(pl.spec, b, b > 0));
        mark(1);
        LH_HIP_TRY(col(pl.spec, g.nS, false));
        mark(2);
        LH_HIP_TRY(window_t<T>(pl, st));
        mark(3);
        LH_HIP_TRY(col(pl.spec, g.nL, true));
        mark(4);
        LH_HIP_TRY(p5(pl.spec, pl.has_m2 ? (const T *)pl.m2 : nullptr, 0));
    } else if (g.nL > 0 && pl.has_m2) {
        // Eqs. (2), (3) with a |M(Q)|^2 map per band pair: the map multiplies
        // after the inverse transforms, so every pair (nu occupied, mu empty)
        // is correlated and transformed back on its own -- the occupied slices
        // of band nu followed by the empty ones of band mu -- and the pairs
        // are summed into the output, in a fixed order
        const size_t nocc = (size_t)(g.j0 - g.jA), nb = (size_t)pl.nb;
        char *bs = (char *)pl.bspec, *sp = (char *)pl.spec;
        for (int b = 0; b < pl.nb; ++b) LH_HIP_TRY(p1(bs + b * g.nS * sb, b, 0));
        mark(1);
        for (int b = 0; b < pl.nb; ++b) LH_HIP_TRY(col(bs + b * g.nS * sb, g.nS, false));
        mark(2);
        const size_t nemp = (size_t)g.nS - nocc;
        for (size_t k = 0; k < pl.m2_pairs.size(); ++k) {
            const size_t nu = (size_t)pl.m2_pairs[k] / nb, mu = (size_t)pl.m2_pairs[k] % nb;
            if (nocc > 0) LH_HIP_TRY(hipMemcpyAsync(sp, bs + nu * g.nS * sb, nocc * sb, hipMemcpyDeviceToDevice, st));
            if (nemp > 0)
                LH_HIP_TRY(hipMemcpyAsync(sp + nocc * sb, bs + (mu * g.nS + nocc) * sb, nemp * sb,
                                          hipMemcpyDeviceToDevice, st));
            LH_HIP_TRY(window_t<T>(pl, st));
            LH_HIP_TRY(col(pl.spec, g.nL, true));
            LH_HIP_TRY(p5(pl.spec, (const T *)pl.m2 + (size_t)pl.m2_pairs[k] * plane_out, k > 0));
        }
        mark(3);
        mark(4);
    } else if (g.nL > 0) {
        // Eq. (2): sum over band pairs (nu occupied, mu empty).  The window
        // pairs occupied slices (energies below j0) with empty ones only and
        // is bilinear in them, so sum_{nu,mu} w S(P_nu, H_mu) =
        // sum_nu S(P_nu, sum_mu w H_mu): for every nu one window of a spliced
        // spectrum -- the occupied slices of band nu followed by the weighted
        // sum of the bands' empty slices -- and the window outputs summed
        // (linear, so one pair of inverse passes serves them all).
        const size_t nocc = (size_t)(g.j0 - g.jA), nb = (size_t)pl.nb;
        const size_t per = sb / sizeof(T);  // T values per slice
        char *bs = (char *)pl.bspec;
        for (int b = 0; b < pl.nb; ++b) LH_HIP_TRY(p1(bs + b * g.nS * sb, b, 0));
        mark(1);
        for (int b = 0; b < pl.nb; ++b) LH_HIP_TRY(col(bs + b * g.nS * sb, g.nS, false));
        mark(2);
        char *sp = (char *)pl.spec;
        const size_t nemp = (size_t)g.nS - nocc;
        int done = 0;
        for (size_t nu = 0; nu < nb; ++nu) {
            int terms = 0;
            for (size_t mu = 0; mu < nb; ++mu) {
                const double w = pl.pairw[nu * nb + mu];
                if (w == 0.0 || nemp == 0) continue;
                LH_HIP_TRY(launch_lin<T>((T *)(sp + nocc * sb), (const T *)(bs + (mu * g.nS + nocc) * sb), w,
                                         terms++ == 0, nemp * per, st));
            }
            if (terms == 0) continue;  // no empty band pairs with nu
            if (nocc > 0) LH_HIP_TRY(hipMemcpyAsync(sp, bs + nu * g.nS * sb, nocc * sb, hipMemcpyDeviceToDevice, st));
            LH_HIP_TRY(window_t<T>(pl, st));
            LH_HIP_TRY(launch_lin<T>((T *)pl.sacc, (const T *)pl.spec, 1.0, done++ == 0, (size_t)g.nL * per, st));
        }
        mark(3);
        LH_HIP_TRY(col(pl.sacc, g.nL, true));
        mark(4);
        LH_HIP_TRY(p5(pl.sacc));
    } else {
        mark(1);
        mark(2);
        mark(3);
        mark(4);
        if (!pl.p.want_rpa) LH_HIP_TRY(p5(pl.spec));  // every plane is zero
    }
    if (pl.p.want_rpa)
        hipLaunchKernelGGL(k_extend<T>, dim3(cdiv(g.nkx, kThreads), g.nky * g.nkz, cdiv(pl.p.nomega, 4)),
                           dim3(kThreads), 0, st, (const T *)pl.im1, g.nkx, g.nky, g.nkz, g.neps, pl.d_lag, pl.d_frac,
                           pl.p.nomega, pl.zx, pl.zy, ff, pl.ff_s, pl.ffx, pl.ffy, out, pl.out_nx, pl.out_ny);
    mark(5);
    return hipGetLastError();
}

// Persistent launch of the matrix-core window: as many blocks as fit on the
// device at once (a multiple of 8, one share per XCD), each walking tiles.
template <typename T, int TR>
static hipError_t launch_e3m(const Plan &pl, T *spr, int ntiles, size_t lds, hipStream_t st)
{
    static std::mutex mu;
    static std::map<std::pair<int, size_t>, int> fit;  // (device, LDS bytes) -> blocks per CU
    int per_cu = 0;
    {
        std::lock_guard<std::mutex> lk(mu);
        auto it = fit.find({pl.device, lds});
        if (it != fit.end()) {
            per_cu = it->second;
        } else {
            LH_HIP_TRY(hipOccupancyMaxActiveBlocksPerMultiprocessor(
                &per_cu, reinterpret_cast<const void *>(&k_e3m<T, TR>), kThreads, lds));
            per_cu = std::max(1, per_cu);
            fit[{pl.device, lds}] = per_cu;
        }
    }
    int ncu = 0;
    LH_HIP_TRY(hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, pl.device));
    const long want = ((long)ntiles + 7) / 8 * 8;
    const int blocks = (int)std::max(8L, std::min(want, (long)ncu * per_cu / 8 * 8));
    hipLaunchKernelGGL((k_e3m<T, TR>), dim3(blocks), dim3(kThreads), lds, st, spr, pl.g, ntiles);
    return hipGetLastError();
}

// The energy-window pass alone (autotuner timing).
template <typename T>
static hipError_t window_t(const Plan &pl, hipStream_t st)
{
    const Geo &g = pl.g;
    if (g.nL == 0) return hipSuccess;
    const size_t cs = sizeof(cx<T>);
    if (g.even) {
        T *spr = (T *)pl.spec;
        const size_t es = sizeof(T);
        const size_t lds3 = (size_t)(g.e3_PL + 16 * (64 >> g.e3_logTR) + 32 + g.m_lo + 16 * ((g.nL + 15) >> 4) - 1) *
                            g.e3_TR * es;
        const dim3 g3(cdiv(g.slice_e, g.e3_TR));
#define LH_E3(TRV)                                                                                    \
    do {                                                                                              \
        if (g.fp64)                                                                                   \
            hipLaunchKernelGGL((k_e3<T, false, TRV>), g3, dim3(kThreads), lds3, st, spr, g);          \
        else                                                                                          \
            hipLaunchKernelGGL((k_e3<T, true, TRV>), g3, dim3(kThreads), lds3, st, spr, g);           \
    } while (0)
        if (g.e3_variant == 2) {
            if constexpr (sizeof(T) == 4) return launch_e3q(pl, g.e3q_W, st);
            return hipErrorInvalidValue;
        }
        if (g.e3_variant == 1) {
            const size_t tile = (size_t)256 * (g.e3m_TR + 1), stage = (size_t)g.e3m_TR * g.e3m_PS;
            const size_t ldsm = (g.e3m_NMG == 1 ? std::max(tile, stage) : tile + stage) * es;
            const int ntiles = (int)cdiv(g.slice_e, g.e3m_TR);
            switch (g.e3m_TR) {
            case 32: return launch_e3m<T, 32>(pl, spr, ntiles, ldsm, st);
            case 16: return launch_e3m<T, 16>(pl, spr, ntiles, ldsm, st);
            case 8: return launch_e3m<T, 8>(pl, spr, ntiles, ldsm, st);
            default: return launch_e3m<T, 4>(pl, spr, ntiles, ldsm, st);
            }
        }
        switch (g.e3_TR) {
        case 64: LH_E3(64); break;
        case 32: LH_E3(32); break;
        case 16: LH_E3(16); break;
        case 8: LH_E3(8); break;
        case 4: LH_E3(4); break;
        case 2: LH_E3(2); break;
        default: LH_E3(1); break;
        }
#undef LH_E3
        return hipGetLastError();
    }
    cx<T> *spec = (cx<T> *)pl.spec;
    if (g.p3_variant == 1) {
#define LH_P3F(LG) launch_p3f<T, LG>(pl, spec, st)
        LH_SWITCH_LOG(g.logNE, LH_P3F)
#undef LH_P3F
    } else if (g.fp64) {
        hipLaunchKernelGGL((k_p3<T, false>), dim3(g.NT * g.nkz, g.nky / g.p3_RY), dim3(kThreads), (size_t)g.nS * g.p3_TR * cs,
                           st, spec, g);
    } else {
        hipLaunchKernelGGL((k_p3<T, true>), dim3(g.NT * g.nkz, g.nky / g.p3_RY), dim3(kThreads), (size_t)g.nS * g.p3_TR * cs,
                           st, spec, g);
    }
    return hipGetLastError();
}

// ------------------------------------------------------------ batched even path
std::string even_group_key(const Plan &pl)
{
    const Geo &g = pl.g;
    if (!g.even || g.bs || g.nkz > 1 || pl.nb > 1 || pl.pairs || pl.has_m2 || pl.p.want_rpa || g.nL == 0 ||
        g.e3_variant == 1)
        return std::string();
    char b[96];
    std::snprintf(b, sizeof b, "e%d %d %d r%d w%d %d", g.fp64, g.logNx, g.logNy, pl.rho ? 1 : 0, g.e3_variant,
                  g.e3_variant == 2 ? 16 : g.e3_TR);
    return b;
}

void even_group_fill(const Plan &pl, void *out, EvenInst &d)
{
    d.g = pl.g;
    d.xi = pl.xi;
    d.rho = pl.rho;
    d.twx = pl.twx;
    d.twy = pl.twy;
    d.spec = pl.spec;
    d.psrc = pl.d_src;
    d.out = out;
    d.ffx = pl.ffx;
    d.ffy = pl.ffy;
    d.emin = pl.p.emin;
    d.deps = pl.deps;
    d.gamma = pl.p.gamma;
    d.scale = pl.scale;
    d.ffs = pl.ff_s;
    d.zx = pl.zx;
    d.zy = pl.zy;
    d.ff = pl.p.ff_kind != LINDHARD_FF_NONE;
    d.onx = pl.out_nx;
    d.ony = pl.out_ny;
    d.nomega = pl.p.nomega;
}

// The five passes of a group of even-path instances (equal group keys), each
// one launch over all of them: grids cover the largest instance and blocks
// past an instance's own extent return at once.
template <typename T>
static hipError_t even_group_t(const Plan *const *pls, int n, const EvenInst *d, hipStream_t st)
{
    const Geo &g = pls[0]->g;
    int ys1 = 0, nS = 0, nL = 0, nw = 0;
    size_t lds3 = 0;
    for (int i = 0; i < n; ++i) {
        const Geo &gi = pls[i]->g;
        ys1 = std::max(ys1, (int)cdiv(gi.nS, gi.e1_jc));
        nS = std::max(nS, gi.nS);
        nL = std::max(nL, gi.nL);
        nw = std::max(nw, pls[i]->p.nomega);
        lds3 = std::max(lds3, (size_t)(gi.e3_PL + 16 * (64 >> gi.e3_logTR) + 32 + gi.m_lo + 16 * ((gi.nL + 15) >> 4) - 1) *
                                  gi.e3_TR * sizeof(T));
    }
    const unsigned nz = (unsigned)n;
    const int np = (g.Hy + 1) / 2;
    const bool rho = pls[0]->rho != nullptr;
    // P1
#define LH_E1B(LG)                                                                                                  \
    do {                                                                                                            \
        using F = RegFFT<T, LG, false, ilog2_c(e1_elems(LG))>;                                                     \
        const size_t lds = row_lds_bytes<T, LG, ilog2_c(e1_elems(LG))>(g.e1_R);                                    \
        const dim3 grid(cdiv(np, g.e1_R), ys1, nz);                                                                 \
        if (rho)                                                                                                    \
            hipLaunchKernelGGL((k_e1_batch<T, LG, true>), grid, dim3(g.e1_R * F::G), lds, st, d);                   \
        else                                                                                                        \
            hipLaunchKernelGGL((k_e1_batch<T, LG, false>), grid, dim3(g.e1_R * F::G), lds, st, d);                  \
    } while (0)
    LH_SWITCH_LOG12(g.logNx, LH_E1B)
#undef LH_E1B
    // P2 / P4
    auto col = [&](int ns, bool inv) -> hipError_t {
#define LH_ECB(LG)                                                                                                  \
    do {                                                                                                            \
        using F = RegFFT<T, LG, false, ilog2_c(kEcolElems)>;                                                       \
        constexpr int C = sizeof(T) == 4 ? 4 : 2;                                                                   \
        constexpr int TPB = (F::G * C >= 256) ? 1 : 256 / (F::G * C);                                               \
        const dim3 grid(cdiv(g.NTe, TPB), ns, nz);                                                                  \
        const size_t lds = (size_t)TPB * C * F::N * sizeof(cx<T>) + tw_lds_bytes<T>(F::N);                         \
        if (inv)                                                                                                    \
            hipLaunchKernelGGL((k_ecol_batch<T, LG, true>), grid, dim3(F::G * TPB * C), lds, st, d);                \
        else                                                                                                        \
            hipLaunchKernelGGL((k_ecol_batch<T, LG, false>), grid, dim3(F::G * TPB * C), lds, st, d);               \
    } while (0)
        LH_SWITCH_LOG12(g.logNy, LH_ECB)
#undef LH_ECB
        return hipGetLastError();
    };
    LH_HIP_TRY(col(nS, false));
    // P3
    if (g.e3_variant == 2) {
        if constexpr (sizeof(T) == 4) {
            LH_HIP_TRY(launch_e3q_group(pls, n, d, st));
        } else {
            return hipErrorInvalidValue;
        }
    } else {
        const dim3 g3(cdiv(g.slice_e, g.e3_TR), 1, nz);
#define LH_E3B(TRV)                                                                                                 \
    do {                                                                                                            \
        if (g.fp64)                                                                                                 \
            hipLaunchKernelGGL((k_e3_batch<T, false, TRV>), g3, dim3(kThreads), lds3, st, d);                       \
        else                                                                                                        \
            hipLaunchKernelGGL((k_e3_batch<T, true, TRV>), g3, dim3(kThreads), lds3, st, d);                        \
    } while (0)
        switch (g.e3_TR) {
        case 64: LH_E3B(64); break;
        case 32: LH_E3B(32); break;
        case 16: LH_E3B(16); break;
        case 8: LH_E3B(8); break;
        case 4: LH_E3B(4); break;
        case 2: LH_E3B(2); break;
        default: LH_E3B(1); break;
        }
#undef LH_E3B
        LH_HIP_TRY(hipGetLastError());
    }
    LH_HIP_TRY(col(nL, true));
    // P5
#define LH_E5B(LG)                                                                                                  \
    do {                                                                                                            \
        using F = RegFFT<T, LG, true>;                                                                              \
        const dim3 grid(cdiv(np, g.e5_R), nw, nz);                                                                  \
        const size_t lds = row_lds_bytes<T, LG, 4>(g.e5_R);                                                         \
        hipLaunchKernelGGL((k_e5_batch<T, LG, 0>), grid, dim3(g.e5_R * F::G), lds, st, d);                          \
    } while (0)
    LH_SWITCH_LOG12(g.logNx, LH_E5B)
#undef LH_E5B
    return hipGetLastError();
}

hipError_t launch_even_group(const Plan *const *pls, int n, const EvenInst *d_desc, hipStream_t st)
{
    return pls[0]->g.fp64 ? even_group_t<double>(pls, n, d_desc, st) : even_group_t<float>(pls, n, d_desc, st);
}

hipError_t launch_window(const Plan &pl, hipStream_t st)
{
    return pl.g.fp64 ? window_t<double>(pl, st) : window_t<float>(pl, st);
}

hipError_t launch_exec(const Plan &pl, void *out, hipStream_t st, hipEvent_t *ev)
{
    return pl.g.fp64 ? exec_t<double>(pl, (double *)out, st, ev) : exec_t<float>(pl, (float *)out, st, ev);
}

template <typename T>
static hipError_t rpa_t(const Plan &pl, int vkind, double U, T *re, T *imr, T *rer, hipStream_t st)
{
    const Geo &g = pl.g;
    const int nk = g.nkx * g.nky * g.nkz;
    if (pl.kk_ntiles > 4)
        hipLaunchKernelGGL((k_kkm<T, 8>), dim3(cdiv(nk, kKkQ), cdiv(pl.kk_ntiles, 8)), dim3(512), 0, st,
                           (const T *)pl.im1, nk, g.neps, pl.kkw, pl.d_kkrow, pl.kk_ntiles, pl.kk_nch, (T *)pl.re1);
    else
        hipLaunchKernelGGL((k_kkm<T, 4>), dim3(cdiv(nk, kKkQ), 1), dim3(256), 0, st, (const T *)pl.im1, nk, g.neps,
                           pl.kkw, pl.d_kkrow, pl.kk_ntiles, pl.kk_nch, (T *)pl.re1);
    const int ff = pl.p.ff_kind != LINDHARD_FF_NONE;
    hipLaunchKernelGGL(k_rpa<T>, dim3(cdiv(g.nkx, kThreads), g.nky * g.nkz, cdiv(pl.p.nomega, 4)), dim3(kThreads), 0,
                       st, (const T *)pl.im1, (const T *)pl.re1, g.nkx, g.nky, g.neps, pl.d_lag, pl.d_frac,
                       pl.d_kkslot, pl.p.nomega, pl.zx, pl.zy, ff, pl.ff_s, pl.ffx, pl.ffy, vkind, U, pl.p.k_zones, re,
                       imr, rer, pl.out_nx, pl.out_ny, g.nkz);
    return hipGetLastError();
}

hipError_t launch_rpa(const Plan &pl, int vkind, double U, void *re, void *imr, void *rer, hipStream_t st)
{
    return pl.g.fp64 ? rpa_t<double>(pl, vkind, U, (double *)re, (double *)imr, (double *)rer, st)
                     : rpa_t<float>(pl, vkind, U, (float *)re, (float *)imr, (float *)rer, st);
}

template <typename T>
static hipError_t sqw_t(const Plan &pl, double kT, const T *im, T *s, hipStream_t st)
{
    const size_t plane = (size_t)pl.out_nx * pl.out_ny;
    constexpr int VEC = 16 / sizeof(T);
    const bool vec = plane % VEC == 0 && ((reinterpret_cast<uintptr_t>(im) | reinterpret_cast<uintptr_t>(s)) & 15) == 0;
    const size_t n = vec ? plane / VEC : plane;
    const dim3 grid((unsigned)std::min<size_t>(cdiv(n, kThreads), 4096), pl.p.nomega);
    if (vec)
        hipLaunchKernelGGL((k_sqw<T, VEC>), grid, dim3(kThreads), 0, st, im, s, pl.d_lag, pl.d_frac, pl.deps, kT, plane);
    else
        hipLaunchKernelGGL((k_sqw<T, 1>), grid, dim3(kThreads), 0, st, im, s, pl.d_lag, pl.d_frac, pl.deps, kT, plane);
    return hipGetLastError();
}

hipError_t launch_sqw(const Plan &pl, double kT, const void *im, void *s, hipStream_t st)
{
    return pl.g.fp64 ? sqw_t<double>(pl, kT, (const double *)im, (double *)s, st)
                     : sqw_t<float>(pl, kT, (const float *)im, (float *)s, st);
}

hipError_t launch_qavg_raw(const void *im, bool fp64, size_t plane, int nw, double *part, double *out,
                           hipStream_t st)
{
    const dim3 grid(kQavgBlocks, nw);
    if (fp64)
        hipLaunchKernelGGL(k_qavg_part<double>, grid, dim3(kThreads), 0, st, (const double *)im, plane, part);
    else
        hipLaunchKernelGGL(k_qavg_part<float>, grid, dim3(kThreads), 0, st, (const float *)im, plane, part);
    hipLaunchKernelGGL(k_qavg_final, dim3(cdiv(nw, kThreads)), dim3(kThreads), 0, st, part, nw, 1.0 / (double)plane,
                       out);
    return hipGetLastError();
}

hipError_t launch_qavg(const Plan &pl, const void *im, double *out, hipStream_t st)
{
    return launch_qavg_raw(im, pl.g.fp64 != 0, (size_t)pl.out_nx * pl.out_ny, pl.p.nomega, pl.scratch, out, st);
}

hipError_t launch_peak(const Plan &pl, const void *im, int32_t *idx, hipStream_t st)
{
    const size_t plane = (size_t)pl.out_nx * pl.out_ny;
    const dim3 grid((unsigned)cdiv(plane, kThreads));
    if (pl.g.fp64)
        hipLaunchKernelGGL(k_peak<double>, grid, dim3(kThreads), 0, st, (const double *)im, idx, plane, pl.p.nomega);
    else
        hipLaunchKernelGGL(k_peak<float>, grid, dim3(kThreads), 0, st, (const float *)im, idx, plane, pl.p.nomega);
    return hipGetLastError();
}

hipError_t launch_cut(const Plan &pl, const void *im, const int *xy, int npts, void *out, hipStream_t st)
{
    const size_t plane = (size_t)pl.out_nx * pl.out_ny;
    const dim3 grid(cdiv(npts, kThreads), pl.p.nomega);
    if (pl.g.fp64)
        hipLaunchKernelGGL(k_cut<double>, grid, dim3(kThreads), 0, st, (const double *)im, plane, pl.out_nx, xy, npts,
                           (double *)out);
    else
        hipLaunchKernelGGL(k_cut<float>, grid, dim3(kThreads), 0, st, (const float *)im, plane, pl.out_nx, xy, npts,
                           (float *)out);
    return hipGetLastError();
}

hipError_t launch_envelope(const Plan &pl, const void *im_plane, int dir, int W, int nseg, double qstep, double *res,
                           hipStream_t st)
{
    const int Xc = pl.out_nx / 2, Yc = pl.out_ny / 2, nk = W;
    if (pl.g.fp64)
        hipLaunchKernelGGL(k_envelope<double>, dim3(1), dim3(kThreads), 0, st, (const double *)im_plane, pl.out_nx, Xc,
                           Yc, nk, dir, nseg, qstep, res);
    else
        hipLaunchKernelGGL(k_envelope<float>, dim3(1), dim3(kThreads), 0, st, (const float *)im_plane, pl.out_nx, Xc,
                           Yc, nk, dir, nseg, qstep, res);
    return hipGetLastError();
}

}  // namespace lh
