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

namespace lh {

constexpr double kPi = 3.14159265358979323846;
constexpr int kThreads = 256;

// ---------------------------------------------------------------- setup
__global__ void __launch_bounds__(kThreads) k_band_tb(double *__restrict__ eps, int nkx, int logNx, int nky,
                                                     double t, double tp, double tpp)
{
    const long nk = (long)nkx * nky;
    const long k = (long)blockIdx.x * kThreads + threadIdx.x;
    if (k >= nk) return;
    const int ix = (int)(k & (nkx - 1));
    const int iy = (int)(k >> logNx);
    const double cx = cospi(2.0 * ix / nkx), cy = cospi(2.0 * iy / nky);
    const double c2x = cospi(4.0 * ix / nkx), c2y = cospi(4.0 * iy / nky);
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

// Per extended column (or row) X: (exp(-s Q^2), Q^2), Q = 2 pi (X - zones n/2)/n.
__global__ void __launch_bounds__(kThreads) k_fftab(double2 *__restrict__ tab, int n, int zones, double s)
{
    const int X = blockIdx.x * kThreads + threadIdx.x;
    if (X >= n * zones) return;
    const double h = (double)(X - (zones * n) / 2) / (double)n;
    const double Q = 2.0 * kPi * h;
    const double Q2 = Q * Q;
    tab[X] = make_double2(exp(-s * Q2), Q2);
}

// Kramers-Kronig weights of the alternate-point rule (Sec. 4):
// w[i][j] = (2/pi) 2j / (j^2 - i^2) for j - i odd, 1 <= j < neps, else 0.
__global__ void __launch_bounds__(kThreads) k_kkw(double *__restrict__ w, const int *__restrict__ lags, int nw,
                                                 int neps)
{
    const long idx = (long)blockIdx.x * kThreads + threadIdx.x;
    if (idx >= (long)nw * neps) return;
    const int wi = (int)(idx / neps), j = (int)(idx % neps);
    const double i = (double)lags[wi];
    double v = 0.0;
    if (j >= 1 && (((long)j - (long)lags[wi]) & 1)) {
        const double dj = (double)j;
        v = (2.0 / kPi) * 2.0 * dj / (dj * dj - i * i);
    }
    w[idx] = v;
}

// |M(Q)|^2 = F(Q)^2 at extended (X, Y), Eq. (3) for the Gaussian d orbital.
__device__ __forceinline__ double form_factor_sq(const double2 fx, const double2 fy, double s)
{
    const double q2 = fx.y + fy.y;
    const double dq = fx.y - fy.y;
    const double F = fx.x * fy.x * (1.0 - 2.0 * s * q2 + s * s * dq * dq);
    return F * F;
}

// ---------------------------------------------------------------- P1
// One block: R rows (ky) of the spectral function for jc consecutive energy
// slices.  Row kx of length nkx is packed as z[n] = A(2n) + i A(2n+1), FFT of
// length L = nkx/2, then split into X[k], k = 0..L (real-to-complex).
// e_j - xi_k is formed in FP64; the Lorentzian and the transform run in T.
template <typename T>
__global__ void __launch_bounds__(kThreads) k_p1(const double *__restrict__ xi, Geo g, double emin, double deps,
                                                double gamma, const cx<T> *__restrict__ twx,
                                                cx<T> *__restrict__ spec)
{
    extern __shared__ __align__(16) unsigned char smem_raw[];
    cx<T> *buf = reinterpret_cast<cx<T> *>(smem_raw);
    const int R = g.p1_R, logR = g.p1_logR, L = g.L, logL = g.logL;
    const int items = R << logL;
    const int tid = threadIdx.x;
    const int ky0 = blockIdx.x * R;
    const int jbeg = g.jA + blockIdx.y * g.p1_jc;
    const int jend = min(g.jB, jbeg + g.p1_jc);

    double xa[16], xb[16];
#pragma unroll
    for (int q = 0; q < 16; ++q) {
        const int it = tid + q * kThreads;
        xa[q] = 0.0;
        xb[q] = 0.0;
        if (it < items) {
            const int row = it & (R - 1), n = it >> logR;
            const double *xr = xi + (size_t)(ky0 + row) * g.nkx;
            xa[q] = xr[2 * n];
            xb[q] = xr[2 * n + 1];
        }
    }
    const T gp = (T)(gamma / kPi), g2 = (T)(gamma * gamma);
    const int C = g.C, logC = g.logC;
    const int nout = g.NT * (R << logC);

    for (int j = jbeg; j < jend; ++j) {
        const double ej = emin + (j + 0.5) * deps;
#pragma unroll
        for (int q = 0; q < 16; ++q) {
            const int it = tid + q * kThreads;
            if (it < items) {
                const T d0 = (T)(ej - xa[q]), d1 = (T)(ej - xb[q]);
                buf[it] = mk<T>(gp / (d0 * d0 + g2), gp / (d1 * d1 + g2));
            }
        }
        __syncthreads();
        fft_dif_lds<T, false>(buf, logL, logR, twx, g.logNx, tid, kThreads);
        cx<T> *dst = spec + (size_t)(j - g.jA) * g.slice_elems;
        for (int it = tid; it < nout; it += kThreads) {
            const int c = it & (C - 1);
            const int row = (it >> logC) & (R - 1);
            const int tile = it >> (logC + logR);
            const int k = tile * C + c;
            cx<T> X = mk<T>((T)0, (T)0);
            if (k <= L) {
                const cx<T> Zk = buf[dif_pos(k & (L - 1), logL) * R + row];
                const cx<T> ZL = cconj(buf[dif_pos((L - k) & (L - 1), logL) * R + row]);
                const cx<T> E = cscale(cadd(Zk, ZL), (T)0.5);
                const cx<T> D = cscale(csub(Zk, ZL), (T)0.5);
                const cx<T> w = twx[k];
                X = cadd(E, cmul(mk<T>(w.y, -w.x), D));
            }
            dst[((size_t)tile * g.nky + ky0 + row) * C + c] = X;
        }
        __syncthreads();
    }
}

// ---------------------------------------------------------------- P2 / P4
// One block: one column tile (C columns, all nky rows) of one slice, which is
// one contiguous block of memory; transformed in place.
template <typename T, bool INV>
__global__ void __launch_bounds__(kThreads) k_col(cx<T> *__restrict__ spec, Geo g,
                                                 const cx<T> *__restrict__ twy)
{
    extern __shared__ __align__(16) unsigned char smem_raw[];
    cx<T> *buf = reinterpret_cast<cx<T> *>(smem_raw);
    const int tid = threadIdx.x;
    const int n = g.nky << g.logC;
    cx<T> *src = spec + (size_t)blockIdx.y * g.slice_elems + (size_t)blockIdx.x * n;
    for (int it = tid; it < n; it += kThreads) buf[it] = src[it];
    __syncthreads();
    fft_dif_lds<T, INV>(buf, g.logNy, g.logC, twy, g.logNy, tid, kThreads);
    const int C = g.C, logC = g.logC;
    for (int it = tid; it < n; it += kThreads) {
        const int ry = it >> logC, c = it & (C - 1);
        src[it] = buf[(dif_pos(ry, g.logNy) << logC) + c];
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
    for (int it = tid; it < (ne << logTR); it += kThreads) {
        const int s = it >> logTR, rp = it & (TR - 1);
        buf[it] = spec[(size_t)s * g.slice_elems + off + rp];
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

// ---------------------------------------------------------------- P5
// One block: R rows (qy) of one output plane.  Complex-to-real inverse over rx
// from the half spectrum X[0..L]: Z'[k] = (X[k] + X*[L-k]) + i e^{+2 pi i k/nkx}
// (X[k] - X*[L-k]), inverse FFT of length L gives x[2n] + i x[2n+1] (no 1/N).
// MODE 0: plane = requested omega; writes the extended, form-factor weighted
//         map out[plane][Y][X] (zeros for an empty window).
// MODE 1: plane = window slot; writes the first-zone map out[m][qy][qx].
template <typename T, int MODE>
__global__ void __launch_bounds__(kThreads) k_p5(const cx<T> *__restrict__ spec, Geo g,
                                                const cx<T> *__restrict__ twx, const int *__restrict__ plane_slot,
                                                double scale, int zx, int zy, int ff, double ffs,
                                                const double2 *__restrict__ ffx, const double2 *__restrict__ ffy,
                                                T *__restrict__ out, int out_nx, int out_ny)
{
    extern __shared__ __align__(16) unsigned char smem_raw[];
    const int R = g.p5_R, logR = g.p5_logR, L = g.L, logL = g.logL;
    cx<T> *xb = reinterpret_cast<cx<T> *>(smem_raw);  // [(L+1)][R]
    cx<T> *zb = xb + (size_t)(L + 1) * R;              // [L][R]
    const int tid = threadIdx.x;
    const int plane = blockIdx.y;
    const int qy0 = blockIdx.x * R;
    const int slot = MODE == 0 ? plane_slot[plane] : plane;
    const int nkx = g.nkx, nky = g.nky;

    if (MODE == 0 && slot < 0) {
        for (int rz = 0; rz < R * zy; ++rz) {
            const int row = rz % R, zi = rz / R;
            const int Y = zi * nky + ((qy0 + row + zy * nky / 2) & (nky - 1));
            T *orow = out + ((size_t)plane * out_ny + Y) * out_nx;
            for (int X = tid; X < out_nx; X += kThreads) orow[X] = (T)0;
        }
        return;
    }

    const int C = g.C, logC = g.logC;
    const cx<T> *src = spec + (size_t)slot * g.slice_elems;
    const int nin = g.NT * (R << logC);
    for (int it = tid; it < nin; it += kThreads) {
        const int c = it & (C - 1);
        const int row = (it >> logC) & (R - 1);
        const int tile = it >> (logC + logR);
        const int k = tile * C + c;
        if (k <= L) xb[k * R + row] = src[((size_t)tile * nky + qy0 + row) * C + c];
    }
    __syncthreads();
    for (int it = tid; it < (L << logR); it += kThreads) {
        const int row = it & (R - 1), k = it >> logR;
        const cx<T> Xk = xb[k * R + row];
        const cx<T> XL = cconj(xb[(L - k) * R + row]);
        const cx<T> A = cadd(Xk, XL);
        const cx<T> D = csub(Xk, XL);
        const cx<T> w = cconj(twx[k]);  // e^{+2 pi i k / nkx}
        const cx<T> wD = cmul(w, D);
        zb[it] = cadd(A, mk<T>(-wD.y, wD.x));  // A + i w D
    }
    __syncthreads();
    fft_dif_lds<T, true>(zb, logL, logR, twx, g.logNx, tid, kThreads);

    const T sc = (T)scale;
    if (MODE == 0) {
        for (int rz = 0; rz < R * zy; ++rz) {
            const int row = rz % R, zi = rz / R;
            const int Y = zi * nky + ((qy0 + row + zy * nky / 2) & (nky - 1));
            T *orow = out + ((size_t)plane * out_ny + Y) * out_nx;
            const double2 fy = ff ? ffy[Y] : make_double2(1.0, 0.0);
            for (int X = tid; X < out_nx; X += kThreads) {
                const int u = (X - (zx * nkx) / 2) & (nkx - 1);
                const cx<T> v = zb[dif_pos(u >> 1, logL) * R + row];
                T val = ((u & 1) ? v.y : v.x) * sc;
                if (ff) val = (T)((double)val * form_factor_sq(ffx[X], fy, ffs));
                orow[X] = val;
            }
        }
    } else {
        const int m = g.m_lo + slot;
        for (int row = 0; row < R; ++row) {
            T *orow = out + ((size_t)m * nky + qy0 + row) * nkx;
            for (int u = tid; u < nkx; u += kThreads) {
                const cx<T> v = zb[dif_pos(u >> 1, logL) * R + row];
                orow[u] = ((u & 1) ? v.y : v.x) * sc;
            }
        }
    }
}

// Extended, form-factor weighted map from the first-zone planes (RPA path).
template <typename T>
__global__ void __launch_bounds__(kThreads) k_extend(const T *__restrict__ im1, int nkx, int nky, int neps,
                                                    const int *__restrict__ lags, int zx, int zy, int ff,
                                                    double ffs, const double2 *__restrict__ ffx,
                                                    const double2 *__restrict__ ffy, T *__restrict__ out,
                                                    int out_nx, int out_ny)
{
    const int X = blockIdx.x * kThreads + threadIdx.x;
    const int Y = blockIdx.y;
    const int w = blockIdx.z;
    if (X >= out_nx) return;
    const int m = lags[w];
    const int u = (X - (zx * nkx) / 2) & (nkx - 1);
    const int v = (Y - (zy * nky) / 2) & (nky - 1);
    T val = (T)0;
    if (m >= 1 && m < neps) {
        val = im1[((size_t)m * nky + v) * nkx + u];
        if (ff) val = (T)((double)val * form_factor_sq(ffx[X], ffy[Y], ffs));
    }
    out[((size_t)w * out_ny + Y) * out_nx + X] = val;
}

// Kramers-Kronig: re1[w][q] = sum_j kkw[w][j] im1[j][q], FP64 accumulation.
// One block: QT consecutive q with every lag staged in LDS.
template <typename T>
__global__ void __launch_bounds__(kThreads) k_kk(const T *__restrict__ im1, int nk, int neps, int nw,
                                                const int *__restrict__ lags, const double *__restrict__ kkw,
                                                T *__restrict__ re1, int logQT)
{
    extern __shared__ __align__(16) unsigned char smem_raw[];
    T *tile = reinterpret_cast<T *>(smem_raw);
    const int QT = 1 << logQT;
    const int tid = threadIdx.x;
    const int q0 = blockIdx.x * QT;
    for (int it = tid; it < neps * QT; it += kThreads) {
        const int j = it >> logQT, c = it & (QT - 1);
        tile[it] = im1[(size_t)j * nk + q0 + c];
    }
    __syncthreads();
    const int c = tid & (QT - 1);
    const int grp = tid >> logQT, ngrp = kThreads >> logQT;
    for (int w = grp; w < nw; w += ngrp) {
        const double *kw = kkw + (size_t)w * neps;
        const int js = (lags[w] & 1) ? 2 : 1;
        double acc = 0.0;
        for (int j = js; j < neps; j += 2) acc += kw[j] * (double)tile[(j << logQT) + c];
        re1[(size_t)w * nk + q0 + c] = (T)acc;
    }
}

// RPA epilogue on the extended map: chi = |M|^2 (Re + i Im),
// chi_RPA = chi / (1 - U chi), FP64 arithmetic, rounded once to T.
template <typename T>
__global__ void __launch_bounds__(kThreads) k_rpa(const T *__restrict__ im1, const T *__restrict__ re1, int nkx,
                                                 int nky, int neps, const int *__restrict__ lags, int zx, int zy,
                                                 int ff, double ffs, const double2 *__restrict__ ffx,
                                                 const double2 *__restrict__ ffy, double U, T *__restrict__ re_out,
                                                 T *__restrict__ imr, T *__restrict__ rer, int out_nx, int out_ny)
{
    const int X = blockIdx.x * kThreads + threadIdx.x;
    const int Y = blockIdx.y;
    const int w = blockIdx.z;
    if (X >= out_nx) return;
    const int m = lags[w];
    const int u = (X - (zx * nkx) / 2) & (nkx - 1);
    const int v = (Y - (zy * nky) / 2) & (nky - 1);
    const size_t q = (size_t)v * nkx + u;
    const size_t nk = (size_t)nkx * nky;
    double im = (m >= 1 && m < neps) ? (double)im1[(size_t)m * nk + q] : 0.0;
    double re = (double)re1[(size_t)w * nk + q];
    if (ff) {
        const double m2 = form_factor_sq(ffx[X], ffy[Y], ffs);
        im = (double)(T)(im * m2);
        re = (double)(T)(re * m2);
    }
    const double a = 1.0 - U * re, b = U * im;
    const double D = a * a + b * b;
    const size_t o = ((size_t)w * out_ny + Y) * out_nx + X;
    if (re_out) re_out[o] = (T)re;
    if (imr) imr[o] = (T)(im / D);
    if (rer) rer[o] = (T)((re * a - U * im * im) / D);
}

// ---------------------------------------------------------------- launchers
static inline unsigned cdiv(long a, long b) { return (unsigned)((a + b - 1) / b); }

hipError_t launch_band(const Plan &pl, const double *d_table, hipStream_t st)
{
    const Geo &g = pl.g;
    const long nk = (long)g.nkx * g.nky;
    if (d_table) return hipMemcpyAsync(pl.xi, d_table, nk * sizeof(double), hipMemcpyDeviceToDevice, st);
    hipLaunchKernelGGL(k_band_tb, dim3(cdiv(nk, kThreads)), dim3(kThreads), 0, st, pl.xi, g.nkx, g.logNx, g.nky,
                       pl.p.t, pl.p.tp, pl.p.tpp);
    return hipGetLastError();
}

hipError_t launch_occ(const Plan &pl, double mu, double *d_out2, hipStream_t st)
{
    const long nk = (long)pl.g.nkx * pl.g.nky;
    const int nb = (int)std::min<long>(kOccBlocks, cdiv(nk, kThreads));
    hipLaunchKernelGGL(k_occ_partial, dim3(nb), dim3(kThreads), 0, st, pl.xi, nk, mu, pl.p.gamma, pl.scratch);
    hipLaunchKernelGGL(k_occ_final, dim3(1), dim3(kThreads), 0, st, pl.scratch, nb, nk, d_out2);
    return hipGetLastError();
}

hipError_t launch_xi_shift(const Plan &pl, double mu, hipStream_t st)
{
    const long nk = (long)pl.g.nkx * pl.g.nky;
    hipLaunchKernelGGL(k_xi_shift, dim3(cdiv(nk, kThreads)), dim3(kThreads), 0, st, pl.xi, nk, mu);
    return hipGetLastError();
}

template <typename T>
static hipError_t tables_t(const Plan &pl, hipStream_t st)
{
    const Geo &g = pl.g;
    hipLaunchKernelGGL(k_twiddle<T>, dim3(cdiv(g.nkx, kThreads)), dim3(kThreads), 0, st, (cx<T> *)pl.twx, g.nkx);
    hipLaunchKernelGGL(k_twiddle<T>, dim3(cdiv(g.nky, kThreads)), dim3(kThreads), 0, st, (cx<T> *)pl.twy, g.nky);
    if (pl.p.ff_kind != LINDHARD_FF_NONE) {
        hipLaunchKernelGGL(k_fftab, dim3(cdiv(pl.out_nx, kThreads)), dim3(kThreads), 0, st, pl.ffx, g.nkx, pl.zx,
                           pl.ff_s);
        hipLaunchKernelGGL(k_fftab, dim3(cdiv(pl.out_ny, kThreads)), dim3(kThreads), 0, st, pl.ffy, g.nky, pl.zy,
                           pl.ff_s);
    }
    if (pl.p.want_rpa) {
        const long n = (long)pl.p.nomega * g.neps;
        hipLaunchKernelGGL(k_kkw, dim3(cdiv(n, kThreads)), dim3(kThreads), 0, st, pl.kkw, pl.d_lag, pl.p.nomega,
                           g.neps);
    }
    return hipGetLastError();
}

hipError_t launch_tables(const Plan &pl, hipStream_t st)
{
    return pl.g.fp64 ? tables_t<double>(pl, st) : tables_t<float>(pl, st);
}

// ev (optional, 6 events): recorded before P1 and after P1, P2, P3, P4, P5.
template <typename T>
static hipError_t exec_t(const Plan &pl, T *out, hipStream_t st, hipEvent_t *ev)
{
    const Geo &g = pl.g;
    const size_t cs = sizeof(cx<T>);
    cx<T> *spec = (cx<T> *)pl.spec;
    const cx<T> *twx = (const cx<T> *)pl.twx, *twy = (const cx<T> *)pl.twy;
    const int ff = pl.p.ff_kind != LINDHARD_FF_NONE;
    auto mark = [&](int i) {
        if (ev) (void)hipEventRecord(ev[i], st);
    };
    mark(0);
    if (g.nL > 0) {
        hipLaunchKernelGGL(k_p1<T>, dim3(g.nky / g.p1_R, cdiv(g.nS, g.p1_jc)), dim3(kThreads),
                           (size_t)g.p1_R * g.L * cs, st, pl.xi, g, pl.p.emin, pl.deps, pl.p.gamma, twx, spec);
        mark(1);
        hipLaunchKernelGGL((k_col<T, false>), dim3(g.NT, g.nS), dim3(kThreads), (size_t)g.nky * g.C * cs, st, spec,
                           g, twy);
        mark(2);
        if (g.fp64)
            hipLaunchKernelGGL((k_p3<T, false>), dim3(g.NT, g.nky / g.p3_RY), dim3(kThreads),
                               (size_t)g.nS * g.p3_TR * cs, st, spec, g);
        else
            hipLaunchKernelGGL((k_p3<T, true>), dim3(g.NT, g.nky / g.p3_RY), dim3(kThreads),
                               (size_t)g.nS * g.p3_TR * cs, st, spec, g);
        mark(3);
        hipLaunchKernelGGL((k_col<T, true>), dim3(g.NT, g.nL), dim3(kThreads), (size_t)g.nky * g.C * cs, st, spec,
                           g, twy);
        mark(4);
    } else {
        mark(1);
        mark(2);
        mark(3);
        mark(4);
    }
    const size_t p5lds = (size_t)(2 * g.L + 1) * g.p5_R * cs;
    if (pl.p.want_rpa) {
        if (g.nL > 0)
            hipLaunchKernelGGL((k_p5<T, 1>), dim3(g.nky / g.p5_R, g.nL), dim3(kThreads), p5lds, st, spec, g, twx,
                               pl.d_slot, pl.scale, pl.zx, pl.zy, ff, pl.ff_s, pl.ffx, pl.ffy, (T *)pl.im1, g.nkx,
                               g.nky);
        hipLaunchKernelGGL(k_extend<T>, dim3(cdiv(pl.out_nx, kThreads), pl.out_ny, pl.p.nomega), dim3(kThreads), 0,
                           st, (const T *)pl.im1, g.nkx, g.nky, g.neps, pl.d_lag, pl.zx, pl.zy, ff, pl.ff_s, pl.ffx,
                           pl.ffy, out, pl.out_nx, pl.out_ny);
    } else {
        hipLaunchKernelGGL((k_p5<T, 0>), dim3(g.nky / g.p5_R, pl.p.nomega), dim3(kThreads), p5lds, st, spec, g, twx,
                           pl.d_slot, pl.scale, pl.zx, pl.zy, ff, pl.ff_s, pl.ffx, pl.ffy, out, pl.out_nx,
                           pl.out_ny);
    }
    mark(5);
    return hipGetLastError();
}

hipError_t launch_exec(const Plan &pl, void *out, hipStream_t st, hipEvent_t *ev)
{
    return pl.g.fp64 ? exec_t<double>(pl, (double *)out, st, ev) : exec_t<float>(pl, (float *)out, st, ev);
}

template <typename T>
static hipError_t rpa_t(const Plan &pl, double U, T *re, T *imr, T *rer, hipStream_t st)
{
    const Geo &g = pl.g;
    const int nk = g.nkx * g.nky;
    int logQT = 6;
    while (logQT > 0 && ((size_t)g.neps << logQT) * sizeof(T) > 65536) --logQT;
    while ((1 << logQT) > nk) --logQT;
    hipLaunchKernelGGL(k_kk<T>, dim3(nk >> logQT), dim3(kThreads), ((size_t)g.neps << logQT) * sizeof(T), st,
                       (const T *)pl.im1, nk, g.neps, pl.p.nomega, pl.d_lag, pl.kkw, (T *)pl.re1, logQT);
    const int ff = pl.p.ff_kind != LINDHARD_FF_NONE;
    hipLaunchKernelGGL(k_rpa<T>, dim3(cdiv(pl.out_nx, kThreads), pl.out_ny, pl.p.nomega), dim3(kThreads), 0, st,
                       (const T *)pl.im1, (const T *)pl.re1, g.nkx, g.nky, g.neps, pl.d_lag, pl.zx, pl.zy, ff,
                       pl.ff_s, pl.ffx, pl.ffy, U, re, imr, rer, pl.out_nx, pl.out_ny);
    return hipGetLastError();
}

hipError_t launch_rpa(const Plan &pl, double U, void *re, void *imr, void *rer, hipStream_t st)
{
    return pl.g.fp64 ? rpa_t<double>(pl, U, (double *)re, (double *)imr, (double *)rer, st)
                     : rpa_t<float>(pl, U, (float *)re, (float *)imr, (float *)rer, st);
}

}  // namespace lh
