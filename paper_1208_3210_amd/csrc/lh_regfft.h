// lh_regfft.h -- register-resident Stockham FFT for one line of length
// N = 2^LOGN held by G = N/E threads with E = min(16, N) elements each.
//
// E = min(N, 2^LOGE_MAX), 16 by default.
// Passes: radix E, ..., radix E, then one pass of the remaining radix
// (2..E), each thread doing E / r butterflies of radix r per pass.  Values stay
// in registers inside a pass; between passes they are exchanged through the
// line's LDS buffer (N complex values, XOR-swizzled so that the stride-r
// writes of the first pass and the unit-stride reads are free of bank
// conflicts; a per-line XOR chosen by the caller for its lane layout spreads
// lanes that work on different lines of the same wave over different banks).
// Autosort: no bit reversal anywhere.
//
// Convention on entry and on exit: thread g of the line holds
// v[s] = x[g + s * G], s = 0 .. E-1 (natural order, stride G), so a column pass
// can load from and store to global memory directly in that pattern.
// Twiddles come from a table tw[x] = exp(-2 pi i x / (N << twsh)) built in FP64
// and rounded once (stored at tw_swz(x) when TWS); the inverse uses the
// conjugates (no 1/N).
#pragma once
#include "lh_fft.h"

namespace lh {

// cos / sin of 2 pi m / 16, m = 0 .. 15
__host__ __device__ constexpr double cos16(int m)
{
    constexpr double c[16] = {1.0,
                              0.92387953251128675613,
                              0.70710678118654752440,
                              0.38268343236508977173,
                              0.0,
                              -0.38268343236508977173,
                              -0.70710678118654752440,
                              -0.92387953251128675613,
                              -1.0,
                              -0.92387953251128675613,
                              -0.70710678118654752440,
                              -0.38268343236508977173,
                              0.0,
                              0.38268343236508977173,
                              0.70710678118654752440,
                              0.92387953251128675613};
    return c[m & 15];
}
__host__ __device__ constexpr double sin16(int m) { return cos16(m + 12); }

// a * exp(-+2 pi i k / R) with compile-time R, k (forward: minus sign).
template <typename T, int R, int K, bool INV>
__device__ __forceinline__ cx<T> rot(cx<T> a)
{
    constexpr int m = (K * (16 / R)) & 15;
    if constexpr (m == 0) {
        return a;
    } else if constexpr (m == 4) {
        return INV ? mk<T>(-a.y, a.x) : mk<T>(a.y, -a.x);
    } else if constexpr (m == 8) {
        return mk<T>(-a.x, -a.y);
    } else if constexpr (m == 12) {
        return INV ? mk<T>(a.y, -a.x) : mk<T>(-a.y, a.x);
    } else {
        constexpr T c = (T)cos16(m), s = (T)sin16(m);
        return INV ? mk<T>(a.x * c - a.y * s, a.y * c + a.x * s) : mk<T>(a.x * c + a.y * s, a.y * c - a.x * s);
    }
}

template <typename T, int R, bool INV, int K = 0>
__device__ __forceinline__ void rdft_combine(cx<T> *v, const cx<T> *e, const cx<T> *o)
{
    if constexpr (K < R / 2) {
        const cx<T> t = rot<T, R, K, INV>(o[K]);
        v[K] = cadd(e[K], t);
        v[K + R / 2] = csub(e[K], t);
        rdft_combine<T, R, INV, K + 1>(v, e, o);
    }
}

// In-register DFT of R = 1, 2, 4, 8, 16 points, natural order in and out.
template <typename T, int R, bool INV>
__device__ __forceinline__ void rdft(cx<T> *v)
{
    if constexpr (R == 2) {
        const cx<T> a = v[0], b = v[1];
        v[0] = cadd(a, b);
        v[1] = csub(a, b);
    } else if constexpr (R > 2) {
        cx<T> e[R / 2], o[R / 2];
#pragma unroll
        for (int i = 0; i < R / 2; ++i) {
            e[i] = v[2 * i];
            o[i] = v[2 * i + 1];
        }
        rdft<T, R / 2, INV>(e);
        rdft<T, R / 2, INV>(o);
        rdft_combine<T, R, INV>(v, e, o);
    }
}

__device__ __forceinline__ int swz(int x) { return x ^ ((x >> 4) & 15); }

// Twiddle tables kept in LDS are stored with this XOR swizzle (a bijection on
// any power-of-two length): the reads of one pass, index (s k) << sh for the
// butterflies of a wave, otherwise fall into a few LDS banks.
__host__ __device__ constexpr int tw_swz(int i) { return i ^ ((i >> 5) & 31); }

// TWS: the twiddle table is stored with tw_swz.
template <typename T, int LOGN, bool INV, int LOGE_MAX = 4, bool TWS = false>
struct RegFFT {
    static constexpr int N = 1 << LOGN;
    static constexpr int LOGE = LOGN < LOGE_MAX ? LOGN : LOGE_MAX;
    static constexpr int E = 1 << LOGE;
    static constexpr int G = N / E;
    static constexpr int NPASS = LOGN == 0 ? 0 : (LOGN + LOGE - 1) / LOGE;

    // One pass of radix 2^LOGR with sub-length p = 2^LOGP.
    template <int LOGR, int LOGP>
    __device__ static __forceinline__ void pass(cx<T> *v, cx<T> *buf, const cx<T> *__restrict__ tw, int twsh,
                                                int g, int lx)
    {
        constexpr int r = 1 << LOGR;
        constexpr int p = 1 << LOGP;
        constexpr int q = E / r;       // butterflies per thread
        constexpr int stride = N / r;  // input stride
        constexpr bool first = LOGP == 0;
        constexpr bool last = LOGP + LOGR == LOGN;
        cx<T> w[E];
        if constexpr (first) {
#pragma unroll
            for (int u = 0; u < q; ++u)
#pragma unroll
                for (int s = 0; s < r; ++s) w[u * r + s] = v[u + s * q];
        } else {
#pragma unroll
            for (int u = 0; u < q; ++u) {
                const int b = g + u * G;
#pragma unroll
                for (int s = 0; s < r; ++s) w[u * r + s] = buf[swz(b + s * stride) ^ lx];
            }
            __syncthreads();
        }
#pragma unroll
        for (int u = 0; u < q; ++u) {
            const int b = g + u * G;
            const int k = b & (p - 1);
            if constexpr (!first) {
                const int sh = LOGN - LOGP - LOGR + twsh;
#pragma unroll
                for (int s = 1; s < r; ++s) {
                    const int x = (s * k) << sh;
                    w[u * r + s] = cmul(w[u * r + s], twid<T, INV>(tw, TWS ? tw_swz(x) : x));
                }
            }
            rdft<T, r, INV>(w + u * r);
            if constexpr (last) {
#pragma unroll
                for (int s = 0; s < r; ++s) v[u + s * q] = w[u * r + s];
            } else {
                const int o = (b - k) * r + k;
#pragma unroll
                for (int s = 0; s < r; ++s) buf[swz(o + s * p) ^ lx] = w[u * r + s];
            }
        }
        if constexpr (!last) __syncthreads();
    }

    template <int T_>
    __device__ static __forceinline__ void passes(cx<T> *v, cx<T> *buf, const cx<T> *__restrict__ tw, int twsh,
                                                  int g, int lx)
    {
        if constexpr (T_ < NPASS) {
            constexpr int LOGP = T_ * LOGE;
            constexpr int LOGR = (LOGN - LOGP) < LOGE ? (LOGN - LOGP) : LOGE;
            pass<LOGR, LOGP>(v, buf, tw, twsh, g, lx);
            passes<T_ + 1>(v, buf, tw, twsh, g, lx);
        }
    }

    // Transform one line.  Every thread of the block must call this (it
    // contains block barriers).  buf: N complex values of LDS for this line;
    // lx: XOR applied to every LDS index of this line (0 <= lx < N; see
    // lds_xor_interleaved / lds_xor_gfast).  Ends with a barrier when there is
    // more than one pass, so buf may be reused right after.
    __device__ static __forceinline__ void run(cx<T> *v, cx<T> *buf, const cx<T> *__restrict__ tw, int twsh,
                                               int g, int lx = 0)
    {
        passes<0>(v, buf, tw, twsh, g, lx);
    }
};

// LDS banks hold 64 dwords: 32 FP32 or 16 FP64 complex values.
template <typename T>
constexpr int lds_bank_elems()
{
    return sizeof(T) == 4 ? 32 : 16;
}

// Per-line XOR when NL lines are interleaved lane by lane (lane = g NL + line):
// the lines of one 32-lane group then occupy disjoint bank ranges.
template <typename T, int N>
__device__ __forceinline__ int lds_xor_interleaved(int line, int NL)
{
    const int m = lds_bank_elems<T>() / NL;
    return (line * (m > 0 ? m : 1)) & (N - 1);
}

// Per-line XOR when each line takes G consecutive lanes (lane = line G + g).
template <int N, int G>
__device__ __forceinline__ int lds_xor_gfast(int line)
{
    return (line * G) & (N - 1);
}

}  // namespace lh

namespace lh {

// Padded-layout variant of the same transform (FP32 passes whose lines have
// G >= 2^PB threads).  Element x of a line sits at x + (x >> PB) of its LDS
// buffer.  The index a thread reads or writes in a pass splits into a part
// that depends only on its g and a part fixed at compile time (butterfly u,
// element s) whose bits never carry across bit PB when added, so the padded
// address is a per-thread base plus an immediate offset: the exchanges cost
// no per-element address arithmetic.  One padding slot per 2^PB elements
// spreads the stride-r writes of a pass over the LDS banks.
//
// Twiddles come from a per-pass table (fill_twiddles): pass t >= 1 (radix r,
// sub-length p) holds exp(-+2 pi i s k / (p r)) for k < min(p, G),
// 1 <= s < r at tw_off(t) + k (r - 1) + s - 1.  A thread's k is (g mod p)
// plus a compile-time multiple of G, so these reads are base plus immediate
// too, and r - 1 is odd, so lanes with different k fall into different banks.
// Only the last pass can have p > G (then p r = N); its butterflies with
// k = g + u G take row g times the constant exp(-+2 pi i s u / E), which keeps
// the table near N / E + N / 8 entries.
// a * exp(-+2 pi i m / 16) (forward: minus sign); m is a constant after
// unrolling, so the branches fold away.
template <typename T, bool INV>
__device__ __forceinline__ cx<T> rot16(cx<T> a, int m)
{
    m &= 15;
    if (m == 0) return a;
    if (m == 4) return INV ? mk<T>(-a.y, a.x) : mk<T>(a.y, -a.x);
    if (m == 8) return mk<T>(-a.x, -a.y);
    if (m == 12) return INV ? mk<T>(a.y, -a.x) : mk<T>(-a.y, a.x);
    const T c = (T)cos16(m), s = (T)sin16(m);
    return INV ? mk<T>(a.x * c - a.y * s, a.y * c + a.x * s) : mk<T>(a.x * c + a.y * s, a.y * c - a.x * s);
}

template <typename T, int LOGN, bool INV, int LOGE_MAX, int PB>
struct RegFFTP {
    static constexpr int N = 1 << LOGN;
    static constexpr int LOGE = LOGN < LOGE_MAX ? LOGN : LOGE_MAX;
    static constexpr int E = 1 << LOGE;
    static constexpr int G = N / E;
    static constexpr int NPASS = (LOGN + LOGE - 1) / LOGE;
    static_assert(G >= (1 << PB), "the padded layout needs at least 2^PB threads per line");
    // LDS elements of one line
    static constexpr int LINE = N + (N >> PB);

    __host__ __device__ static constexpr int pad(int x) { return x + (x >> PB); }
    __host__ __device__ static constexpr int log_radix(int t) { return LOGN - t * LOGE < LOGE ? LOGN - t * LOGE : LOGE; }
    // table rows of pass t: k < min(p, G)
    __host__ __device__ static constexpr int rows(int t) { return (1 << (t * LOGE)) < G ? (1 << (t * LOGE)) : G; }
    // offset of pass t's twiddles in the table; tw_off(NPASS) is its length
    __host__ __device__ static constexpr int tw_off(int t)
    {
        int off = 0;
        for (int u = 1; u < t; ++u) off += rows(u) * ((1 << log_radix(u)) - 1);
        return off;
    }
    static constexpr int TWN = tw_off(NPASS);

    // Build the per-pass table at dst from tw[x] = exp(-2 pi i x / (N << twsh)).
    // Every thread of the block calls it; no barrier (the caller orders it
    // before the first pass that reads it).
    __device__ static void fill_twiddles(cx<T> *dst, const cx<T> *__restrict__ tw, int tid, int nthr,
                                         int twsh = 0)
    {
#pragma unroll
        for (int t = 1; t < NPASS; ++t) {
            const int lr = log_radix(t), lp = t * LOGE;
            const int r = 1 << lr, items = rows(t) << lr;
            const int sh = LOGN - lp - lr + twsh;
            cx<T> *d = dst + tw_off(t);
            for (int i = tid; i < items; i += nthr) {
                const int s = i & (r - 1), k = i >> lr;
                if (s) d[k * (r - 1) + s - 1] = tw[(s * k) << sh];
            }
        }
    }

    template <int LOGR, int LOGP>
    __device__ static __forceinline__ void pass(cx<T> *v, cx<T> *buf, const cx<T> *tw, int g)
    {
        constexpr int r = 1 << LOGR;
        constexpr int p = 1 << LOGP;
        constexpr int q = E / r;
        constexpr int stride = N / r;
        constexpr bool first = LOGP == 0;
        constexpr bool last = LOGP + LOGR == LOGN;
        cx<T> w[E];
        if constexpr (first) {
#pragma unroll
            for (int u = 0; u < q; ++u)
#pragma unroll
                for (int s = 0; s < r; ++s) w[u * r + s] = v[u + s * q];
        } else {
            const cx<T> *rb = buf + pad(g);
#pragma unroll
            for (int u = 0; u < q; ++u)
#pragma unroll
                for (int s = 0; s < r; ++s) w[u * r + s] = rb[pad(u * G + s * stride)];
            __syncthreads();
        }
        const cx<T> *tb = tw + tw_off(LOGP / LOGE) + (g & (p - 1)) * (r - 1);
        cx<T> *wb = buf + pad(((g >> LOGP) << (LOGP + LOGR)) + (g & (p - 1)));
#pragma unroll
        for (int u = 0; u < q; ++u) {
            if constexpr (!first) {
#pragma unroll
                for (int s = 1; s < r; ++s) {
                    cx<T> tws;
                    if constexpr (p <= G) {
                        tws = twid<T, INV>(tb, s - 1);
                    } else {
                        // k = g + u G: row g turned by exp(-+2 pi i s u G / N)
                        static_assert(LOGP + LOGR == LOGN && E <= 16, "p > G only in the last pass");
                        tws = rot16<T, INV>(twid<T, INV>(tb, s - 1), s * u * (16 / E));
                    }
                    w[u * r + s] = cmul(w[u * r + s], tws);
                }
            }
            rdft<T, r, INV>(w + u * r);
            if constexpr (last) {
#pragma unroll
                for (int s = 0; s < r; ++s) v[u + s * q] = w[u * r + s];
            } else {
#pragma unroll
                for (int s = 0; s < r; ++s) wb[pad((((u * G) >> LOGP) << (LOGP + LOGR)) + s * p)] = w[u * r + s];
            }
        }
        if constexpr (!last) __syncthreads();
    }

    template <int T_>
    __device__ static __forceinline__ void passes(cx<T> *v, cx<T> *buf, const cx<T> *tw, int g)
    {
        if constexpr (T_ < NPASS) {
            constexpr int LOGP = T_ * LOGE;
            constexpr int LOGR = (LOGN - LOGP) < LOGE ? (LOGN - LOGP) : LOGE;
            pass<LOGR, LOGP>(v, buf, tw, g);
            passes<T_ + 1>(v, buf, tw, g);
        }
    }

    // Same entry and exit convention as RegFFT::run; buf holds LINE elements
    // of this line, tw the per-pass table.
    __device__ static __forceinline__ void run(cx<T> *v, cx<T> *buf, const cx<T> *tw, int g) { passes<0>(v, buf, tw, g); }
};

}  // namespace lh
