// lh_fft.h -- complex arithmetic and the in-LDS radix-4/2 FFT engine used by
// every transform pass (gfx950, wave64).
//
// Layout convention for every LDS buffer: element n of line l sits at
// buf[n * NL + l] (line index fastest), so consecutive threads touch
// consecutive addresses in every stage.  The engine is an in-place
// decimation-in-frequency transform: a first radix-2 stage when log2(L) is
// odd, then radix-4 stages.  Butterflies of one stage touch disjoint elements,
// so one barrier per stage suffices and no ping-pong buffer is needed.  The
// output is in mixed-radix digit-reversed order; dif_pos(k) gives the slot of
// frequency k.
#pragma once
#include <hip/hip_runtime.h>

namespace lh {

template <typename T>
struct __align__(2 * sizeof(T)) cx {
    T x, y;
};

template <typename T>
__device__ __forceinline__ cx<T> mk(T a, T b)
{
    cx<T> r;
    r.x = a;
    r.y = b;
    return r;
}
template <typename T>
__device__ __forceinline__ cx<T> cadd(cx<T> a, cx<T> b)
{
    return mk<T>(a.x + b.x, a.y + b.y);
}
template <typename T>
__device__ __forceinline__ cx<T> csub(cx<T> a, cx<T> b)
{
    return mk<T>(a.x - b.x, a.y - b.y);
}
template <typename T>
__device__ __forceinline__ cx<T> cmul(cx<T> a, cx<T> b)
{
    return mk<T>(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}
template <typename T>
__device__ __forceinline__ cx<T> cconj(cx<T> a)
{
    return mk<T>(a.x, -a.y);
}
template <typename T>
__device__ __forceinline__ cx<T> cscale(cx<T> a, T s)
{
    return mk<T>(a.x * s, a.y * s);
}

// Twiddle table entry tw[s] = exp(-2 pi i s / Ntw); the inverse transform uses
// the conjugate.
template <typename T, bool INV>
__device__ __forceinline__ cx<T> twid(const cx<T> *__restrict__ tw, int s)
{
    cx<T> w = tw[s];
    if (INV) w.y = -w.y;
    return w;
}

// Slot of frequency k after the DIF transform of length 2^logL.
__device__ __forceinline__ int dif_pos(int k, int logL)
{
    int p = 0, rem = logL;
    if (logL & 1) {
        rem -= 1;
        p |= (k & 1) << rem;
        k >>= 1;
    }
    while (rem > 0) {
        rem -= 2;
        p |= (k & 3) << rem;
        k >>= 2;
    }
    return p;
}

// In-place DIF FFT of NL = 2^logNL lines of length L = 2^logL held in LDS.
// Forward: X[k] = sum_n x[n] exp(-2 pi i n k / L); INV uses exp(+...), no
// normalisation.  tw has 2^logNtw >= L entries.  Ends with a barrier.
template <typename T, bool INV>
__device__ void fft_dif_lds(cx<T> *buf, int logL, int logNL, const cx<T> *__restrict__ tw, int logNtw,
                            int tid, int nthr)
{
    const int L = 1 << logL;
    const int NL = 1 << logNL;
    int logM = logL;
    if (logL & 1) {
        const int h = L >> 1;
        const int items = NL * h;
        const int sh = logNtw - logM;
        for (int it = tid; it < items; it += nthr) {
            const int line = it & (NL - 1);
            const int t = it >> logNL;
            cx<T> *p0 = buf + t * NL + line;
            cx<T> *p1 = p0 + h * NL;
            const cx<T> a = *p0, b = *p1;
            *p0 = cadd(a, b);
            *p1 = cmul(csub(a, b), twid<T, INV>(tw, t << sh));
        }
        __syncthreads();
        logM -= 1;
    }
    const int items4 = NL * (L >> 2);
    while (logM >= 2) {
        const int logq = logM - 2;
        const int q = 1 << logq;
        const int sh = logNtw - logM;
        for (int it = tid; it < items4; it += nthr) {
            const int line = it & (NL - 1);
            const int bf = it >> logNL;
            const int t = bf & (q - 1);
            const int base = ((bf >> logq) << logM) + t;
            cx<T> *p = buf + base * NL + line;
            const int st = q * NL;
            const cx<T> x0 = p[0], x1 = p[st], x2 = p[2 * st], x3 = p[3 * st];
            const cx<T> a0 = cadd(x0, x2), a1 = csub(x0, x2), a2 = cadd(x1, x3);
            cx<T> a3 = csub(x1, x3);
            // forward: multiply by -i; inverse: by +i
            a3 = INV ? mk<T>(-a3.y, a3.x) : mk<T>(a3.y, -a3.x);
            p[0] = cadd(a0, a2);
            if (t == 0) {
                p[st] = cadd(a1, a3);
                p[2 * st] = csub(a0, a2);
                p[3 * st] = csub(a1, a3);
            } else {
                p[st] = cmul(cadd(a1, a3), twid<T, INV>(tw, t << sh));
                p[2 * st] = cmul(csub(a0, a2), twid<T, INV>(tw, (2 * t) << sh));
                p[3 * st] = cmul(csub(a1, a3), twid<T, INV>(tw, (3 * t) << sh));
            }
        }
        __syncthreads();
        logM -= 2;
    }
}

}  // namespace lh
