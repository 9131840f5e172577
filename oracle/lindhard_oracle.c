/*
 * lindhard_oracle.c -- plain, slow FP64 reference for the bare Lindhard
 * susceptibility of Wang et al., "Lindhard and RPA susceptibility computations
 * in extended momentum space in electron doped cuprates" (arXiv:1208.3210).
 *
 * TEST INFRASTRUCTURE ONLY.  This file is the oracle that the GPU library is
 * checked against.  Only the test suite, the smoke check and the CPU-baseline
 * leg of the benchmark may load it; the library never calls it and shares no
 * source with it.
 *
 * What is computed (the discrete definition, written out directly):
 *   k-grid        k = (2 pi ix / Nkx, 2 pi iy / Nky), Nk = Nkx * Nky, periodic.
 *   energy grid   d = (emax - emin) / Neps, e_j = emin + (j + 1/2) d (cell centred).
 *   occupied set  j < j0, j0 = #{ j : e_j <= 0 }.
 *   spectral fn   A(k, j) = (G / pi) / ((e_j - xi_k)^2 + G^2)        -- Eq. (5)
 *   bare chi      Im chi(q, m) = -(d / Nk) sum_k sum_j A(k, j) A(k + q, j + m),
 *                 j over max(0, j0 - m) <= j < min(j0, Neps - m)     -- Eqs. (2), (9), (A3)
 *                 i.e. the energy integral over -w < e <= 0 at w = m d of the
 *                 occupied/unoccupied product, per site and per spin, with the
 *                 Lorentzian normalised to unit area and no extra 1/(2 pi).
 *   chemical pot. n(mu) = (2 / Nk) sum_k [1/2 + atan((mu - eps_k) / G) / pi]
 *                 solved for n(mu) = filling by bisection (rigid band, Sec. 3).
 *
 * Sums over k and over j use Neumaier compensation so that the oracle's own
 * rounding error stays near the FP64 unit roundoff.
 *
 * Parity status: every function here is pinned by CPU tests against identities,
 * closed forms and brute force (see tests/test_oracle_pins.py).
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#ifdef _OPENMP
#include <omp.h>
#endif

#define ORACLE_PI 3.14159265358979323846

/* Neumaier (improved Kahan-Babuska) running sum. */
typedef struct {
    double s, c;
} nsum;

static inline void nsum_add(nsum *a, double x)
{
    double t = a->s + x;
    if (fabs(a->s) >= fabs(x))
        a->c += (a->s - t) + x;
    else
        a->c += (x - t) + a->s;
    a->s = t;
}

static inline double nsum_get(const nsum *a) { return a->s + a->c; }

void oracle_band_tb_z(double t, double tp, double tpp, int nkx, int nky, int kz, double *eps);

/* Tight-binding band of the square lattice (single Cu-O band, Sec. 3):
 * eps(k) = -2t (cos kx + cos ky) - 4t' cos kx cos ky - 2t'' (cos 2kx + cos 2ky).
 * eps is row major [iy][ix]. */
void oracle_band_tb(double t, double tp, double tpp, int nkx, int nky, double *eps)
{
    oracle_band_tb_z(t, tp, tpp, nkx, nky, 1, eps);
}

/* The same band on a momentum grid spanning kz Brillouin zones per axis
 * (extended momentum p = 2 pi kz (ix/nkx, iy/nky), Eq. (9)). */
void oracle_band_tb_z(double t, double tp, double tpp, int nkx, int nky, int kz, double *eps)
{
    for (int iy = 0; iy < nky; ++iy) {
        double ky = 2.0 * ORACLE_PI * kz * iy / nky;
        for (int ix = 0; ix < nkx; ++ix) {
            double kx = 2.0 * ORACLE_PI * kz * ix / nkx;
            eps[(size_t)iy * nkx + ix] = -2.0 * t * (cos(kx) + cos(ky)) - 4.0 * tp * cos(kx) * cos(ky) -
                                         2.0 * tpp * (cos(2.0 * kx) + cos(2.0 * ky));
        }
    }
}

/* Electrons per site (both spins) of the Lorentzian-broadened band, Eq. (5)
 * integrated up to mu: each state holds 1/2 + atan((mu - eps)/G)/pi per spin.
 * Summed in fixed chunks so the result does not depend on the thread count. */
double oracle_filling(const double *eps, long nk, double gamma, double mu)
{
    const long chunk = 4096;
    long nchunks = (nk + chunk - 1) / chunk;
    double *part = (double *)malloc(sizeof(double) * (size_t)(nchunks > 0 ? nchunks : 1));
#pragma omp parallel for schedule(static)
    for (long c = 0; c < nchunks; ++c) {
        nsum s = {0.0, 0.0};
        long hi = (c + 1) * chunk < nk ? (c + 1) * chunk : nk;
        for (long k = c * chunk; k < hi; ++k)
            nsum_add(&s, 0.5 + atan((mu - eps[k]) / gamma) / ORACLE_PI);
        part[c] = nsum_get(&s);
    }
    nsum tot = {0.0, 0.0};
    for (long c = 0; c < nchunks; ++c)
        nsum_add(&tot, part[c]);
    free(part);
    return 2.0 * nsum_get(&tot) / (double)nk;
}

/* Rigid-band chemical potential (Sec. 3): bisection of n(mu) = filling on
 * [min eps - 100, max eps + 100] until the bracket is 1e-14 eV wide. */
double oracle_mu(const double *eps, long nk, double gamma, double filling)
{
    double lo = eps[0], hi = eps[0];
    for (long k = 1; k < nk; ++k) {
        if (eps[k] < lo) lo = eps[k];
        if (eps[k] > hi) hi = eps[k];
    }
    lo -= 100.0;
    hi += 100.0;
    while (hi - lo > 1e-14) {
        double mid = 0.5 * (lo + hi);
        if (mid <= lo || mid >= hi) break;
        if (oracle_filling(eps, nk, gamma, mid) < filling)
            lo = mid;
        else
            hi = mid;
    }
    return 0.5 * (lo + hi);
}

/* Number of occupied energy points: j0 = #{ j : e_j <= 0 }. */
int oracle_j0(int neps, double emin, double emax)
{
    double d = (emax - emin) / neps;
    int j0 = 0;
    for (int j = 0; j < neps; ++j)
        if (emin + (j + 0.5) * d <= 0.0) ++j0;
    return j0;
}

static inline double lorentz(double e, double xi, double gamma)
{
    double x = e - xi;
    return (gamma / ORACLE_PI) / (x * x + gamma * gamma);
}

/* Sum over k of the energy-window product for one q and a list of lags.
 * acc[im] receives sum_k sum_j A(k, j) A(k+q, j+m_im) (not yet scaled).
 * Only the energy points that some requested lag can reach are evaluated:
 * occupied j >= j0 - max(m) for A(k, j), unoccupied j < j0 + max(m) for
 * A(k+q, j). */
static void chi_one_q(const double *xi, const double *rho, int nkx, int nky, int neps, double emin, double d,
                      int j0, double gamma, int qx, int qy, int nm, const int *ms, double *acc, double *arow,
                      double *brow, nsum *sums)
{
    int mmax = 0;
    for (int im = 0; im < nm; ++im) {
        sums[im].s = 0.0;
        sums[im].c = 0.0;
        if (ms[im] > mmax) mmax = ms[im];
    }
    int alo = j0 - mmax > 0 ? j0 - mmax : 0;
    int bhi = j0 + mmax < neps ? j0 + mmax : neps;
    int qxm = ((qx % nkx) + nkx) % nkx, qym = ((qy % nky) + nky) % nky;
    for (int iy = 0; iy < nky; ++iy) {
        int iy2 = (iy + qym) % nky;
        for (int ix = 0; ix < nkx; ++ix) {
            int ix2 = (ix + qxm) % nkx;
            double xa = xi[(size_t)iy * nkx + ix];
            double xb = xi[(size_t)iy2 * nkx + ix2];
            for (int j = alo; j < j0; ++j)
                arow[j] = lorentz(emin + (j + 0.5) * d, xa, gamma);
            for (int j = j0; j < bhi; ++j)
                brow[j] = lorentz(emin + (j + 0.5) * d, xb, gamma);
            for (int im = 0; im < nm; ++im) {
                int m = ms[im];
                int jlo = j0 - m > 0 ? j0 - m : 0;
                int jhi = neps - m < j0 ? neps - m : j0;
                if (jlo >= jhi) continue;
                nsum p = {0.0, 0.0};
                for (int j = jlo; j < jhi; ++j)
                    nsum_add(&p, arow[j] * brow[j + m]);
                /* momentum-density weights of Eq. (4): rho(k) rho(k+q) */
                double w = rho ? rho[(size_t)iy * nkx + ix] * rho[(size_t)iy2 * nkx + ix2] : 1.0;
                nsum_add(&sums[im], w * nsum_get(&p));
            }
        }
    }
    for (int im = 0; im < nm; ++im)
        acc[im] = nsum_get(&sums[im]);
}

/* Im chi_1BZ(q, m) on a q-list x lag-list grid (Eq. (9) in the discrete
 * form above).  xi = eps - mu, row major [iy][ix].  out[iq * nm + im].
 * Lags outside 1 <= m < neps have an empty energy window and give 0. */
int oracle_chi_grid_w(const double *xi, const double *rho, int nkx, int nky, int neps, double emin,
                      double emax, double gamma, int nq, const int *qx, const int *qy, int nm, const int *ms,
                      double *out);

int oracle_chi_grid(const double *xi, int nkx, int nky, int neps, double emin, double emax,
                    double gamma, int nq, const int *qx, const int *qy, int nm, const int *ms,
                    double *out)
{
    return oracle_chi_grid_w(xi, NULL, nkx, nky, neps, emin, emax, gamma, nq, qx, qy, nm, ms, out);
}

/* The same with momentum-density weights rho[iy][ix] on the spectral
 * function (A(p, e) = rho(p) A_band(p, e), Eq. (4)); rho = NULL means 1. */
int oracle_chi_grid_w(const double *xi, const double *rho, int nkx, int nky, int neps, double emin,
                      double emax, double gamma, int nq, const int *qx, const int *qy, int nm, const int *ms,
                      double *out)
{
    if (nkx <= 0 || nky <= 0 || neps <= 0 || !(emax > emin) || !(gamma > 0)) return -1;
    double d = (emax - emin) / neps;
    int j0 = oracle_j0(neps, emin, emax);
    double scale = -d / ((double)nkx * (double)nky);
    int bad = 0;
#pragma omp parallel
    {
        double *arow = (double *)malloc(sizeof(double) * (size_t)neps);
        double *brow = (double *)malloc(sizeof(double) * (size_t)neps);
        double *acc = (double *)malloc(sizeof(double) * (size_t)(nm > 0 ? nm : 1));
        nsum *sums = (nsum *)malloc(sizeof(nsum) * (size_t)(nm > 0 ? nm : 1));
        if (!arow || !brow || !acc || !sums) {
#pragma omp atomic write
            bad = 1;
        } else {
#pragma omp for schedule(dynamic, 1)
            for (int iq = 0; iq < nq; ++iq) {
                chi_one_q(xi, rho, nkx, nky, neps, emin, d, j0, gamma, qx[iq], qy[iq], nm, ms, acc, arow,
                          brow, sums);
                for (int im = 0; im < nm; ++im)
                    out[(size_t)iq * nm + im] = scale * acc[im];
            }
        }
        free(arow);
        free(brow);
        free(acc);
        free(sums);
    }
    return bad ? -3 : 0;
}

/* Im chi_1BZ at an explicit list of (qx, qy, m) samples; out[i]. */
int oracle_chi_pairs_w(const double *xi, const double *rho, int nkx, int nky, int neps, double emin,
                       double emax, double gamma, long npairs, const int *qx, const int *qy, const int *ms,
                       double *out);

int oracle_chi_pairs(const double *xi, int nkx, int nky, int neps, double emin, double emax,
                     double gamma, long npairs, const int *qx, const int *qy, const int *ms,
                     double *out)
{
    return oracle_chi_pairs_w(xi, NULL, nkx, nky, neps, emin, emax, gamma, npairs, qx, qy, ms, out);
}

/* Sampled form with momentum-density weights (rho = NULL means 1). */
int oracle_chi_pairs_w(const double *xi, const double *rho, int nkx, int nky, int neps, double emin,
                       double emax, double gamma, long npairs, const int *qx, const int *qy, const int *ms,
                       double *out)
{
    if (nkx <= 0 || nky <= 0 || neps <= 0 || !(emax > emin) || !(gamma > 0)) return -1;
    double d = (emax - emin) / neps;
    int j0 = oracle_j0(neps, emin, emax);
    double scale = -d / ((double)nkx * (double)nky);
    int bad = 0;
#pragma omp parallel
    {
        double *arow = (double *)malloc(sizeof(double) * (size_t)neps);
        double *brow = (double *)malloc(sizeof(double) * (size_t)neps);
        if (!arow || !brow) {
#pragma omp atomic write
            bad = 1;
        } else {
#pragma omp for schedule(dynamic, 1)
            for (long i = 0; i < npairs; ++i) {
                double acc;
                nsum s;
                chi_one_q(xi, rho, nkx, nky, neps, emin, d, j0, gamma, qx[i], qy[i], 1, &ms[i], &acc,
                          arow, brow, &s);
                out[i] = scale * acc;
            }
        }
        free(arow);
        free(brow);
    }
    return bad ? -3 : 0;
}

/* Several bands (Eqs. (2), (4)).  xi and rho (NULL = 1) hold nb planes
 * [band][iy][ix]; the spectral function of band n at k is
 * rho_n(k) A(e - xi_n(k)).
 *   pairw == NULL: Eq. (4) sums the bands, A(k, e) = sum_n rho_n(k) A_n(k, e),
 *                  and acc[im] = sum_k sum_j A(k, j) A(k+q, j+m);
 *   otherwise:     Eq. (2), acc[im] = sum_{nu,mu} pairw[nu nb + mu]
 *                  sum_k sum_j A_nu(k, j) A_mu(k+q, j+m)
 * with j occupied and j + m empty as in chi_one_q.  ar, br: nb * neps. */
static void chi_one_q_mb(const double *xi, const double *rho, int nb, const double *pairw, int nkx, int nky,
                         int nkz, int neps, double emin, double d, int j0, double gamma, int qx, int qy, int qz,
                         int nm, const int *ms, double *acc, double *ar, double *br, nsum *sums)
{
    int mmax = 0;
    for (int im = 0; im < nm; ++im) {
        sums[im].s = 0.0;
        sums[im].c = 0.0;
        if (ms[im] > mmax) mmax = ms[im];
    }
    int alo = j0 - mmax > 0 ? j0 - mmax : 0;
    int bhi = j0 + mmax < neps ? j0 + mmax : neps;
    int qxm = ((qx % nkx) + nkx) % nkx, qym = ((qy % nky) + nky) % nky, qzm = ((qz % nkz) + nkz) % nkz;
    size_t nk = (size_t)nkx * nky * nkz;
    for (int izy = 0; izy < nkz * nky; ++izy) {  /* k = (iz, iy, ix), the kz planes one after another */
        int iz = izy / nky, iy = izy % nky;
        int iz2 = (iz + qzm) % nkz, iy2 = (iy + qym) % nky;
        for (int ix = 0; ix < nkx; ++ix) {
            int ix2 = (ix + qxm) % nkx;
            size_t k1 = ((size_t)iz * nky + iy) * nkx + ix, k2 = ((size_t)iz2 * nky + iy2) * nkx + ix2;
            for (int n = 0; n < nb; ++n) {
                double ra = rho ? rho[n * nk + k1] : 1.0, rb = rho ? rho[n * nk + k2] : 1.0;
                for (int j = alo; j < j0; ++j)
                    ar[(size_t)n * neps + j] = ra * lorentz(emin + (j + 0.5) * d, xi[n * nk + k1], gamma);
                for (int j = j0; j < bhi; ++j)
                    br[(size_t)n * neps + j] = rb * lorentz(emin + (j + 0.5) * d, xi[n * nk + k2], gamma);
            }
            if (!pairw) {  /* the summed spectral function goes into band slot 0 */
                for (int j = alo; j < j0; ++j)
                    for (int n = 1; n < nb; ++n) ar[j] += ar[(size_t)n * neps + j];
                for (int j = j0; j < bhi; ++j)
                    for (int n = 1; n < nb; ++n) br[j] += br[(size_t)n * neps + j];
            }
            for (int im = 0; im < nm; ++im) {
                int m = ms[im];
                int jlo = j0 - m > 0 ? j0 - m : 0;
                int jhi = neps - m < j0 ? neps - m : j0;
                if (jlo >= jhi) continue;
                int np = pairw ? nb : 1;
                for (int nu = 0; nu < np; ++nu)
                    for (int mu = 0; mu < np; ++mu) {
                        double w = pairw ? pairw[nu * nb + mu] : 1.0;
                        if (w == 0.0) continue;
                        nsum p = {0.0, 0.0};
                        for (int j = jlo; j < jhi; ++j)
                            nsum_add(&p, ar[(size_t)nu * neps + j] * br[(size_t)mu * neps + j + m]);
                        nsum_add(&sums[im], w * nsum_get(&p));
                    }
            }
        }
    }
    for (int im = 0; im < nm; ++im)
        acc[im] = nsum_get(&sums[im]);
}

/* Three-dimensional k-grid [iz][iy][ix] (the d^3p of Eq. (9)) with several
 * bands as above; q = (qx, qy, qz); per-site normalisation over nkx nky nkz. */
int oracle_chi_grid_3d(const double *xi, const double *rho, int nb, const double *pairw, int nkx, int nky,
                       int nkz, int neps, double emin, double emax, double gamma, int nq, const int *qx,
                       const int *qy, const int *qz, int nm, const int *ms, double *out)
{
    if (nb < 1 || nkx <= 0 || nky <= 0 || nkz <= 0 || neps <= 0 || !(emax > emin) || !(gamma > 0)) return -1;
    double d = (emax - emin) / neps;
    int j0 = oracle_j0(neps, emin, emax);
    double scale = -d / ((double)nkx * (double)nky * (double)nkz);
    int bad = 0;
#pragma omp parallel
    {
        double *ar = (double *)malloc(sizeof(double) * (size_t)nb * neps);
        double *br = (double *)malloc(sizeof(double) * (size_t)nb * neps);
        double *acc = (double *)malloc(sizeof(double) * (size_t)(nm > 0 ? nm : 1));
        nsum *sums = (nsum *)malloc(sizeof(nsum) * (size_t)(nm > 0 ? nm : 1));
        if (!ar || !br || !acc || !sums) {
#pragma omp atomic write
            bad = 1;
        } else {
#pragma omp for schedule(dynamic, 1)
            for (int iq = 0; iq < nq; ++iq) {
                chi_one_q_mb(xi, rho, nb, pairw, nkx, nky, nkz, neps, emin, d, j0, gamma, qx[iq], qy[iq],
                             qz ? qz[iq] : 0, nm, ms, acc, ar, br, sums);
                for (int im = 0; im < nm; ++im)
                    out[(size_t)iq * nm + im] = scale * acc[im];
            }
        }
        free(ar);
        free(br);
        free(acc);
        free(sums);
    }
    return bad ? -3 : 0;
}

int oracle_chi_grid_mb(const double *xi, const double *rho, int nb, const double *pairw, int nkx, int nky,
                       int neps, double emin, double emax, double gamma, int nq, const int *qx, const int *qy,
                       int nm, const int *ms, double *out)
{
    return oracle_chi_grid_3d(xi, rho, nb, pairw, nkx, nky, 1, neps, emin, emax, gamma, nq, qx, qy, NULL, nm, ms,
                              out);
}

/* Threads the OpenMP runtime will use (for reporting the baseline's cores). */
int oracle_num_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}
