// lh_api.hip -- C ABI entry points: validation, planning (band, chemical
// potential, tables, workspace) and execution.
#include <algorithm>
#include <climits>
#include <cmath>
#include <complex>
#include <condition_variable>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <map>
#include <mutex>
#include <string>
#include <new>
#include <set>
#include <vector>

#include "lh_internal.h"

namespace lh {

static bool is_pow2(long v) { return v > 0 && (v & (v - 1)) == 0; }
static int ilog2(long v)
{
    int r = 0;
    while ((1L << r) < v) ++r;
    return r;
}

// Cell-centred energy grid of the window (emin, emax]: j0 = #{e_j <= 0}.
static int count_occupied(int neps, double emin, double emax)
{
    const double d = (emax - emin) / neps;
    int j0 = 0;
    for (int j = 0; j < neps; ++j)
        if (emin + (j + 0.5) * d <= 0.0) ++j0;
    return j0;
}

// Point stride of the matrix-core even window with TR points per block: at
// least the staged rows, and congruent to 64 / TR modulo 64 so that the
// staging writes of one wave (TR points x 64 / TR consecutive rows) hit 64
// different banks.
static int even_mfma_ps(const Geo &g, int TR)
{
    const int base = g.e3m_PA + g.e3m_nHe + 64;
    return base + (((64 / TR - base) % 64) + 64) % 64;
}

// LDS bytes of the matrix-core even window with TR points per block: the
// staged points, and the output tile (laid over them with one lag group).
static size_t even_mfma_lds(const Geo &g, int TR)
{
    const size_t tile = (size_t)256 * (TR + 1), stage = (size_t)TR * even_mfma_ps(g, TR);
    return (g.e3m_NMG == 1 ? std::max(tile, stage) : tile + stage) * (g.fp64 ? 8 : 4);
}

static void describe_schedule(Plan &pl)
{
    const Geo &g = pl.g;
    char buf[96];
    const char *tn = g.tuned == 1 ? " tuned" : g.tuned == 2 ? " cached" : "";
    if (g.even)
        std::snprintf(buf, sizeof buf, "%s even lags[%d,%d] slices[%d,%d) P1 R%d jc%d P3 %s TR%d%s P5 R%d%s",
                      g.fp64 ? "fp64" : "fp32c", g.m_lo, g.m_hi, g.jA, g.jB, g.e1_R, g.e1_jc,
                      g.e3_variant == 2 ? "mfma4" : g.e3_variant ? "mfma" : "direct",
                      g.e3_variant == 2 ? 16 * g.e3q_W : g.e3_variant ? g.e3m_TR : g.e3_TR, tn, g.e5_R,
                      pl.p.want_rpa ? " +kk/rpa" : "");
    else
        std::snprintf(buf, sizeof buf, "%s lags[%d,%d] slices[%d,%d) P1 R%d jc%d P3 %s TR%d%s P5 R%d%s",
                      g.fp64 ? "fp64" : "fp32c", g.m_lo, g.m_hi, g.jA, g.jB, g.p1_R, g.p1_jc,
                      g.p3_variant ? "fft" : "direct", g.p3_variant ? g.p3f_TR : g.p3_TR, tn, g.p5_R,
                      pl.p.want_rpa ? " +kk/rpa" : "");
    pl.schedule = buf;
}

lindhard_status plan_describe(const lindhard_problem *p, Plan &pl)
{
    if (!p) return LINDHARD_EINVAL;
    if (p->precision != LINDHARD_FP32C && p->precision != LINDHARD_FP64) return LINDHARD_EINVAL;
    // powers of two up to 4096; other sizes (Bluestein transforms) up to 4097
    // in FP32 and 2049 in FP64, two dimensions and one band
    const bool any_size = !is_pow2(p->nkx) || !is_pow2(p->nky);
    if (p->nkx < 4 || p->nky < 4) return LINDHARD_EINVAL;
    if (!any_size && (p->nkx > 4096 || p->nky > 4096)) return LINDHARD_EINVAL;
    if (any_size) {
        const int lim = p->precision == LINDHARD_FP64 ? 2049 : 4097;
        if (p->nkx > lim || p->nky > lim) return LINDHARD_EINVAL;
        if (p->nkz > 1 || p->n_bands > 1 || p->pair_weight) return LINDHARD_EINVAL;
    }
    if (!is_pow2(p->neps) || p->neps < 4 || p->neps > 2048) return LINDHARD_EINVAL;
    if (!std::isfinite(p->emin) || !std::isfinite(p->emax) || !(p->emin < 0.0) || !(p->emax > 0.0))
        return LINDHARD_EINVAL;
    if (!std::isfinite(p->gamma) || !(p->gamma > 0.0)) return LINDHARD_EINVAL;
    if (p->nomega < 1 || p->nomega > 65535 || !p->omega) return LINDHARD_EINVAL;
    if (p->zones_x < 1 || p->zones_y < 1 || !(p->zones_x & 1) || !(p->zones_y & 1)) return LINDHARD_EINVAL;
    if ((long)p->zones_x * p->nkx > 65536 || (long)p->zones_y * p->nky > 65535) return LINDHARD_EINVAL;
    if (p->ff_kind != LINDHARD_FF_NONE && p->ff_kind != LINDHARD_FF_GAUSS_DX2Y2) return LINDHARD_EINVAL;
    if (p->ff_kind == LINDHARD_FF_GAUSS_DX2Y2 && (!std::isfinite(p->ff_width) || !(p->ff_width > 0.0)))
        return LINDHARD_EINVAL;
    if (std::isnan(p->mu)) {
        if (!std::isfinite(p->filling) || !(p->filling > 0.0) || !(p->filling < 2.0)) return LINDHARD_EINVAL;
    } else if (!std::isfinite(p->mu)) {
        return LINDHARD_EINVAL;
    }
    const int nkz = p->nkz < 1 ? 1 : p->nkz;
    if (p->nkz < 0 || p->nkz > 256 || !is_pow2(nkz)) return LINDHARD_EINVAL;
    // three dimensions: a caller table, the first momentum zone of the k-grid,
    // and for RPA at most 65535 rows of the first-zone map (launch grid)
    if (nkz > 1 && (!p->eps_table || p->k_zones > 1 || (p->want_rpa && (long)nkz * p->nky > 65535)))
        return LINDHARD_EINVAL;
    const long nk = (long)p->nkx * p->nky * nkz;
    const int nbands = p->n_bands < 1 ? 1 : p->n_bands;
    if (p->n_bands < 0 || p->n_bands > LINDHARD_MAX_BANDS) return LINDHARD_EINVAL;
    if (nbands > 1 && !p->eps_table) return LINDHARD_EINVAL;
    const long nall = nk * nbands;
    if (p->eps_table) {
        for (long k = 0; k < nall; ++k)
            if (!std::isfinite(p->eps_table[k])) return LINDHARD_EINVAL;
    } else if (!std::isfinite(p->t) || !std::isfinite(p->tp) || !std::isfinite(p->tpp)) {
        return LINDHARD_EINVAL;
    }
    if (p->k_zones < 0 || p->k_zones > 64) return LINDHARD_EINVAL;
    if (p->rho_table)
        for (long k = 0; k < nall; ++k)
            if (!std::isfinite(p->rho_table[k])) return LINDHARD_EINVAL;
    if (p->pair_m2) {
        if (p->pair_weight || p->ff_kind != LINDHARD_FF_NONE || p->want_rpa || nkz > 1 || any_size)
            return LINDHARD_EINVAL;
        const size_t n = (size_t)nbands * nbands * p->zones_x * p->nkx * p->zones_y * p->nky;
        for (size_t i = 0; i < n; ++i)
            if (!std::isfinite(p->pair_m2[i]) || p->pair_m2[i] < 0.0) return LINDHARD_EINVAL;
    }
    if (p->pair_weight) {
        bool any = false;
        for (int i = 0; i < nbands * nbands; ++i) {
            if (!std::isfinite(p->pair_weight[i]) || p->pair_weight[i] < 0.0) return LINDHARD_EINVAL;
            any = any || p->pair_weight[i] > 0.0;
        }
        if (!any) return LINDHARD_EINVAL;
    }

    pl.p = *p;
    pl.p.omega = nullptr;
    pl.p.eps_table = nullptr;
    pl.p.rho_table = nullptr;
    pl.p.pair_weight = nullptr;
    pl.p.pair_m2 = nullptr;
    pl.p.k_zones = std::max(1, p->k_zones);
    pl.p.n_bands = nbands;
    pl.p.nkz = nkz;
    pl.has_rho = p->rho_table != nullptr;
    pl.nb = nbands;
    pl.pairs = p->pair_weight != nullptr;
    if (pl.pairs) pl.pairw.assign(p->pair_weight, p->pair_weight + nbands * nbands);
    pl.has_m2 = p->pair_m2 != nullptr;
    pl.m2_pairs.clear();
    if (pl.has_m2) {
        const size_t plane = (size_t)p->zones_x * p->nkx * p->zones_y * p->nky;
        for (int k = 0; k < nbands * nbands; ++k) {
            const double *m = p->pair_m2 + (size_t)k * plane;
            if (std::any_of(m, m + plane, [](double v) { return v != 0.0; })) pl.m2_pairs.push_back(k);
        }
        if (pl.m2_pairs.empty()) pl.m2_pairs.push_back(0);  // all zero: one pair gives the zero map
    }
    pl.omega.assign(p->omega, p->omega + p->nomega);
    pl.deps = (p->emax - p->emin) / p->neps;
    Geo &g = pl.g;
    g = Geo{};
    g.fp64 = p->precision == LINDHARD_FP64;
    g.nkx = p->nkx;
    g.nky = p->nky;
    g.logNx = ilog2(p->nkx);
    g.logNy = ilog2(p->nky);
    g.L = p->nkx / 2;
    g.logL = g.logNx - 1;
    g.C = g.fp64 ? 2 : 4;
    g.logC = ilog2(g.C);
    g.NT = g.L / g.C + 1;
    g.bs = any_size ? 1 : 0;
    if (g.bs) {
        // real rows: the columns kx <= nkx / 2 hold the whole spectrum
        g.NT = (p->nkx / 2 + 1 + g.C - 1) / g.C;
        auto clog2 = [](int v) {
            int l = 0;
            while ((1 << l) < v) ++l;
            return l;
        };
        // the chirp is even (b_-m = b_m), so the lags -(N-1) and N-1 may share
        // one place: a circular convolution of length 2N - 2 suffices
        g.logMx = clog2(2 * p->nkx - 2);
        g.logMy = clog2(2 * p->nky - 2);
        const size_t cs = g.fp64 ? 16 : 8;
        auto lines = [&](int logM, int cap) {
            const int M = 1 << logM, E = std::min(16, M), G = M / E;
            int R = 1;
            while (R * 2 <= cap && R * 2 * G <= 256 && (size_t)(R * 2) * M * cs <= 65536) R *= 2;
            return R;
        };
        g.bs_Rr = lines(g.logMx, (p->nky + 1) / 2);
        g.bs_Rc = lines(g.logMy, g.NT * g.C);
        g.bs_SJ = 8;
    }
    g.neps = p->neps;
    g.j0 = count_occupied(p->neps, p->emin, p->emax);

    // omega -> lag m (omega = m d within 1e-9 d, m >= 0); with omega_interp an
    // omega strictly between lags m and m + 1 keeps frac f = omega / d - m
    pl.lag.resize(p->nomega);
    pl.frac.assign(p->nomega, 0.0);
    int mlo = INT_MAX, mhi = -1;
    auto need = [&](long m) {
        if (m >= 1 && m < p->neps) {
            mlo = std::min(mlo, (int)m);
            mhi = std::max(mhi, (int)m);
        }
    };
    for (int w = 0; w < p->nomega; ++w) {
        const double om = p->omega[w];
        if (!std::isfinite(om)) return LINDHARD_EOFFGRID;
        const double r = om / pl.deps;
        if (r < -0.5 || r > (double)INT_MAX / 2) return LINDHARD_EOFFGRID;
        long m = std::lround(r);
        double f = 0.0;
        if (m < 0 || std::fabs(om - (double)m * pl.deps) > 1e-9 * pl.deps) {
            if (!p->omega_interp || r <= 0.0) return LINDHARD_EOFFGRID;
            m = (long)std::floor(r);
            f = r - (double)m;
            need(m + 1);
        }
        pl.lag[w] = (int)m;
        pl.frac[w] = f;
        need(m);
    }
    if (p->want_rpa) {
        mlo = 1;
        mhi = p->neps - 1;
    }
    if (mhi >= mlo) {
        g.m_lo = mlo;
        g.m_hi = mhi;
        g.nL = mhi - mlo + 1;
        g.jA = std::max(0, g.j0 - mhi);
        g.jB = std::min(p->neps, g.j0 + mhi);
        g.nS = g.jB - g.jA;
    } else {
        g.m_lo = g.m_hi = 0;
        g.nL = 0;
        g.jA = g.jB = g.nS = 0;
    }
    g.nslots = std::max(g.nS, g.nL);
    g.nkz = nkz;
    g.logNz = ilog2(nkz);
    g.plane_elems = (size_t)g.NT * g.nky * g.C;
    g.slice_elems = g.plane_elems * nkz;
    pl.src.resize(p->nomega);
    for (int w = 0; w < p->nomega; ++w) {
        auto slot_of = [&](int m) { return (g.nL > 0 && m >= g.m_lo && m <= g.m_hi) ? m - g.m_lo : -1; };
        const int m = pl.lag[w];
        const double f = pl.frac[w];
        PlaneSrc ps{slot_of(m), -1, 1.0, 0.0};
        if (f > 0.0) {
            ps.wa = 1.0 - f;
            ps.b = slot_of(m + 1);
            ps.wb = f;
            if (ps.a < 0) {  // lag m contributes 0: keep the other term alone
                ps.a = ps.b;
                ps.wa = ps.wb;
                ps.b = -1;
                ps.wb = 0.0;
            }
            if (ps.b < 0) ps.wb = 0.0;
        }
        pl.src[w] = ps;
    }

    // launch shapes
    const size_t cs = g.fp64 ? 16 : 8;
    {
        // P1: G = L / E threads per row (E = min(kP1Elems, L)), up to 256 threads
        const int E = std::min(kP1Elems, g.L), G = g.L / E;
        g.p1_R = std::min(p->nky, std::max(1, 256 / G));
        g.p1_logR = ilog2(g.p1_R);
    }
    {
        const long gx = p->nky / g.p1_R;
        long jc = (gx * std::max(g.nS, 1)) / 4096;
        g.p1_jc = (int)std::max(1L, std::min(16L, jc));
    }
    {
        int TR = 32;
        while (TR > g.C && (size_t)std::max(g.nS, 1) * TR * cs > 65536) TR >>= 1;
        TR = std::min(TR, g.C * p->nky);
        g.p3_TR = TR;
        g.p3_logTR = ilog2(TR);
        g.p3_RY = TR / g.C;
        g.p3_logRY = ilog2(g.p3_RY);
    }
    {
        // energy-window FFT variant: length 2^logNE >= nS, TR points per block
        g.logNE = std::max(1, ilog2(std::max(g.nS, 2)));
        const int NE = 1 << g.logNE;
        const int E = std::min(16, NE), G = NE / E;
        // at most 256 threads per block: the kernel needs ~170 registers, so a
        // 512-thread block fills a CU on its own and its loads, transforms and
        // stores cannot overlap with another block's (512 energies: 7.99 ->
        // 6.73 ms for the 2048^2 window)
        int TR = 32;
        while (TR > g.C && ((size_t)NE * TR * cs > 65536 || TR * G > 256)) TR >>= 1;
        TR = std::min(TR, g.C * p->nky);
        g.p3f_TR = TR;
        g.p3f_logTR = ilog2(TR);
        // direct form: complex MACs per real-space point; FFT form: ~3 transforms
        double direct = 0.0;
        for (int m = g.m_lo; m <= g.m_hi && g.nL > 0; ++m) {
            const int jl = std::max(0, g.j0 - m), jh = std::min(g.j0, p->neps - m);
            direct += std::max(0, jh - jl);
        }
        const double fftw = 3.0 * NE * (g.logNE + 1);
        g.p3_variant = direct > fftw ? 1 : 0;
        if (const char *ev = std::getenv("LINDHARD_WINDOW")) {
            if (!std::strcmp(ev, "direct")) g.p3_variant = 0;
            if (!std::strcmp(ev, "fft")) g.p3_variant = 1;
        }
    }
    if (g.bs) {
        // rows of any count: one row of C points per window block
        g.p3_TR = g.C;
        g.p3_logTR = g.logC;
        g.p3_RY = 1;
        g.p3_logRY = 0;
        g.p3f_TR = g.C;
        g.p3f_logTR = g.logC;
    }
    {
        // P5: R rows of (L + 1) complex values in LDS (<= 64 KiB), <= 256 threads
        const int E = std::min(16, g.L), G = g.L / E;
        int R = 1;
        while (R * 2 <= p->nky && R * 2 * G <= 256 && (size_t)(g.L + 1) * (R * 2) * cs <= 65536) R *= 2;
        g.p5_R = R;
        g.p5_logR = ilog2(R);
    }
    // mirror symmetry of the band -> real even transforms on the quarter plane
    {
        bool sym = true;
        // a table (band or momentum density) must be mirror symmetric bit for bit
        auto mirror = [&](const double *tab) {
            const int nx = p->nkx, ny = p->nky;
            for (int iy = 0; iy < ny; ++iy)
                for (int ix = 0; ix < nx; ++ix) {
                    const double e = tab[(size_t)iy * nx + ix];
                    if (e != tab[(size_t)iy * nx + ((nx - ix) & (nx - 1))] ||
                        e != tab[(size_t)((ny - iy) & (ny - 1)) * nx + ix])
                        return false;
                }
            return true;
        };
        if (nkz > 1 || g.bs) sym = false;  // the real even form: two dimensions, powers of two
        for (int b = 0; b < nbands && sym; ++b) {
            if (p->eps_table) sym = mirror(p->eps_table + b * nk);
            if (sym && p->rho_table) sym = mirror(p->rho_table + b * nk);
        }
        if (const char *ev = std::getenv("LINDHARD_SYMMETRY"))
            if (!std::strcmp(ev, "off")) sym = false;
        g.even = sym ? 1 : 0;
        const size_t es = g.fp64 ? 8 : 4;
        g.Ce = (int)(32 / es);
        g.logCe = ilog2(g.Ce);
        g.NTe = (g.L + 1 + g.Ce - 1) / g.Ce;
        g.Hy = p->nky / 2 + 1;
        // groups of four rows (the rows of a row-pair block) start on 128-byte lines
        g.HyS = (g.Hy + 3) & ~3;
        g.slice_e = (size_t)g.NTe * g.HyS * g.Ce;
        const int np = (g.Hy + 1) / 2;
        // row pairs per block for register FFTs of E elements per thread
        auto rows_per_block = [&](int E) {
            const int Gx = p->nkx / std::min(E, p->nkx);
            int R = std::max(1, 256 / Gx);
            // LDS: R line buffers of nkx complex (+ the FP32 twiddle table)
            while (R > 1 && (size_t)(R + (g.fp64 ? 0 : 1)) * p->nkx * cs > 65536) R >>= 1;
            R = std::min(R, 1 << ilog2(np));
            if ((1 << ilog2(np)) > np) R = std::min(R, 1 << (ilog2(np) - 1));
            return std::max(1, R);
        };
        g.e1_R = rows_per_block(e1_elems(g.logNx));
        g.e5_R = rows_per_block(16);
        if (!g.fp64 && g.logNx >= 10 && g.logNx <= 11) {
            // FP32 rows of 1024 and 2048 points (padded engine): kE5MaxThreads per block
            const int Gx = p->nkx / 16;
            g.e5_R = std::max(1, std::min(kE5MaxThreads / Gx, 1 << ilog2(np)));
            if ((1 << ilog2(np)) > np) g.e5_R = std::min(g.e5_R, 1 << (ilog2(np) - 1));
        }
        {
            const long blocks = (np + g.e1_R - 1) / g.e1_R;
            long jc = (blocks * std::max(g.nS, 1)) / 4096;
            g.e1_jc = (int)std::max(1L, std::min(16L, jc));
        }
        // even window: TR points per block, arrays P' [PL] and H' [HP + HL]
        const int nB = (g.nL + 15) / 16;
        const int HL = g.m_lo + 16 * nB - 1;
        int TR = 64;
        for (; TR > 1; TR >>= 1) {
            const int SU = 64 / TR;
            const int PL = std::min(HL, g.j0 - g.jA) + 16 * SU + 16;
            const int HP = 16 * SU + 32;
            if ((size_t)(PL + HP + HL) * TR * es <= 65536) break;
        }
        g.e3_TR = TR;
        g.e3_logTR = ilog2(TR);
        g.e3_PL = std::max(1, std::min(HL, g.j0 - g.jA) + 16 * (64 / TR) + 16);
        // matrix-core window: groups of 256 occupied energies and lags
        const int j0r = g.j0 - g.jA;
        g.e3m_nA = g.nL > 0 ? std::max(0, std::min(j0r, g.m_hi)) : 0;
        g.e3m_NAG = std::max(1, (g.e3m_nA + 255) / 256);
        g.e3m_PA = 256 * g.e3m_NAG;
        g.e3m_nHe = g.nL > 0 ? std::max(0, std::min(g.nS - j0r, g.m_hi)) : 0;
        g.e3m_NMG = (g.nL + 255) / 256;
        g.e3m_PS = even_mfma_ps(g, 4);
        {
            const size_t lim = 0xFFFFFF00u, es3 = g.fp64 ? 8 : 4;
            g.e3m_buf = (size_t)g.e3m_nA * g.slice_e * es3 < lim && (size_t)g.e3m_nHe * g.slice_e * es3 < lim;
        }
        g.e3m_TR = 4;
        // rank-1 matrix window (FP32): tiles of 16 lags, chunks of 16 steps
        g.e3q_ok = 0;
        if (!g.fp64 && g.nL > 0 && g.e3m_nA > 0 && g.e3m_nHe > 0) {
            g.e3q_nT = (g.nL + 15) / 16;
            g.e3q_U0 = (g.m_lo + 14) / 16;
            g.e3q_a0 = g.m_lo + 2 - 16 * g.e3q_U0;
            g.e3q_offP = 15 - g.e3q_a0;
            g.e3q_umax = std::min((g.e3m_nA - g.e3q_a0 + 14) / 16, g.e3q_nT - 1 + g.e3q_U0);
            g.e3q_cmax = std::min((g.e3m_nHe + 2) / 16, g.e3q_nT - 1 + g.e3q_U0);
            // P' row: 16 zeros, then P'[a] at 16 + offP + a, zeros up to the
            // set u = umax + 1 (out-of-range sets read zeros, no branch)
            g.e3q_LP = 16 * g.e3q_umax + 60;
            g.e3q_LH = 16 * g.e3q_cmax + 20;
            g.e3q_nAst = std::max(0, std::min(g.e3m_nA, g.e3q_LP - 16 - g.e3q_offP));
            g.e3q_nHst = std::max(0, std::min(g.e3m_nHe, g.e3q_LH - 3));
            g.e3q_PSP = g.e3q_LP + (((16 - g.e3q_LP) % 32) + 32) % 32;
            g.e3q_PSH = g.e3q_LH + (((4 - g.e3q_LH) % 32) + 32) % 32;
            g.e3q_W = 1;
            // byte offsets of the buffer loads and stores stay below 4 GiB
            // (the zero rows of the staging wrap to offsets past the range)
            const double sl4 = (double)g.slice_e * 4.0, lim = 4294967040.0;
            const bool fits32 = (g.e3q_nAst + 96) * sl4 < lim && (g.e3q_nHst + 96) * sl4 < lim && g.nL * sl4 < lim;
            g.e3q_big = fits32 ? 0 : 1;  // else 64-bit addresses
            g.e3q_ok = g.e3q_umax >= 0 && e3q_lds_bytes(g, 1) <= 65536;
        }
        g.e3_variant = 0;
        if (const char *ev = std::getenv("LINDHARD_EVEN_WINDOW")) {
            if (!std::strcmp(ev, "mfma") && even_mfma_lds(g, 4) <= 65536) g.e3_variant = 1;
            if (!std::strcmp(ev, "mfma4") && g.e3q_ok) g.e3_variant = 2;
        }
    }

    if (p->want_rpa) {
        // Kramers-Kronig rows: every lag an omega reads (and the next one
        // for an omega between lags), by parity in tiles of 16
        std::vector<int> need;
        for (int w = 0; w < p->nomega; ++w) {
            need.push_back(pl.lag[w]);
            if (pl.frac[w] > 0.0) need.push_back(pl.lag[w] + 1);
        }
        std::sort(need.begin(), need.end());
        need.erase(std::unique(need.begin(), need.end()), need.end());
        pl.kk_lags = need;
        pl.kk_rows.clear();
        for (int par = 0; par < 2; ++par) {
            int n = 0;
            for (size_t s = 0; s < need.size(); ++s)
                if ((need[s] & 1) == par) {
                    pl.kk_rows.push_back(make_int2(need[s], (int)s));
                    ++n;
                }
            while (n % 16) {
                pl.kk_rows.push_back(make_int2(-1, -1));
                ++n;
            }
        }
        pl.kk_ntiles = (int)pl.kk_rows.size() / 16;
        pl.kk_nch = (p->neps + 31) / 32;
        pl.kk_slot.assign((size_t)2 * p->nomega, -1);
        auto slot = [&](int m) { return (int)(std::lower_bound(need.begin(), need.end(), m) - need.begin()); };
        for (int w = 0; w < p->nomega; ++w) {
            pl.kk_slot[2 * w] = slot(pl.lag[w]);
            if (pl.frac[w] > 0.0) pl.kk_slot[2 * w + 1] = slot(pl.lag[w] + 1);
        }
    }

    pl.zx = p->zones_x;
    pl.zy = p->zones_y;
    pl.out_nx = p->zones_x * p->nkx;
    pl.out_ny = p->zones_y * p->nky * nkz;  // three dimensions: nkz blocks of zones_y * nky rows
    pl.out_elems = (size_t)p->nomega * pl.out_nx * pl.out_ny;
    pl.elem_bytes = g.fp64 ? 8 : 4;
    pl.scale = -pl.deps / ((double)nk * (double)nk);
    pl.ff_s = p->ff_kind == LINDHARD_FF_GAUSS_DX2Y2 ? p->ff_width * p->ff_width / 4.0 : 0.0;
    pl.ws_bytes = plan_footprint(pl);
    describe_schedule(pl);
    return LINDHARD_OK;
}

// Plan scratch: the partial sums of the mu solve, or those of the q-average.
static size_t scratch_bytes(const Plan &pl)
{
    return std::max<size_t>(2 * kOccBlocks + 2, (size_t)pl.p.nomega * kQavgBlocks) * sizeof(double);
}

// The device buffers of a plan in a fixed order, each with its size for the
// plan's geometry (0: not needed).  Planning allocates them; rebinding a
// cached plan to another problem of its class grows the ones that are short.
std::vector<BufSpec> plan_buffers(const Plan &cpl)
{
    Plan &pl = const_cast<Plan &>(cpl);
    const Geo &g = pl.g;
    const size_t cs = g.fp64 ? 16 : 8, es = g.fp64 ? 8 : 4;
    const size_t nk = (size_t)g.nkx * g.nky * g.nkz;
    const size_t sl = g.even ? g.slice_e * es : g.slice_elems * cs;  // bytes per slice
    const bool pair_ws = pl.pairs && g.nL > 0, rpa = pl.p.want_rpa != 0;
    const bool band_ws = (pl.pairs || (pl.has_m2 && pl.nb > 1)) && g.nL > 0;  // per-band spectra
    const size_t Mx = g.bs ? ((size_t)1 << g.logMx) * cs : 0, My = g.bs ? ((size_t)1 << g.logMy) * cs : 0;
    const size_t nw = (size_t)pl.p.nomega;
    return {
        {(void **)&pl.xi, nk * 8 * pl.nb},
        {&pl.rho, pl.has_rho ? nk * es * pl.nb : 0},
        {&pl.bspec, band_ws ? (size_t)pl.nb * g.nS * sl : 0},
        {&pl.sacc, pair_ws ? (size_t)g.nL * sl : 0},
        {&pl.twx, g.nkx * cs},
        {&pl.twy, g.nky * cs},
        {&pl.twz, g.nkz * cs},
        {&pl.bsx[0], g.bs ? g.nkx * cs : 0},
        {&pl.bsy[0], g.bs ? g.nky * cs : 0},
        {&pl.bsx[1], Mx}, {&pl.bsx[2], Mx}, {&pl.bsx[3], Mx},
        {&pl.bsy[1], My}, {&pl.bsy[2], My}, {&pl.bsy[3], My},
        {&pl.twe, ((size_t)1 << g.logNE) * cs},
        {(void **)&pl.ffx, (size_t)pl.out_nx * 16},
        {(void **)&pl.ffy, (size_t)pl.out_ny * 16},
        {(void **)&pl.d_src, nw * sizeof(PlaneSrc)},
        {(void **)&pl.d_frac, nw * sizeof(double)},
        {(void **)&pl.d_lag, nw * sizeof(int)},
        {&pl.spec, (size_t)g.nslots * sl},
        {(void **)&pl.scratch, scratch_bytes(pl)},
        {&pl.im1, rpa ? (size_t)g.neps * nk * es : 0},
        {&pl.re1, rpa ? pl.kk_lags.size() * nk * es : 0},
        {(void **)&pl.kkw, rpa ? (size_t)pl.kk_ntiles * 16 * pl.kk_nch * 16 * 8 : 0},
        {(void **)&pl.d_kkrow, rpa ? pl.kk_rows.size() * sizeof(int2) : 0},
        {(void **)&pl.d_kkslot, rpa ? pl.kk_slot.size() * sizeof(int) : 0},
        {&pl.m2, pl.has_m2 ? (size_t)pl.nb * pl.nb * pl.out_nx * pl.out_ny * es : 0},
    };
}

size_t plan_footprint(const Plan &pl)
{
    size_t b = 0;
    for (const BufSpec &r : plan_buffers(pl)) b += (r.bytes + 255) & ~(size_t)255;
    return b;
}

// ------------------------------------------------------------ device pool
// Plans take their device buffers from a per-process pool of exact-size
// buckets instead of hipMalloc / hipFree: a served job then allocates
// nothing in the common case, and no hipFree (which waits for the whole
// device) sits between concurrent jobs.  Buffers return to the pool when the
// plan is destroyed, after its last work has completed.  Sizes are rounded up
// (power of two below 1 MiB, 1 MiB multiples above); the pool keeps at most
// LINDHARD_POOL_LIMIT bytes (default 64 GiB) of idle buffers.
namespace {
std::mutex g_dpool_mu;
std::multimap<std::pair<int, size_t>, void *> g_dpool;
size_t g_dpool_idle = 0;

size_t pool_round(size_t b)
{
    if (b == 0) b = 256;
    if (b < (1u << 20)) {
        size_t r = 256;
        while (r < b) r <<= 1;
        return r;
    }
    return (b + (1u << 20) - 1) & ~(size_t)((1u << 20) - 1);
}

size_t pool_limit()
{
    const char *e = std::getenv("LINDHARD_POOL_LIMIT");
    return e ? (size_t)std::strtoull(e, nullptr, 10) : ((size_t)64 << 30);
}
}  // namespace

static hipError_t pool_alloc(void **p, size_t bytes, int device)
{
    const size_t b = pool_round(bytes);
    {
        std::lock_guard<std::mutex> lk(g_dpool_mu);
        auto it = g_dpool.find({device, b});
        if (it != g_dpool.end()) {
            *p = it->second;
            g_dpool.erase(it);
            g_dpool_idle -= b;
            return hipSuccess;
        }
    }
    hipError_t e = hipMalloc(p, b);
    if (e == hipErrorOutOfMemory) {
        // give idle buffers back to the device and retry once
        std::vector<void *> drop;
        {
            std::lock_guard<std::mutex> lk(g_dpool_mu);
            for (auto it = g_dpool.begin(); it != g_dpool.end();) {
                if (it->first.first == device) {
                    drop.push_back(it->second);
                    g_dpool_idle -= it->first.second;
                    it = g_dpool.erase(it);
                } else {
                    ++it;
                }
            }
        }
        (void)hipGetLastError();
        for (void *q : drop) (void)hipFree(q);
        e = hipMalloc(p, b);
    }
    if (e != hipSuccess) *p = nullptr;
    return e;
}

static void pool_free(void *p, size_t bytes, int device)
{
    if (!p) return;
    const size_t b = pool_round(bytes);
    bool keep = false;
    {
        std::lock_guard<std::mutex> lk(g_dpool_mu);
        if (g_dpool_idle + b <= pool_limit()) {
            g_dpool.insert({{device, b}, p});
            g_dpool_idle += b;
            keep = true;
        }
    }
    if (!keep) (void)hipFree(p);
}

void plan_free(Plan &pl)
{
    for (auto &a : pl.allocs) pool_free(a.first, a.second, pl.device);
    pl.allocs.clear();
    void **ptrs[] = {(void **)&pl.xi,     (void **)&pl.twx,  (void **)&pl.twy, &pl.twz, &pl.twe, (void **)&pl.ffx,
                     (void **)&pl.ffy,    (void **)&pl.d_src, (void **)&pl.d_lag, (void **)&pl.d_frac, &pl.spec,
                     &pl.im1,             &pl.re1,           (void **)&pl.kkw, (void **)&pl.scratch,
                     &pl.rho,              &pl.bspec,         &pl.sacc,         &pl.bsx[0], &pl.bsx[1], &pl.bsx[2], &pl.bsx[3],
                     &pl.bsy[0],           &pl.bsy[1],        &pl.bsy[2], &pl.bsy[3], (void **)&pl.d_kkrow,
                     (void **)&pl.d_kkslot, &pl.m2};
    for (void **p : ptrs) *p = nullptr;
}

#define LH_TRY(x)                                                                                         \
    do {                                                                                                   \
        hipError_t e_ = (x);                                                                               \
        if (e_ != hipSuccess) return e_ == hipErrorOutOfMemory ? LINDHARD_ENOMEM : LINDHARD_EDEVICE;       \
    } while (0)

static lindhard_status dalloc(Plan &pl, void **p, size_t bytes)
{
    hipError_t e = pool_alloc(p, bytes, pl.device);
    if (e != hipSuccess) {
        (void)hipGetLastError();
        return e == hipErrorOutOfMemory ? LINDHARD_ENOMEM : LINDHARD_EDEVICE;
    }
    pl.allocs.push_back({*p, bytes});
    return LINDHARD_OK;
}

// ------------------------------------------------------------ autotuner
// The energy-window pass has several schedules: the direct and the energy-FFT
// form on the general path, and the points-per-block width on the even path.
// The first plan of a shape times each candidate on its own workspace (the
// timing does not depend on the data) and keeps the fastest; the decision is
// cached per process, and in the text file LINDHARD_TUNE_CACHE if set.
// LINDHARD_AUTOTUNE=0 keeps the built-in heuristics; LINDHARD_WINDOW forces
// the general-path form.
namespace {
std::mutex g_tune_mu;
std::condition_variable g_tune_cv;
std::map<std::string, std::pair<int, int>> g_tune;  // key -> (variant, TR)
std::set<std::string> g_tune_busy;                  // keys being timed right now
bool g_tune_loaded = false;

// Marks a key as being timed; clears the mark (and wakes the plans waiting
// for it) on every way out of the timing.
struct TuneBusy {
    std::string key;
    explicit TuneBusy(const std::string &k) : key(k) { g_tune_busy.insert(k); }
    ~TuneBusy()
    {
        {
            std::lock_guard<std::mutex> lk(g_tune_mu);
            g_tune_busy.erase(key);
        }
        g_tune_cv.notify_all();
    }
};

bool even_tr_fits(const Geo &g, int TR);

std::string tune_key(const Geo &g)
{
    char b[160];
    // the widest points-per-block that fits LDS fixes the candidate set
    int maxfit = 0;
    if (g.even)
        for (int TR = 64; TR >= 1 && !maxfit; TR >>= 1)
            if (even_tr_fits(g, TR)) maxfit = TR;
    // lag ranges are bucketed (32 lags) so that served jobs of one grid share
    // decisions; a cached width that does not fit the plan is re-timed
    int maxfit_m = 0;
    if (g.even)
        for (int TR = 32; TR >= 4 && !maxfit_m; TR >>= 1)
            if (even_mfma_lds(g, TR) <= 65536) maxfit_m = TR;
    const char *ev = g.even ? std::getenv("LINDHARD_EVEN_WINDOW") : nullptr;
    std::snprintf(b, sizeof b, "w5 %d %d %d %d %d %d %d %d %d %d %d %s z%d", g.even, g.fp64, g.nkx, g.nky, g.neps,
                  g.j0, g.m_lo, (g.m_hi + 31) / 32, maxfit, maxfit_m, g.e3q_ok, ev ? ev : "auto", g.nkz);
    return b;
}

void tune_load_file()
{
    if (g_tune_loaded) return;
    g_tune_loaded = true;
    const char *path = std::getenv("LINDHARD_TUNE_CACHE");
    if (!path) return;
    FILE *f = std::fopen(path, "r");
    if (!f) return;
    char line[256];
    while (std::fgets(line, sizeof line, f)) {
        char *bar = std::strchr(line, '|');
        if (!bar) continue;
        *bar = 0;
        int v = 0, tr = 0;
        if (std::sscanf(bar + 1, "%d %d", &v, &tr) == 2) g_tune[line] = {v, tr};
    }
    std::fclose(f);
}

void tune_store_file(const std::string &key, int v, int tr)
{
    const char *path = std::getenv("LINDHARD_TUNE_CACHE");
    if (!path) return;
    FILE *f = std::fopen(path, "a");
    if (!f) return;
    std::fprintf(f, "%s|%d %d\n", key.c_str(), v, tr);
    std::fclose(f);
}

int ilog2c(int v)
{
    int r = 0;
    while ((1 << r) < v) ++r;
    return r;
}

void set_even_tr(Geo &g, int TR)
{
    const int nB = (g.nL + 15) / 16;
    const int HL = g.m_lo + 16 * nB - 1;
    g.e3_TR = TR;
    g.e3_logTR = ilog2c(TR);
    g.e3_PL = std::max(1, std::min(HL, g.j0 - g.jA) + 16 * (64 / TR) + 16);
}

// An even-window schedule: variant 0 direct (TR points per block), 1 matrix cores.
void set_even(Geo &g, int variant, int TR)
{
    g.e3_variant = variant;
    if (variant == 2) {
        g.e3q_W = TR / 16;
    } else if (variant == 1) {
        g.e3m_TR = TR;
        g.e3m_PS = even_mfma_ps(g, TR);
    } else
        set_even_tr(g, TR);
}

bool even_fits(const Geo &g, int variant, int TR)
{
    if (variant == 2) return g.e3q_ok && TR == 16 && e3q_lds_bytes(g, 1) <= 65536;
    if (variant == 1) return TR >= 4 && TR <= 32 && even_mfma_lds(g, TR) <= 65536;
    return even_tr_fits(g, TR);
}

bool even_tr_fits(const Geo &g, int TR)
{
    const int nB = (g.nL + 15) / 16;
    const int HL = g.m_lo + 16 * nB - 1;
    const int SU = 64 / TR;
    const size_t es = g.fp64 ? 8 : 4;
    const int PL = std::min(HL, g.j0 - g.jA) + 16 * SU + 16;
    return (size_t)(PL + 16 * SU + 32 + HL) * TR * es <= 65536;
}
}  // namespace

static lindhard_status autotune_window(Plan &pl, hipStream_t st)
{
    Geo &g = pl.g;
    if (g.nL == 0) return LINDHARD_OK;
    const char *at = std::getenv("LINDHARD_AUTOTUNE");
    if (at && !std::strcmp(at, "0")) return LINDHARD_OK;
    const bool forced = !g.even && std::getenv("LINDHARD_WINDOW") != nullptr;
    if (forced) return LINDHARD_OK;
    const std::string key = tune_key(g);
    // One decision per shape for the whole process.  A shape is timed by one
    // plan at a time: concurrent plans of that shape (served jobs) wait for
    // its decision and take it, which keeps their results bit-identical,
    // while plans of other shapes go on (the lock is not held while timing).
    std::unique_lock<std::mutex> lk(g_tune_mu);
    tune_load_file();
    for (;;) {
        auto it = g_tune.find(key);
        if (it != g_tune.end() && (!g.even || even_fits(g, it->second.first, it->second.second))) {
            if (g.even)
                set_even(g, it->second.first, it->second.second);
            else
                g.p3_variant = it->second.first;
            g.tuned = 2;
            return LINDHARD_OK;
        }
        if (!g_tune_busy.count(key)) break;
        g_tune_cv.wait(lk);
    }
    TuneBusy busy(key);
    lk.unlock();
    std::vector<std::pair<int, int>> cands;
    if (g.even) {
        const char *ev = std::getenv("LINDHARD_EVEN_WINDOW");
        const bool want_direct = !ev || !std::strcmp(ev, "direct");
        const bool want_mfma = !ev || !std::strcmp(ev, "mfma");
        const bool want_mfma4 = !ev || !std::strcmp(ev, "mfma4");
        if (want_direct)
            for (int TR = 64, n = 0; TR >= 1 && n < 3; TR >>= 1)
                if (even_tr_fits(g, TR)) {
                    cands.push_back({0, TR});
                    ++n;
                }
        if (want_mfma)
            for (int TR = 32, n = 0; TR >= 4 && n < 2; TR >>= 1)
                if (even_fits(g, 1, TR)) {
                    cands.push_back({1, TR});
                    ++n;
                }
        if (want_mfma4 && even_fits(g, 2, 16)) cands.push_back({2, 16});
        if (cands.empty()) cands.push_back({0, g.e3_TR});
    } else {
        cands.push_back({0, 0});
        cands.push_back({1, 0});
    }
    if (cands.size() == 1 && g.even) set_even(g, cands[0].first, cands[0].second);
    if (cands.size() > 1) {
        hipEvent_t e0 = nullptr, e1 = nullptr;
        LH_TRY(hipEventCreate(&e0));
        LH_TRY(hipEventCreate(&e1));
        float best = 1e30f;
        std::pair<int, int> pick = cands[0];
        const Geo keep = g;
        for (const auto &c : cands) {
            if (g.even)
                set_even(g, c.first, c.second);
            else
                g.p3_variant = c.first;
            float tmin = 1e30f;
            for (int rep = 0; rep < 3; ++rep) {
                LH_TRY(hipEventRecord(e0, st));
                LH_TRY(launch_window(pl, st));
                LH_TRY(hipEventRecord(e1, st));
                LH_TRY(hipEventSynchronize(e1));
                float ms = 0.f;
                LH_TRY(hipEventElapsedTime(&ms, e0, e1));
                if (rep > 0) tmin = std::min(tmin, ms);
            }
            if (tmin < best) {
                best = tmin;
                pick = c;
            }
            g = keep;
        }
        (void)hipEventDestroy(e0);
        (void)hipEventDestroy(e1);
        if (g.even)
            set_even(g, pick.first, pick.second);
        else
            g.p3_variant = pick.first;
        g.tuned = 1;
        std::lock_guard<std::mutex> lk2(g_tune_mu);
        g_tune[key] = pick;
        tune_store_file(key, pick.first, pick.second);
    }
    return LINDHARD_OK;
}

static lindhard_status solve_mu(Plan &pl, hipStream_t st, double band_lo, double band_hi)
{
    // Safeguarded Newton on n(mu) - filling with the bracket
    // [min eps - 100, max eps + 100]; n and dn/dmu are FP64 device reductions.
    double *d2 = pl.scratch + 2 * kOccBlocks;
    double lo = band_lo - 100.0, hi = band_hi + 100.0;
    double mu = 0.5 * (band_lo + band_hi);
    const double f0 = pl.p.filling;
    double h2[2];
    int it = 0;
    for (; it < 200; ++it) {
        LH_TRY(launch_occ(pl, mu, d2, st));
        LH_TRY(hipMemcpyAsync(h2, d2, 2 * sizeof(double), hipMemcpyDeviceToHost, st));
        LH_TRY(hipStreamSynchronize(st));
        const double f = h2[0] - f0, df = h2[1];
        if (f == 0.0) break;
        if (f < 0.0)
            lo = mu;
        else
            hi = mu;
        double nxt = (df > 0.0) ? mu - f / df : 0.5 * (lo + hi);
        if (!(nxt > lo && nxt < hi)) nxt = 0.5 * (lo + hi);
        const double step = std::fabs(nxt - mu);
        mu = nxt;
        if (step <= 4e-16 * std::max(1.0, std::fabs(mu)) || hi - lo <= 1e-15) break;
    }
    pl.mu_iters = it + 1;
    if (it >= 200) return LINDHARD_ENOCONV;
    pl.mu = mu;
    return LINDHARD_OK;
}

lindhard_status plan_build(Plan &pl, hipStream_t st)
{
    (void)st;
    for (const BufSpec &r : plan_buffers(pl)) {
        if (!r.bytes) continue;
        const lindhard_status s = dalloc(pl, r.ptr, r.bytes);
        if (s != LINDHARD_OK) return s;
    }
    return LINDHARD_OK;
}

}  // namespace lh

using namespace lh;

struct lindhard_plan_s {
    Plan pl;
    hipStream_t setup = nullptr;
    hipEvent_t done = nullptr;  // recorded after each exec / rpa
    int32_t *d_cut = nullptr;   // staged (X, Y) pairs of lindhard_cut (owned by pl.allocs)
    size_t cut_cap = 0;
    std::string key;            // class key (plan caching in the server)
    std::vector<size_t> cap;    // allocated bytes of each buffer of plan_buffers
};

// One setup stream per host thread and device, kept for the life of the
// thread: plans built on a thread reuse it (plan building is synchronous).
static hipStream_t thread_setup_stream(int device)
{
    thread_local std::vector<std::pair<int, hipStream_t>> streams;
    for (auto &d : streams)
        if (d.first == device) return d.second;
    hipStream_t st = nullptr;
    if (hipStreamCreateWithFlags(&st, hipStreamNonBlocking) != hipSuccess) return nullptr;
    streams.push_back({device, st});
    return st;
}

// In-place FFT of a power-of-two length in FP64 (host; plan tables only).
static void fft_host(std::vector<std::complex<double>> &a)
{
    const size_t n = a.size();
    for (size_t i = 1, j = 0; i < n; ++i) {
        size_t bit = n >> 1;
        for (; j & bit; bit >>= 1) j ^= bit;
        j ^= bit;
        if (i < j) std::swap(a[i], a[j]);
    }
    for (size_t len = 2; len <= n; len <<= 1) {
        for (size_t k = 0; k < len / 2; ++k) {
            const double ang = -2.0 * M_PI * (double)k / (double)len;
            const std::complex<double> w(std::cos(ang), std::sin(ang));
            for (size_t i = 0; i < n; i += len) {
                const std::complex<double> u = a[i + k], v = a[i + k + len / 2] * w;
                a[i + k] = u + v;
                a[i + k + len / 2] = u - v;
            }
        }
    }
}

// Bluestein tables of one axis of length n (a grid of any size): chirp
// b_k = exp(i pi (k^2 mod 2n) / n), the spectra FFT_M(B) / M and FFT_M(conj B) / M
// of the chirp sequence B (B_m = b_m = B_(M-m) for m < n, zero between; with
// M = 2n - 2 the place n - 1 serves both m = n - 1 and m = -(n - 1)), and
// the FFT twiddles exp(-2 pi i s / M); FP64, rounded once to the precision.
// `keep` holds the host arrays until the copies have run.
static hipError_t bs_tables(const Plan &pl, int n, int logM, void *const *dst, hipStream_t st,
                            std::vector<std::vector<double>> &keep)
{
    const size_t M = (size_t)1 << logM;
    std::vector<std::complex<double>> b(n), B(M, 0.0), Bc(M, 0.0), tw(M);
    for (int k = 0; k < n; ++k) {
        const double ang = M_PI * (double)(((long)k * k) % (2L * n)) / (double)n;
        b[k] = std::complex<double>(std::cos(ang), std::sin(ang));
    }
    for (int m = 0; m < n; ++m) {
        B[m] = b[m];
        if (m > 0) B[M - m] = b[m];
    }
    for (size_t m = 0; m < M; ++m) Bc[m] = std::conj(B[m]);
    fft_host(B);
    fft_host(Bc);
    for (size_t s = 0; s < M; ++s) {
        const double ang = -2.0 * M_PI * (double)s / (double)M;
        tw[s] = std::complex<double>(std::cos(ang), std::sin(ang));
    }
    const std::vector<std::complex<double>> *src[4] = {&b, &B, &Bc, &tw};
    const double sc[4] = {1.0, 1.0 / (double)M, 1.0 / (double)M, 1.0};
    for (int i = 0; i < 4; ++i) {
        const auto &v = *src[i];
        const size_t nv = 2 * v.size();  // interleaved (re, im)
        // one host array per table, in the plan's precision (FP32 pairs are
        // packed into the storage of nv / 2 doubles)
        keep.emplace_back(pl.g.fp64 ? nv : nv / 2);
        double *hd = keep.back().data();
        float *hf = reinterpret_cast<float *>(hd);
        for (size_t k = 0; k < v.size(); ++k) {
            const double re = v[k].real() * sc[i], im = v[k].imag() * sc[i];
            if (pl.g.fp64) {
                hd[2 * k] = re;
                hd[2 * k + 1] = im;
            } else {
                hf[2 * k] = (float)re;
                hf[2 * k + 1] = (float)im;
            }
        }
        const hipError_t e = hipMemcpyAsync(dst[i], hd, nv * (pl.g.fp64 ? sizeof(double) : sizeof(float)),
                                            hipMemcpyHostToDevice, st);
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}

// Band-dependent state of a plan: the band (caller table or tight-binding),
// momentum-density and band-pair weights, the chemical potential and
// xi = eps - mu, on stream st (synchronous: the host tables may go after).
static lindhard_status plan_bind_band(Plan &pl, const lindhard_problem *p, hipStream_t st)
{
    pl.p.t = p->t;
    pl.p.tp = p->tp;
    pl.p.tpp = p->tpp;
    pl.p.mu = p->mu;
    pl.p.filling = p->filling;
    pl.p.gamma = p->gamma;
    if (pl.pairs) pl.pairw.assign(p->pair_weight, p->pair_weight + pl.nb * pl.nb);
    std::vector<float> m2_32;
    if (pl.has_m2) {
        // the pair maps, rounded once to the plan's precision
        const size_t n = (size_t)pl.nb * pl.nb * pl.out_nx * pl.out_ny;
        if (pl.g.fp64) {
            LH_TRY(hipMemcpyAsync(pl.m2, p->pair_m2, n * sizeof(double), hipMemcpyHostToDevice, st));
        } else {
            m2_32.assign(p->pair_m2, p->pair_m2 + n);
            LH_TRY(hipMemcpyAsync(pl.m2, m2_32.data(), n * sizeof(float), hipMemcpyHostToDevice, st));
        }
    }
    const size_t nk = (size_t)pl.g.nkx * pl.g.nky * pl.g.nkz;
    double band_lo = 0.0, band_hi = 0.0;
    const size_t nall = nk * pl.nb;
    if (p->eps_table) {
        // the caller's table is read during planning only
        LH_TRY(hipMemcpyAsync(pl.xi, p->eps_table, nall * sizeof(double), hipMemcpyHostToDevice, st));
        band_lo = *std::min_element(p->eps_table, p->eps_table + nall);
        band_hi = *std::max_element(p->eps_table, p->eps_table + nall);
    } else {
        LH_TRY(launch_band(pl, nullptr, st));
        const double bnd = 4.0 * (std::fabs(p->t) + std::fabs(p->tp) + std::fabs(p->tpp));
        band_lo = -bnd;
        band_hi = bnd;
    }
    std::vector<float> rho32;
    if (p->rho_table) {
        // momentum-density weights, rounded once to the plan's precision
        if (pl.g.fp64) {
            LH_TRY(hipMemcpyAsync(pl.rho, p->rho_table, nall * sizeof(double), hipMemcpyHostToDevice, st));
        } else {
            rho32.assign(p->rho_table, p->rho_table + nall);
            LH_TRY(hipMemcpyAsync(pl.rho, rho32.data(), nall * sizeof(float), hipMemcpyHostToDevice, st));
        }
    }
    if (std::isnan(p->mu)) {
        const lindhard_status s = solve_mu(pl, st, band_lo, band_hi);
        if (s != LINDHARD_OK) return s;
    } else {
        pl.mu = p->mu;
        pl.mu_iters = 0;
    }
    LH_TRY(launch_xi_shift(pl, pl.mu, st));
    LH_TRY(hipStreamSynchronize(st));
    return LINDHARD_OK;
}

// Omega-dependent state: lag, fraction and window slot of every omega, and
// the Kramers-Kronig weights of an RPA plan (asynchronous on st; the host
// vectors live in the plan).
static lindhard_status plan_bind_omega(Plan &pl, hipStream_t st)
{
    LH_TRY(hipMemcpyAsync(pl.d_src, pl.src.data(), pl.src.size() * sizeof(PlaneSrc), hipMemcpyHostToDevice, st));
    LH_TRY(hipMemcpyAsync(pl.d_frac, pl.frac.data(), pl.frac.size() * sizeof(double), hipMemcpyHostToDevice, st));
    LH_TRY(hipMemcpyAsync(pl.d_lag, pl.lag.data(), pl.lag.size() * sizeof(int), hipMemcpyHostToDevice, st));
    if (pl.p.want_rpa) {
        LH_TRY(hipMemcpyAsync(pl.d_kkrow, pl.kk_rows.data(), pl.kk_rows.size() * sizeof(int2), hipMemcpyHostToDevice,
                              st));
        LH_TRY(hipMemcpyAsync(pl.d_kkslot, pl.kk_slot.data(), pl.kk_slot.size() * sizeof(int), hipMemcpyHostToDevice,
                              st));
    }
    return LINDHARD_OK;
}

static lindhard_status build_plan_object(const lindhard_problem *p, lindhard_plan_s *o)
{
    Plan &pl = o->pl;
    lindhard_status s = plan_describe(p, pl);
    if (s != LINDHARD_OK) return s;
    if (hipGetDevice(&pl.device) != hipSuccess) return LINDHARD_EDEVICE;
    o->setup = thread_setup_stream(pl.device);
    if (!o->setup) return LINDHARD_EDEVICE;
    if (hipEventCreateWithFlags(&o->done, hipEventDisableTiming) != hipSuccess) return LINDHARD_EDEVICE;
    hipStream_t st = o->setup;
    s = plan_build(pl, st);
    if (s != LINDHARD_OK) return s;
    s = plan_bind_band(pl, p, st);
    if (s != LINDHARD_OK) return s;
    s = plan_bind_omega(pl, st);
    if (s != LINDHARD_OK) return s;
    LH_TRY(launch_tables(pl, st));
    std::vector<std::vector<double>> keep;
    if (pl.g.bs) {
        LH_TRY(bs_tables(pl, pl.g.nkx, pl.g.logMx, pl.bsx, st, keep));
        LH_TRY(bs_tables(pl, pl.g.nky, pl.g.logMy, pl.bsy, st, keep));
    }
    const size_t nk = (size_t)pl.g.nkx * pl.g.nky * pl.g.nkz;
    if (pl.p.want_rpa)
        LH_TRY(hipMemsetAsync(pl.im1, 0, (size_t)pl.g.neps * nk * pl.elem_bytes, st));
    if (pl.g.even) {
        // the padding rows of the tiles (ry >= Hy) are carried through the
        // window but never read back; keep them zero rather than stale
        const size_t sl = pl.g.slice_e * pl.elem_bytes;
        LH_TRY(hipMemsetAsync(pl.spec, 0, (size_t)pl.g.nslots * sl, st));
        if (pl.bspec) LH_TRY(hipMemsetAsync(pl.bspec, 0, (size_t)pl.nb * pl.g.nS * sl, st));
        if (pl.sacc) LH_TRY(hipMemsetAsync(pl.sacc, 0, (size_t)pl.g.nL * sl, st));
    }
    LH_TRY(hipStreamSynchronize(st));
    s = autotune_window(pl, st);
    if (s != LINDHARD_OK) return s;
    describe_schedule(pl);
    o->key = plan_class_key(pl);
    for (const BufSpec &r : plan_buffers(pl)) o->cap.push_back(r.bytes);
    return LINDHARD_OK;
}

namespace lh {

// Everything that fixes a plan's tables and the layout of its buffers, and
// nothing that a cached plan may change when it is rebound to another
// problem: the band, broadening, filling or chemical potential, and the omega
// list (its lag range sizes some buffers, which grow as needed).
std::string plan_class_key(const Plan &pl)
{
    const lindhard_problem &p = pl.p;
    const Geo &g = pl.g;
    char b[320];
    std::snprintf(b, sizeof b, "p%d k%dx%dx%d e%d[%a,%a] z%dx%d ff%d:%a rpa%d kz%d nb%d pr%d m2%d rho%d ev%d bs%d",
                  p.precision, g.nkx, g.nky, g.nkz, g.neps, p.emin, p.emax, p.zones_x, p.zones_y, p.ff_kind,
                  p.ff_kind ? p.ff_width : 0.0, p.want_rpa ? 1 : 0, p.k_zones, pl.nb, pl.pairs ? 1 : 0,
                  pl.has_m2 ? 1 : 0, pl.has_rho ? 1 : 0, g.even, g.bs);
    return b;
}

const std::string &plan_key(lindhard_plan_t plan) { return plan->key; }

std::vector<size_t> plan_capacity(lindhard_plan_t plan) { return plan->cap; }

size_t plan_resident_bytes(lindhard_plan_t plan)
{
    size_t b = 0;
    for (const size_t c : plan->cap) b += (c + 255) & ~(size_t)255;
    return b;
}

// Rebind a built plan to another problem of its class: the geometry of the
// new omega list, the band, mu and the tables are redone in place, buffers
// that are too small for the new geometry are replaced, and the window
// schedule is taken from the tuning cache.  The result equals that of a plan
// built for the problem afresh, bit for bit (the same geometry, schedule and
// kernels; every buffer is written before it is read).  Synchronous on st;
// the plan's earlier work must have completed.  EINVAL if the class differs.
lindhard_status plan_rebind(lindhard_plan_t plan, const lindhard_problem *p, hipStream_t st)
{
    if (!plan || !p) return LINDHARD_EINVAL;
    Plan d;
    lindhard_status s = plan_describe(p, d);
    if (s != LINDHARD_OK) return s;
    if (plan_class_key(d) != plan->key) return LINDHARD_EINVAL;
    Plan &pl = plan->pl;
    // the new description takes over the device buffers
    const std::vector<BufSpec> oldb = plan_buffers(pl);
    d.device = pl.device;
    d.allocs = std::move(pl.allocs);
    std::vector<BufSpec> nb = plan_buffers(d);
    for (size_t i = 0; i < nb.size(); ++i) *nb[i].ptr = *oldb[i].ptr;
    pl = std::move(d);
    nb = plan_buffers(pl);
    std::vector<bool> grown(nb.size(), false);
    for (size_t i = 0; i < nb.size(); ++i) {
        if (nb[i].bytes <= plan->cap[i]) continue;
        void *old = *nb[i].ptr;
        if (old) {
            for (auto it = pl.allocs.begin(); it != pl.allocs.end(); ++it)
                if (it->first == old) {
                    pool_free(it->first, it->second, pl.device);
                    pl.allocs.erase(it);
                    break;
                }
            *nb[i].ptr = nullptr;
        }
        plan->cap[i] = 0;
        s = dalloc(pl, nb[i].ptr, nb[i].bytes);
        if (s != LINDHARD_OK) return s;
        plan->cap[i] = nb[i].bytes;
        grown[i] = true;
    }
    s = plan_bind_omega(pl, st);
    if (s != LINDHARD_OK) return s;
    LH_TRY(launch_tables(pl, st));
    if (pl.g.even) {
        // replaced spectral buffers: padding rows zero, as at planning
        const size_t sl = pl.g.slice_e * pl.elem_bytes;
        for (size_t i = 0; i < nb.size(); ++i)
            if (grown[i] && (nb[i].ptr == &pl.spec || nb[i].ptr == &pl.bspec || nb[i].ptr == &pl.sacc))
                LH_TRY(hipMemsetAsync(*nb[i].ptr, 0, nb[i].bytes / sl * sl, st));
    }
    s = plan_bind_band(pl, p, st);
    if (s != LINDHARD_OK) return s;
    s = autotune_window(pl, st);
    if (s != LINDHARD_OK) return s;
    describe_schedule(pl);
    pl.executed = false;
    return LINDHARD_OK;
}

// Run plans of one even-path group (equal even_group_key) as one launch per
// pass on st: their descriptors are staged in host (kept by the caller until
// the work completes) and copied to d_desc (room for n).
hipError_t plan_exec_group(const lindhard_plan_t *plans, int n, void *const *outs, EvenInst *d_desc,
                           std::vector<EvenInst> &host, hipStream_t st)
{
    host.resize(n);
    std::vector<const Plan *> pls(n);
    for (int i = 0; i < n; ++i) {
        even_group_fill(plans[i]->pl, outs[i], host[i]);
        pls[i] = &plans[i]->pl;
    }
    hipError_t e = hipMemcpyAsync(d_desc, host.data(), n * sizeof(EvenInst), hipMemcpyHostToDevice, st);
    if (e == hipSuccess) e = launch_even_group(pls.data(), n, d_desc, st);
    for (int i = 0; i < n && e == hipSuccess; ++i) {
        e = hipEventRecord(plans[i]->done, st);
        plans[i]->pl.executed = true;
    }
    return e;
}

const Plan &plan_of(lindhard_plan_t plan) { return plan->pl; }

}  // namespace lh

extern "C" {

lindhard_status lindhard_plan(const lindhard_problem *p, lindhard_plan_t *out)
{
    if (!p || !out) return LINDHARD_EINVAL;
    *out = nullptr;
    lindhard_plan_s *o = new (std::nothrow) lindhard_plan_s();
    if (!o) return LINDHARD_ENOMEM;
    lindhard_status s = build_plan_object(p, o);
    if (s != LINDHARD_OK) {
        if (o->setup) (void)hipStreamSynchronize(o->setup);
        plan_free(o->pl);
        if (o->done) (void)hipEventDestroy(o->done);
        delete o;
        (void)hipGetLastError();
        return s;
    }
    *out = o;
    return LINDHARD_OK;
}

lindhard_status lindhard_problem_shape(const lindhard_problem *p, int32_t *nomega, int32_t *out_ny, int32_t *out_nx,
                                       int32_t *elem_bytes)
{
    if (!p || !nomega || !out_ny || !out_nx || !elem_bytes) return LINDHARD_EINVAL;
    Plan pl;
    const lindhard_status s = plan_describe(p, pl);
    if (s != LINDHARD_OK) return s;
    *nomega = pl.p.nomega;
    *out_ny = pl.out_ny;
    *out_nx = pl.out_nx;
    *elem_bytes = (int32_t)pl.elem_bytes;
    return LINDHARD_OK;
}

lindhard_status lindhard_plan_info(lindhard_plan_t plan, lindhard_info *info)
{
    if (!plan || !info) return LINDHARD_EINVAL;
    const Plan &pl = plan->pl;
    std::memset(info, 0, sizeof *info);
    info->mu = pl.mu;
    info->deps = pl.deps;
    info->j0 = pl.g.j0;
    info->out_nx = pl.out_nx;
    info->out_ny = pl.out_ny;
    info->nomega = pl.p.nomega;
    info->lag_lo = pl.g.m_lo;
    info->lag_hi = pl.g.m_hi;
    info->mu_iterations = pl.mu_iters;
    info->workspace_bytes = pl.ws_bytes;
    info->out_elems = pl.out_elems;
    info->elem_bytes = pl.elem_bytes;
    std::snprintf(info->schedule, sizeof info->schedule, "%s", pl.schedule.c_str());
    return LINDHARD_OK;
}

lindhard_status lindhard_exec(lindhard_plan_t plan, void *im_chi, void *stream)
{
    if (!plan || !im_chi) return LINDHARD_EINVAL;
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) return LINDHARD_EDEVICE;
    if (dev != plan->pl.device && hipSetDevice(plan->pl.device) != hipSuccess) return LINDHARD_EDEVICE;
    hipError_t e = launch_exec(plan->pl, im_chi, (hipStream_t)stream);
    if (e == hipSuccess) e = hipEventRecord(plan->done, (hipStream_t)stream);
    if (dev != plan->pl.device) (void)hipSetDevice(dev);
    if (e != hipSuccess) return LINDHARD_EDEVICE;
    plan->pl.executed = true;
    return LINDHARD_OK;
}

lindhard_status lindhard_exec_timed(lindhard_plan_t plan, void *im_chi, void *stream, float *pass_ms)
{
    if (!plan || !im_chi || !pass_ms) return LINDHARD_EINVAL;
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) return LINDHARD_EDEVICE;
    if (dev != plan->pl.device && hipSetDevice(plan->pl.device) != hipSuccess) return LINDHARD_EDEVICE;
    hipEvent_t ev[6] = {};
    hipError_t e = hipSuccess;
    for (int i = 0; i < 6 && e == hipSuccess; ++i) e = hipEventCreate(&ev[i]);
    if (e == hipSuccess) e = launch_exec(plan->pl, im_chi, (hipStream_t)stream, ev);
    if (e == hipSuccess) e = hipEventRecord(plan->done, (hipStream_t)stream);
    if (e == hipSuccess) e = hipEventSynchronize(ev[5]);
    for (int i = 0; i < 5 && e == hipSuccess; ++i) e = hipEventElapsedTime(&pass_ms[i], ev[i], ev[i + 1]);
    for (int i = 0; i < 6; ++i)
        if (ev[i]) (void)hipEventDestroy(ev[i]);
    if (dev != plan->pl.device) (void)hipSetDevice(dev);
    if (e != hipSuccess) return LINDHARD_EDEVICE;
    plan->pl.executed = true;
    return LINDHARD_OK;
}

lindhard_status lindhard_rpa(lindhard_plan_t plan, double U, void *re_chi, void *im_rpa, void *re_rpa, void *stream)
{
    if (!plan || !std::isfinite(U)) return LINDHARD_EINVAL;
    if (!plan->pl.p.want_rpa || !plan->pl.executed) return LINDHARD_ESTATE;
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) return LINDHARD_EDEVICE;
    if (dev != plan->pl.device && hipSetDevice(plan->pl.device) != hipSuccess) return LINDHARD_EDEVICE;
    hipError_t e = launch_rpa(plan->pl, 0, U, re_chi, im_rpa, re_rpa, (hipStream_t)stream);
    if (e == hipSuccess) e = hipEventRecord(plan->done, (hipStream_t)stream);
    if (dev != plan->pl.device) (void)hipSetDevice(dev);
    return e == hipSuccess ? LINDHARD_OK : LINDHARD_EDEVICE;
}

lindhard_status lindhard_rpa_coulomb(lindhard_plan_t plan, double v, void *re_chi, void *im_rpa, void *re_rpa,
                                     void *stream)
{
    if (!plan || !std::isfinite(v)) return LINDHARD_EINVAL;
    if (!plan->pl.p.want_rpa || !plan->pl.executed) return LINDHARD_ESTATE;
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) return LINDHARD_EDEVICE;
    if (dev != plan->pl.device && hipSetDevice(plan->pl.device) != hipSuccess) return LINDHARD_EDEVICE;
    hipError_t e = launch_rpa(plan->pl, 1, v, re_chi, im_rpa, re_rpa, (hipStream_t)stream);
    if (e == hipSuccess) e = hipEventRecord(plan->done, (hipStream_t)stream);
    if (dev != plan->pl.device) (void)hipSetDevice(dev);
    return e == hipSuccess ? LINDHARD_OK : LINDHARD_EDEVICE;
}

lindhard_status lindhard_structure_factor(lindhard_plan_t plan, double kT, const void *im, void *s_out, void *stream)
{
    if (!plan || !im || !s_out || !std::isfinite(kT) || kT < 0.0) return LINDHARD_EINVAL;
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) return LINDHARD_EDEVICE;
    if (dev != plan->pl.device && hipSetDevice(plan->pl.device) != hipSuccess) return LINDHARD_EDEVICE;
    hipError_t e = launch_sqw(plan->pl, kT, im, s_out, (hipStream_t)stream);
    if (e == hipSuccess) e = hipEventRecord(plan->done, (hipStream_t)stream);
    if (dev != plan->pl.device) (void)hipSetDevice(dev);
    return e == hipSuccess ? LINDHARD_OK : LINDHARD_EDEVICE;
}

lindhard_status lindhard_q_average(lindhard_plan_t plan, const void *im, double *out, void *stream)
{
    if (!plan || !im || !out) return LINDHARD_EINVAL;
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) return LINDHARD_EDEVICE;
    if (dev != plan->pl.device && hipSetDevice(plan->pl.device) != hipSuccess) return LINDHARD_EDEVICE;
    hipError_t e = launch_qavg(plan->pl, im, out, (hipStream_t)stream);
    if (e == hipSuccess) e = hipEventRecord(plan->done, (hipStream_t)stream);
    if (dev != plan->pl.device) (void)hipSetDevice(dev);
    return e == hipSuccess ? LINDHARD_OK : LINDHARD_EDEVICE;
}

lindhard_status lindhard_peak_index(lindhard_plan_t plan, const void *im, int32_t *peak, void *stream)
{
    if (!plan || !im || !peak) return LINDHARD_EINVAL;
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) return LINDHARD_EDEVICE;
    if (dev != plan->pl.device && hipSetDevice(plan->pl.device) != hipSuccess) return LINDHARD_EDEVICE;
    hipError_t e = launch_peak(plan->pl, im, peak, (hipStream_t)stream);
    if (e == hipSuccess) e = hipEventRecord(plan->done, (hipStream_t)stream);
    if (dev != plan->pl.device) (void)hipSetDevice(dev);
    return e == hipSuccess ? LINDHARD_OK : LINDHARD_EDEVICE;
}

lindhard_status lindhard_cut(lindhard_plan_t plan, const void *im, const int32_t *X, const int32_t *Y, int32_t npts,
                             void *out, void *stream)
{
    if (!plan || !im || !X || !Y || !out || npts < 1) return LINDHARD_EINVAL;
    Plan &pl = plan->pl;
    std::vector<int32_t> xy((size_t)2 * npts);
    for (int32_t p = 0; p < npts; ++p) {
        if (X[p] < 0 || X[p] >= pl.out_nx || Y[p] < 0 || Y[p] >= pl.out_ny) return LINDHARD_EINVAL;
        xy[2 * p] = X[p];
        xy[2 * p + 1] = Y[p];
    }
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) return LINDHARD_EDEVICE;
    if (dev != pl.device && hipSetDevice(pl.device) != hipSuccess) return LINDHARD_EDEVICE;
    lindhard_status st = LINDHARD_OK;
    if ((size_t)npts > plan->cut_cap) {
        void *p = nullptr;
        st = dalloc(pl, &p, (size_t)2 * npts * sizeof(int32_t));
        if (st == LINDHARD_OK) {
            plan->d_cut = (int32_t *)p;
            plan->cut_cap = (size_t)npts;
        }
    }
    if (st == LINDHARD_OK) {
        hipError_t e = hipMemcpyAsync(plan->d_cut, xy.data(), xy.size() * sizeof(int32_t), hipMemcpyHostToDevice,
                                      (hipStream_t)stream);
        if (e == hipSuccess) e = launch_cut(pl, im, plan->d_cut, npts, out, (hipStream_t)stream);
        if (e == hipSuccess) e = hipEventRecord(plan->done, (hipStream_t)stream);
        if (e != hipSuccess) st = LINDHARD_EDEVICE;
    }
    if (dev != pl.device) (void)hipSetDevice(dev);
    return st;
}

lindhard_status lindhard_high_symmetry_path(lindhard_plan_t plan, int32_t *X, int32_t *Y, int32_t capacity,
                                            int32_t *npts)
{
    if (!plan || !X || !Y || !npts) return LINDHARD_EINVAL;
    const Plan &pl = plan->pl;
    const int kz = std::max(1, pl.p.k_zones);
    if (pl.g.nkz > 1 || pl.g.nkx != pl.g.nky || pl.g.nkx % (2 * kz)) return LINDHARD_EINVAL;
    const int h = pl.g.nkx / kz / 2, Xc = pl.out_nx / 2, Yc = pl.out_ny / 2;
    const int n = 3 * h + 1;
    *npts = n;
    if (capacity < n) return LINDHARD_EINVAL;
    int p = 0;
    auto put = [&](int x, int y) {
        X[p] = x % pl.out_nx;
        Y[p] = y % pl.out_ny;
        ++p;
    };
    for (int s = 0; s < h; ++s) put(Xc + s, Yc);          // Gamma -> X
    for (int s = 0; s < h; ++s) put(Xc + h, Yc + s);      // X -> M
    for (int s = 0; s <= h; ++s) put(Xc + h - s, Yc + h - s);  // M -> Gamma
    return LINDHARD_OK;
}

lindhard_status lindhard_zone_envelope(lindhard_plan_t plan, const void *im, int32_t omega_index, int32_t direction,
                                       double q_scale, lindhard_envelope *out, void *stream)
{
    if (!plan || !im || !out) return LINDHARD_EINVAL;
    const Plan &pl = plan->pl;
    if (omega_index < 0 || omega_index >= pl.p.nomega || (direction != 0 && direction != 1)) return LINDHARD_EINVAL;
    if (!(q_scale > 0.0) || !std::isfinite(q_scale)) return LINDHARD_EINVAL;
    if (direction == 1 && pl.g.nkx != pl.g.nky) return LINDHARD_EINVAL;
    if (pl.g.nkz > 1) return LINDHARD_EINVAL;
    // zone width W grid steps: the whole k-grid, or 1/k_zones of it
    const int kz = std::max(1, pl.p.k_zones);
    if (pl.g.nkx % (2 * kz)) return LINDHARD_EINVAL;
    const int W = pl.g.nkx / kz;
    const int zones = (direction == 0 ? pl.zx : std::min(pl.zx, pl.zy)) * kz;
    const int nseg = (zones + 1) / 2;
    if (nseg > LINDHARD_ENVELOPE_MAX) return LINDHARD_EINVAL;
    const double qstep = 2.0 * M_PI / W * (direction ? std::sqrt(2.0) : 1.0) * q_scale;
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) return LINDHARD_EDEVICE;
    if (dev != pl.device && hipSetDevice(pl.device) != hipSuccess) return LINDHARD_EDEVICE;
    const hipStream_t st = (hipStream_t)stream;
    const void *plane = (const char *)im + (size_t)omega_index * pl.out_nx * pl.out_ny * pl.elem_bytes;
    std::vector<double> res(3 + 4 * (size_t)nseg);
    static_assert(3 + 4 * LINDHARD_ENVELOPE_MAX <= 2 * kOccBlocks + 2, "envelope results fit the scratch");
    hipError_t e = launch_envelope(pl, plane, direction, W, nseg, qstep, pl.scratch, st);
    if (e == hipSuccess)
        e = hipMemcpyAsync(res.data(), pl.scratch, res.size() * sizeof(double), hipMemcpyDeviceToHost, st);
    if (e == hipSuccess) e = hipStreamSynchronize(st);
    if (dev != pl.device) (void)hipSetDevice(dev);
    if (e != hipSuccess) return LINDHARD_EDEVICE;
    *out = lindhard_envelope{};
    out->k0 = res[0];
    out->c_max = res[1];
    out->nseg = nseg;
    for (int k = 0; k < nseg; ++k) {
        out->X[k] = (int32_t)res[3 + 4 * k];
        out->Y[k] = (int32_t)res[4 + 4 * k];
        out->q[k] = res[5 + 4 * k];
        out->y[k] = res[6 + 4 * k];
    }
    return LINDHARD_OK;
}

// Batched execution: the instances are spread over a small pool of worker
// streams (fork from `stream`, join back into it), so independent instances
// of mixed sizes overlap on the device.
namespace {
constexpr int kBatchStreams = 8;
struct BatchPool {
    int device = -1;
    hipStream_t st[kBatchStreams] = {};
    hipEvent_t fork = nullptr;
    hipEvent_t join[kBatchStreams] = {};
};
std::mutex g_pool_mu;
std::vector<BatchPool *> g_pools;

BatchPool *batch_pool(int device)
{
    std::lock_guard<std::mutex> lk(g_pool_mu);
    for (BatchPool *bp : g_pools)
        if (bp->device == device) return bp;
    BatchPool *bp = new (std::nothrow) BatchPool();
    if (!bp) return nullptr;
    bp->device = device;
    bool ok = hipEventCreateWithFlags(&bp->fork, hipEventDisableTiming) == hipSuccess;
    for (int i = 0; i < kBatchStreams && ok; ++i) {
        ok = hipStreamCreateWithFlags(&bp->st[i], hipStreamNonBlocking) == hipSuccess &&
             hipEventCreateWithFlags(&bp->join[i], hipEventDisableTiming) == hipSuccess;
    }
    if (!ok) return nullptr;
    g_pools.push_back(bp);
    return bp;
}
std::mutex g_batch_mu;  // one batch at a time per process (the pool is shared)

// Captured batches: the fork / launches / join sequence of a batch is captured
// once into a HIP graph and replayed when the same plans and outputs come
// again (one graph launch instead of five kernels per instance).  A graph is
// dropped when one of its plans is destroyed.  LINDHARD_BATCH_GRAPH=0 keeps
// eager launches.
struct BatchGraph {
    std::vector<const void *> sig;
    hipGraphExec_t exec = nullptr;
};
std::vector<BatchGraph> g_graphs;
// Batched groups of a batch: instances of the even path with equal group
// keys run every pass as one launch over the group (descriptors in device
// memory, kept with the batch's signature until one of its plans goes);
// `single` lists the instances that run on their own.
struct BatchGroups {
    std::vector<const void *> sig;
    std::vector<std::vector<int>> groups;
    std::vector<int> single;
    EvenInst *d_desc = nullptr;
};
std::vector<BatchGroups> g_groups;
hipStream_t g_capture_stream = nullptr;

bool batch_graphs_enabled()
{
    const char *e = std::getenv("LINDHARD_BATCH_GRAPH");
    return !(e && !std::strcmp(e, "0"));
}
}  // namespace

// The groups of a batch (made on its first call, with their descriptors).
static hipError_t batch_groups(const std::vector<const void *> &sig, const lindhard_plan_t *plans, int n,
                               void *const *outs, const BatchGroups **out)
{
    for (const BatchGroups &bg : g_groups)
        if (bg.sig == sig) {
            *out = &bg;
            return hipSuccess;
        }
    BatchGroups bg;
    bg.sig = sig;
    std::map<std::string, std::vector<int>> by_key;
    for (int i = 0; i < n; ++i) {
        const std::string k = even_group_key(plans[i]->pl);
        if (k.empty())
            bg.single.push_back(i);
        else
            by_key[k].push_back(i);
    }
    std::vector<EvenInst> desc;
    for (auto &kv : by_key) {
        if (kv.second.size() < 2) {
            bg.single.push_back(kv.second[0]);
            continue;
        }
        bg.groups.push_back(kv.second);
        for (int i : kv.second) {
            desc.emplace_back();
            even_group_fill(plans[i]->pl, outs[i], desc.back());
        }
    }
    if (!desc.empty()) {
        hipError_t e = hipMalloc((void **)&bg.d_desc, desc.size() * sizeof(EvenInst));
        if (e == hipSuccess) e = hipMemcpy(bg.d_desc, desc.data(), desc.size() * sizeof(EvenInst), hipMemcpyHostToDevice);
        if (e != hipSuccess) {
            if (bg.d_desc) (void)hipFree(bg.d_desc);
            return e;
        }
    }
    g_groups.push_back(std::move(bg));
    *out = &g_groups.back();
    return hipSuccess;
}

// Fork the batch over the worker streams and join it back into `origin`:
// each group of even-path instances runs its passes as one launch each, the
// other instances on their own; largest work first, round-robin over the
// streams.
static hipError_t batch_launch(BatchPool *bp, const lindhard_plan_t *plans, int n, void *const *outs,
                               const BatchGroups &bg, hipStream_t origin)
{
    hipError_t e = hipEventRecord(bp->fork, origin);
    struct Unit {
        int group;  // index into bg.groups, or -1 - instance
        size_t work;
    };
    std::vector<Unit> units;
    for (size_t k = 0; k < bg.groups.size(); ++k) {
        size_t w = 0;
        for (int i : bg.groups[k]) w += plans[i]->pl.out_elems;
        units.push_back({(int)k, w});
    }
    for (int i : bg.single) units.push_back({-1 - i, plans[i]->pl.out_elems});
    std::stable_sort(units.begin(), units.end(), [](const Unit &a, const Unit &b) { return a.work > b.work; });
    const int ns = std::min((int)units.size(), kBatchStreams);
    for (int i = 0; i < ns && e == hipSuccess; ++i) e = hipStreamWaitEvent(bp->st[i], bp->fork, 0);
    size_t off = 0;
    std::vector<size_t> first(bg.groups.size());
    for (size_t k = 0; k < bg.groups.size(); ++k) {
        first[k] = off;
        off += bg.groups[k].size();
    }
    for (size_t u = 0; u < units.size() && e == hipSuccess; ++u) {
        hipStream_t st = bp->st[u % ns];
        if (units[u].group >= 0) {
            const std::vector<int> &gi = bg.groups[units[u].group];
            std::vector<const Plan *> pls;
            for (int i : gi) pls.push_back(&plans[i]->pl);
            e = launch_even_group(pls.data(), (int)pls.size(), bg.d_desc + first[units[u].group], st);
        } else {
            const int i = -1 - units[u].group;
            e = launch_exec(plans[i]->pl, outs[i], st);
        }
    }
    for (int i = 0; i < ns && e == hipSuccess; ++i) {
        e = hipEventRecord(bp->join[i], bp->st[i]);
        if (e == hipSuccess) e = hipStreamWaitEvent(origin, bp->join[i], 0);
    }
    return e;
}

lindhard_status lindhard_exec_batch(const lindhard_plan_t *plans, int32_t n, void *const *outs, void *stream)
{
    if (!plans || !outs || n < 0) return LINDHARD_EINVAL;
    for (int i = 0; i < n; ++i)
        if (!plans[i] || !outs[i] || plans[i]->pl.device != plans[0]->pl.device) return LINDHARD_EINVAL;
    {
        // a plan's workspace serves one instance at a time: no plan twice
        std::vector<lindhard_plan_t> seen(plans, plans + n);
        std::sort(seen.begin(), seen.end());
        if (std::adjacent_find(seen.begin(), seen.end()) != seen.end()) return LINDHARD_EINVAL;
    }
    if (n == 0) return LINDHARD_OK;
    if (n == 1) return lindhard_exec(plans[0], outs[0], stream);
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) return LINDHARD_EDEVICE;
    const int pdev = plans[0]->pl.device;
    if (dev != pdev && hipSetDevice(pdev) != hipSuccess) return LINDHARD_EDEVICE;
    std::lock_guard<std::mutex> lk(g_batch_mu);
    BatchPool *bp = batch_pool(pdev);
    hipStream_t caller = (hipStream_t)stream;
    hipError_t e = bp ? hipSuccess : hipErrorOutOfMemory;
    std::vector<const void *> sig;
    sig.reserve(2 * n + 1);
    sig.push_back((const void *)(intptr_t)pdev);
    for (int i = 0; i < n; ++i) {
        sig.push_back(plans[i]);
        sig.push_back(outs[i]);
    }
    const BatchGroups *bg = nullptr;
    if (e == hipSuccess) e = batch_groups(sig, plans, n, outs, &bg);
    hipGraphExec_t gexec = nullptr;
    if (e == hipSuccess && batch_graphs_enabled()) {
        for (const BatchGraph &bg : g_graphs)
            if (bg.sig == sig) gexec = bg.exec;
        if (!gexec) {
            if (!g_capture_stream) e = hipStreamCreateWithFlags(&g_capture_stream, hipStreamNonBlocking);
            hipGraph_t graph = nullptr;
            if (e == hipSuccess) e = hipStreamBeginCapture(g_capture_stream, hipStreamCaptureModeThreadLocal);
            if (e == hipSuccess) {
                const hipError_t el = batch_launch(bp, plans, n, outs, *bg, g_capture_stream);
                e = hipStreamEndCapture(g_capture_stream, &graph);
                if (e == hipSuccess) e = el;
            }
            if (e == hipSuccess) e = hipGraphInstantiate(&gexec, graph, nullptr, nullptr, 0);
            if (graph) (void)hipGraphDestroy(graph);
            if (e == hipSuccess) g_graphs.push_back({sig, gexec});
        }
        if (e == hipSuccess) e = hipGraphLaunch(gexec, caller);
    } else if (e == hipSuccess) {
        e = batch_launch(bp, plans, n, outs, *bg, caller);
    }
    for (int i = 0; i < n && e == hipSuccess; ++i) {
        e = hipEventRecord(plans[i]->done, caller);
        plans[i]->pl.executed = true;
    }
    if (dev != pdev) (void)hipSetDevice(dev);
    if (e != hipSuccess) (void)hipGetLastError();
    return e == hipSuccess ? LINDHARD_OK : LINDHARD_EDEVICE;
}

lindhard_status lindhard_plan_destroy(lindhard_plan_t plan)
{
    if (!plan) return LINDHARD_EINVAL;
    {
        std::lock_guard<std::mutex> lk(g_batch_mu);
        for (size_t i = 0; i < g_graphs.size();) {
            if (std::find(g_graphs[i].sig.begin(), g_graphs[i].sig.end(), (const void *)plan) != g_graphs[i].sig.end()) {
                (void)hipGraphExecDestroy(g_graphs[i].exec);
                g_graphs.erase(g_graphs.begin() + i);
            } else {
                ++i;
            }
        }
        for (size_t i = 0; i < g_groups.size();) {
            if (std::find(g_groups[i].sig.begin(), g_groups[i].sig.end(), (const void *)plan) != g_groups[i].sig.end()) {
                if (g_groups[i].d_desc) {
                    (void)hipDeviceSynchronize();  // no launch of the batch may still read them
                    (void)hipFree(g_groups[i].d_desc);
                }
                g_groups.erase(g_groups.begin() + i);
            } else {
                ++i;
            }
        }
    }
    int dev = 0;
    (void)hipGetDevice(&dev);
    (void)hipSetDevice(plan->pl.device);
    if (plan->done) {
        (void)hipEventSynchronize(plan->done);
        (void)hipEventDestroy(plan->done);
    }
    if (plan->setup) (void)hipStreamSynchronize(plan->setup);
    plan_free(plan->pl);
    (void)hipSetDevice(dev);
    delete plan;
    return LINDHARD_OK;
}

const char *lindhard_strerror(lindhard_status st)
{
    switch (st) {
    case LINDHARD_OK: return "ok";
    case LINDHARD_EINVAL: return "invalid argument";
    case LINDHARD_EOFFGRID: return "omega is not on the energy-lag grid";
    case LINDHARD_ENOMEM: return "out of memory";
    case LINDHARD_ETOOBIG: return "job footprint exceeds the HBM budget";
    case LINDHARD_EBUSY: return "busy (queue full or timeout)";
    case LINDHARD_EDEVICE: return "HIP device error";
    case LINDHARD_ENOCONV: return "chemical potential did not converge";
    case LINDHARD_ECANCELED: return "job cancelled";
    case LINDHARD_ESTATE: return "call out of order";
    }
    return "unknown status";
}

}  // extern "C"
