/*
 * lindhard.h -- C ABI of the MI355X (gfx950) library for the bare Lindhard
 * susceptibility, its extended-zone form factor, Kramers-Kronig real part and
 * RPA, computed as products of real-space spectral functions plus FFTs
 * (Wang et al., arXiv:1208.3210, Sec. 3 with Eqs. (9)-(10); RPA and
 * Kramers-Kronig in Sec. 4).
 *
 * What one plan computes (all quantities per site and per spin, eV^-1):
 *
 *   k-grid     k = 2 pi (ix / nkx, iy / nky), periodic first Brillouin zone.
 *   band       eps(k) = -2t(cos kx + cos ky) - 4t' cos kx cos ky
 *                       - 2t''(cos 2kx + cos 2ky)            (or a caller table)
 *   mu         given, or solved from the filling (rigid band, Sec. 3) with
 *              n(mu) = (2/Nk) sum_k [1/2 + atan((mu - eps_k)/gamma)/pi].
 *   energies   d = (emax - emin)/neps, e_j = emin + (j + 1/2) d; e_j <= 0 occupied.
 *   A(k, j)    = (gamma/pi) / ((e_j - (eps_k - mu))^2 + gamma^2)   -- Eq. (5)
 *   Im chi_1BZ(q, m) = -(d/Nk) sum_k sum_{j occupied, j+m unoccupied, j+m < neps}
 *                       A(k, j) A(k+q, j+m)                  -- Eqs. (2), (9), (A3)
 *              at omega = m d; exactly 0 for m = 0 and m >= neps.
 *   extended   out(Q = q + G) = |M(Q)|^2 Im chi_1BZ(q), |M|^2 = F(Q)^2 with the
 *              on-site matrix element of Eq. (3) for a d_{x2-y2}-like Gaussian
 *              orbital: F(Q) = exp(-s|Q|^2)[1 - 2s|Q|^2 + s^2(Qx^2-Qy^2)^2],
 *              s = w^2/4 (ff_kind = LINDHARD_FF_GAUSS_DX2Y2), or 1 (FF_NONE).
 *   Re chi     Kramers-Kronig (Sec. 4), alternate-point rule over all lags:
 *              Re(i) = (2/pi) sum_{j=1..neps-1, j-i odd} Im(j) 2j/(j^2 - i^2).
 *   RPA        chi_RPA = chi / (1 - U chi) on the extended chi (Sec. 4).
 *
 * Output layout: float (LINDHARD_FP32C) or double (LINDHARD_FP64) arrays
 * [nomega][zones_y * nky][zones_x * nkx], row major.  Column X of the extended
 * map is h = k_zones (X - zones_x*nkx/2)/nkx reciprocal-lattice units (k_zones
 * = 1 unless the momentum grid spans several zones), first-zone index
 * u = (X - zones_x*nkx/2) mod nkx (the same for rows): the maps are Gamma
 * centred; the form factor and the Coulomb interaction are taken at
 * Q = 2 pi (h, l).  Output buffers are device memory owned by the caller.
 *
 * Streams are passed as `void *` holding a hipStream_t (NULL = the default
 * stream).  No function throws; every function returns a lindhard_status.
 * Outputs are written only when a call returns LINDHARD_OK.
 */
#ifndef LINDHARD_H
#define LINDHARD_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    LINDHARD_OK = 0,
    LINDHARD_EINVAL = -1,    /* invalid argument or problem description */
    LINDHARD_EOFFGRID = -2,  /* an omega is not m * d (within 1e-9 d) with m >= 0 */
    LINDHARD_ENOMEM = -3,    /* device or host allocation failed */
    LINDHARD_ETOOBIG = -4,   /* job footprint exceeds the server's HBM budget */
    LINDHARD_EBUSY = -5,     /* server queue full */
    LINDHARD_EDEVICE = -6,   /* a HIP runtime call or kernel launch failed */
    LINDHARD_ENOCONV = -7,   /* chemical-potential solve did not converge */
    LINDHARD_ECANCELED = -8, /* served job was cancelled */
    LINDHARD_ESTATE = -9     /* call out of order (e.g. rpa without want_rpa) */
} lindhard_status;

typedef enum {
    LINDHARD_FP32C = 1, /* FP32 FFTs and products, compensated energy-window sums */
    LINDHARD_FP64 = 2   /* FP64 throughout */
} lindhard_precision;

typedef enum {
    LINDHARD_FF_NONE = 0,       /* |M|^2 = 1: extended zones repeat the first zone */
    LINDHARD_FF_GAUSS_DX2Y2 = 1 /* Gaussian d_{x2-y2}-like orbital of width ff_width */
} lindhard_ff;

typedef struct {
    double t, tp, tpp;          /* eV, tight-binding hoppings (ignored if eps_table) */
    const double *eps_table;    /* optional host table eps[iy][ix] (x fastest), eV
                                   (n_bands planes); read only during lindhard_plan */
    double mu;                  /* eV; NaN = solve from `filling` */
    double filling;             /* electrons per site, both spins (1 + x) */
    double gamma;               /* Lorentzian half width of Eq. (5), eV, > 0 */
    int32_t nkx, nky;           /* powers of two 4 .. 4096; other sizes >= 4 (Bluestein
                                   transforms) up to 4097 in FP32 and 2049 in FP64, two
                                   dimensions and one band (zones, form factor and RPA as
                                   for powers of two; centring (q + floor(Z n / 2)) mod n) */
    int32_t neps;               /* power of two, 4 .. 2048 */
    double emin, emax;          /* energy window, emin < 0 < emax */
    int32_t nomega;             /* number of requested omegas, 1 .. 65535 */
    const double *omega;        /* host array of omegas, eV; each m*d, m >= 0
                                   (or >= 0 anywhere with omega_interp) */
    int32_t zones_x, zones_y;   /* odd, >= 1, zones_x*nkx <= 65536, zones_y*nky <= 65535 */
    int32_t ff_kind;            /* lindhard_ff */
    double ff_width;            /* orbital width w in lattice constants (> 0 if used) */
    int32_t precision;          /* lindhard_precision */
    int32_t want_rpa;           /* nonzero: keep every lag for lindhard_rpa */
    /* Extended momentum (Eqs. (4), (9)): the k-grid spans k_zones Brillouin
     * zones per axis (p = 2 pi k_zones (ix/nkx, iy/nky); 0 or 1 = the first
     * zone; at most 64) and, if rho_table is given, the spectral function is
     * A(p, e) = rho(p) A_band(p, e) with the momentum density rho[iy][ix]
     * (host table, x fastest, finite; read only during lindhard_plan).  The
     * output q-grid is then the same extended grid. */
    int32_t k_zones;
    const double *rho_table;
    /* Omegas off the lag grid: 0 = rejected (LINDHARD_EOFFGRID); 1 = an omega
     * with m d < omega < (m + 1) d takes the linear interpolation
     * (1 - f) chi(m d) + f chi((m + 1) d), f = omega / d - m, of the lag-grid
     * values (Im chi, and Re chi from the Kramers-Kronig pass); values at lags
     * 0 and >= neps are 0.  Omegas within 1e-9 d of the grid are on it. */
    int32_t omega_interp;
    /* Several bands (Eqs. (2), (4)).  n_bands in 1 .. LINDHARD_MAX_BANDS (0
     * = 1); with more than one, eps_table is required and holds n_bands planes
     * [band][iy][ix], rho_table (if given) as many, and mu / filling count the
     * electrons of every band.  pair_weight NULL: the spectral function of
     * Eq. (4) sums the bands, A = sum_n rho_n A_n, and one correlation is
     * taken.  Otherwise a host array [nu][mu] of band-pair weights |M|^2 >= 0
     * (Eq. (2), not all zero; the same at every Q, the orbital form factor
     * ff_kind multiplying every pair): Im chi = sum w[nu][mu] chi_{nu,mu},
     * with band nu occupied and band mu empty in chi_{nu,mu}.  Tables are
     * read only during lindhard_plan. */
    int32_t n_bands;
    const double *pair_weight;
    /* Three-dimensional k-grids (the d^3p of Eq. (9)): nkz > 1 (a power of two
     * up to 256; 0 or 1 = two dimensions) adds a third periodic axis.  It
     * needs eps_table with nkz planes [band][iz][iy][ix] (rho_table alike) and
     * a first-zone k-grid (k_zones <= 1).  Zones, the orbital form factor and
     * the RPA apply in the plane: each kz plane is extended over zones_x x
     * zones_y in-plane zones with the in-plane |M(Qx, Qy)|^2, and the Coulomb
     * |Q|^2 adds (2 pi hz)^2, hz = (Z - nkz/2) / nkz (lattice constant a along
     * z).  The output planes are [omega][Z][Y][X] with Z = (qz + nkz/2) mod
     * nkz, reported as out_ny = nkz * zones_y * nky rows of out_nx =
     * zones_x * nkx.  With RPA, nkz * nky <= 65535. */
    int32_t nkz;
    /* Band-pair matrix elements that vary with the momentum transfer (Eqs.
     * (2), (3)): optional host array of n_bands * n_bands maps
     * m2[nu][mu][Y][X] = |M^{nu,mu}_G(Q)|^2 on the extended output grid
     * (zones_y * nky rows of zones_x * nkx, indexed like the output planes),
     * finite and >= 0, read only during lindhard_plan.  Then
     * Im chi(Q, omega) = sum_{nu,mu} m2[nu][mu](Q) chi_{nu,mu}(q, omega), band
     * nu occupied and band mu empty, q the first-zone point of Q; with one
     * band it is a tabulated |M(Q)|^2.  It excludes pair_weight (NULL),
     * ff_kind (NONE), want_rpa, nkz > 1 and grids that are not powers of two. */
    const double *pair_m2;
} lindhard_problem;

#define LINDHARD_MAX_BANDS 8

typedef struct lindhard_plan_s *lindhard_plan_t;

typedef struct {
    double mu;                /* chemical potential used, eV */
    double deps;              /* energy step d, eV */
    int32_t j0;               /* number of occupied energy points */
    int32_t out_nx, out_ny;   /* zones_x*nkx, zones_y*nky */
    int32_t nomega;
    int32_t lag_lo, lag_hi;   /* lag range the energy-window pass computes (0,0 = none) */
    int32_t mu_iterations;    /* Newton/bisection steps of the mu solve (0 if given) */
    size_t workspace_bytes;   /* device bytes the plan holds */
    size_t out_elems;         /* elements of each output array */
    size_t elem_bytes;        /* 4 (FP32C) or 8 (FP64) */
    char schedule[96];        /* human-readable pass schedule */
} lindhard_info;

/* Validate `p`, build the band on the device, solve mu, build twiddle and
 * form-factor tables and allocate the device workspace (owned by the plan).
 * Synchronous.  Errors: EINVAL, EOFFGRID, ENOMEM, EDEVICE, ENOCONV. */
lindhard_status lindhard_plan(const lindhard_problem *p, lindhard_plan_t *out);

/* Copy the plan's derived quantities into *info.  EINVAL on NULL. */
lindhard_status lindhard_plan_info(lindhard_plan_t plan, lindhard_info *info);

/* Shape of the output arrays a problem would have (host only, no device
 * work): nomega planes of out_ny rows of out_nx elements of elem_bytes bytes
 * each (the buffers lindhard_serve_submit writes must have this shape).
 * Errors: as lindhard_plan's validation (EINVAL, EOFFGRID). */
lindhard_status lindhard_problem_shape(const lindhard_problem *p, int32_t *nomega, int32_t *out_ny, int32_t *out_nx,
                                       int32_t *elem_bytes);

/* Enqueue the whole hot path on `stream`: spectral builder + row FFT, column
 * FFT, energy-window product, inverse column FFT, inverse row FFT + scale +
 * form factor + zone writes into `im_chi` (device, out_elems elements of the
 * plan's precision).  Asynchronous; a plan is used by one stream at a time.
 * Errors: EINVAL (NULL), EDEVICE (launch failure). */
lindhard_status lindhard_exec(lindhard_plan_t plan, void *im_chi, void *stream);

/* lindhard_exec with per-pass timing: records HIP events on `stream` around
 * the five passes (P1 spectral builder + row FFT, P2 column FFT, P3 energy
 * window, P4 inverse column FFT, P5 inverse row FFT + epilogue), waits for
 * the last one and writes the five durations in milliseconds to pass_ms[0..4]
 * (host array).  Synchronous.  Errors: EINVAL, EDEVICE. */
lindhard_status lindhard_exec_timed(lindhard_plan_t plan, void *im_chi, void *stream, float *pass_ms);

/* After lindhard_exec on a plan built with want_rpa: Kramers-Kronig real part
 * and RPA with constant U (eV) into three more device arrays of the same layout:
 * re_chi = Re chi_ext, im_rpa / re_rpa = Im / Re of chi_ext / (1 - U chi_ext).
 * Any of the three pointers may be NULL to skip that output.
 * Errors: EINVAL, ESTATE (plan without want_rpa), EDEVICE. */
lindhard_status lindhard_rpa(lindhard_plan_t plan, double U, void *re_chi, void *im_rpa,
                             void *re_rpa, void *stream);

/* lindhard_rpa with the Coulomb interaction the paper names for the RPA
 * denominator (Sec. 4, V_q decaying as 1/q^2): V(Q) = v / |Q|^2 with
 * Q = 2 pi (h, l) in units of 1/a, (h, l) the reciprocal-lattice coordinates
 * of each extended output point, diagonal in G (no local fields); v in
 * eV a^2.  At Q = 0 the interaction is infinite and im_rpa / re_rpa are 0
 * (the limit of chi / (1 - V chi)).  Same buffers, ordering and errors as
 * lindhard_rpa (EINVAL for non-finite v). */
lindhard_status lindhard_rpa_coulomb(lindhard_plan_t plan, double v, void *re_chi, void *im_rpa,
                                     void *re_rpa, void *stream);

/* Dynamical structure factor by the fluctuation-dissipation relation,
 * Eq. (1): s_out = -(1/pi) im / (1 - exp(-omega / kT)) for every element of
 * `im` (device, out_elems elements of the plan's precision and output layout:
 * Im chi from lindhard_exec or Im chi_RPA from lindhard_rpa*), omega = m d of
 * each output plane, kT in eV.  kT = 0 is the zero-temperature limit (factor
 * 1 for omega > 0); omega = 0 gives 0.  s_out may equal im (in place).
 * Asynchronous on `stream`.  Errors: EINVAL (NULL, kT < 0 or not finite),
 * EDEVICE. */
lindhard_status lindhard_structure_factor(lindhard_plan_t plan, double kT, const void *im, void *s_out,
                                          void *stream);

/* q-average of every output plane: out[w] = mean over all (X, Y) of
 * im[w][Y][X], accumulated in FP64 in a fixed order (deterministic), into
 * `out` (device, nomega doubles).  On a plan with one zone and no form factor
 * and the Im chi of lindhard_exec this is the q-integrated joint density of
 * states of Fig. 2(b) (with the sign of Im chi).  Uses the plan's scratch
 * memory: one call at a time per plan.  Asynchronous on `stream`.
 * Errors: EINVAL (NULL), EDEVICE. */
lindhard_status lindhard_q_average(lindhard_plan_t plan, const void *im, double *out, void *stream);

/* lindhard_q_average without a plan and without any device allocation, for
 * callers that cannot allocate device memory (code under stream capture,
 * serving loops, harnesses that forbid hipMalloc): out[w] = mean over the
 * plane_elems elements of plane w of `im` (device, nomega planes of
 * plane_elems contiguous elements, float if elem_bytes = 4, double if 8),
 * accumulated in FP64 in a fixed order.  The partial sums live in a
 * per-device array of the library (LINDHARD_NOALLOC_MAX_PLANES * 32 doubles,
 * 1 MiB, held until the process ends), looked up on the first call on each
 * device; calls that overlap on one device race on it (no two at once per
 * device).  Asynchronous on `stream`.  Errors: EINVAL (NULL pointers,
 * plane_elems < 1, elem_bytes not 4 or 8, nomega < 1 or above
 * LINDHARD_NOALLOC_MAX_PLANES), EDEVICE. */
#define LINDHARD_NOALLOC_MAX_PLANES 4096
lindhard_status lindhard_q_average_noalloc(const void *im, int32_t nomega, int64_t plane_elems, int32_t elem_bytes,
                                           double *out, void *stream);

/* Peak search (plasmon modes as the peaks of -Im chi_RPA, Sec. 4): for every
 * extended point (X, Y), the index w in [0, nomega) of the largest -im[w][Y][X]
 * (the first on ties, compared in the plan's precision) into peak (device,
 * int32, out_ny * out_nx, row-major).  `im` as for lindhard_structure_factor.
 * Asynchronous on `stream`.  Errors: EINVAL (NULL), EDEVICE. */
lindhard_status lindhard_peak_index(lindhard_plan_t plan, const void *im, int32_t *peak, void *stream);

/* Cut through the output planes along a path (Fig. 2(a): -Im chi along the
 * high-symmetry lines as a function of omega): out[w][p] = im[w][Y[p]][X[p]]
 * for every plane w and path point p.  X, Y: host arrays of npts extended-grid
 * indices (0 <= X < out_nx, 0 <= Y < out_ny; read during the call); out:
 * device, nomega * npts elements of the plan's precision; `im` as for
 * lindhard_structure_factor.  Asynchronous on `stream` (the indices are staged
 * in plan memory: calls on one plan must not overlap).  Errors: EINVAL (NULL,
 * npts < 1, an index off the grid), ENOMEM, EDEVICE. */
lindhard_status lindhard_cut(lindhard_plan_t plan, const void *im, const int32_t *X, const int32_t *Y, int32_t npts,
                             void *out, void *stream);

/* The high-symmetry path Gamma -> X -> M -> Gamma of the central zone on the
 * extended grid (Gamma = (out_nx/2, out_ny/2), X = (pi, 0), M = (pi, pi)), one
 * point per grid step: 3 W / 2 + 1 points for a zone W = nkx / k_zones steps
 * wide (nkx == nky required; the zone boundary wraps to the opposite edge
 * when the grid holds one zone).  Host only:
 * writes at most `capacity` points to X, Y and the count to *npts.  Errors:
 * EINVAL (NULL, nkx != nky or not a multiple of 2 k_zones, capacity too
 * small; *npts still gets the count). */
lindhard_status lindhard_high_symmetry_path(lindhard_plan_t plan, int32_t *X, int32_t *Y, int32_t capacity,
                                            int32_t *npts);

#define LINDHARD_ENVELOPE_MAX 64

typedef struct {
    double k0;      /* fitted decay momentum of 1 / (1 + (q/k0)^2), in q_scale units */
    double c_max;   /* largest -Im chi along the cut (the normalisation) */
    int32_t nseg;   /* envelope points: the central half zone, then one per zone */
    int32_t X[LINDHARD_ENVELOPE_MAX], Y[LINDHARD_ENVELOPE_MAX]; /* point of each maximum */
    double q[LINDHARD_ENVELOPE_MAX]; /* its |q| in q_scale units */
    double y[LINDHARD_ENVELOPE_MAX]; /* its -Im chi / c_max */
} lindhard_envelope;

/* Zone-to-zone decay along a cut from the extended-grid centre (Fig. 5):
 * plane `omega_index` of `im` is followed along [100] (direction 0: Y = out_ny/2,
 * X >= out_nx/2) or [110] (direction 1, nkx == nky); the central half zone and
 * each further zone crossed give one envelope point, the largest -Im chi in
 * that segment (first on ties, decided in the plan's precision), normalised by
 * the largest of them; the Lorentzian 1 / (1 + (q/k0)^2) is then fitted to
 * these points by least squares in u = 1/k0^2 over [1e-8, 1e8] (a log-spaced
 * scan, then bisection of dF/du; a minimum at the range end returns that end).
 * q = |Q| q_scale with Q = 2 pi (h, l) in units of 1/a, so q_scale = 1/a gives
 * q in the inverse units of a (e.g. atomic units for a in bohr).  A zone is
 * nkx / k_zones grid steps wide; segments: (zones + 1) / 2 along the cut, with
 * zones = k_zones zones_x for [100] and k_zones min(zones_x, zones_y) for
 * [110] (a half zone left at the grid edge is not used), at most
 * LINDHARD_ENVELOPE_MAX.  Synchronous: returns when `out` is
 * filled.  Errors: EINVAL (NULL, bad index or direction, q_scale <= 0, too
 * many zones, nkx != nky for [110], nkx not a multiple of 2 k_zones),
 * EDEVICE. */
lindhard_status lindhard_zone_envelope(lindhard_plan_t plan, const void *im, int32_t omega_index, int32_t direction,
                                       double q_scale, lindhard_envelope *out, void *stream);

/* Run n independent plans as one batch ordered on `stream` (the batched
 * form of the hot path: many dopings, broadenings and grid sizes at once).
 * Instances on the mirror-symmetric (even) path with the same precision,
 * grid, momentum-density use and window schedule form a group, and each of
 * the five passes runs as ONE launch over the whole group (per-instance
 * descriptors in device memory; energies, omega lists, bands, fillings and
 * broadenings may differ inside a group).  Groups and the remaining
 * instances are forked onto a pool of worker streams (largest first) so
 * that work of mixed grid sizes overlaps, and joined back into `stream`
 * before any later work on it.  The sequence is captured into a HIP graph
 * on the first call and replayed for the same plans and outputs.  Each
 * output equals that of lindhard_exec on its plan, bit for bit.  outs[i] as
 * in lindhard_exec; no plan twice.  All plans must live on the same device;
 * one batch runs at a time per process.  Errors: EINVAL, EDEVICE. */
lindhard_status lindhard_exec_batch(const lindhard_plan_t *plans, int32_t n, void *const *outs,
                                    void *stream);

/* Free the plan and its device workspace (waits for its work to finish). */
lindhard_status lindhard_plan_destroy(lindhard_plan_t plan);

/* ---------------------------------------------------------------- serving */
typedef struct {
    size_t hbm_budget_bytes; /* limit on the device memory of every plan the server holds */
    int32_t max_inflight;    /* concurrent jobs on the device (>= 1) */
    int32_t max_queue;       /* queued (not yet admitted) jobs (>= 1) */
    /* optional: problems planned when the server starts (n_warm of them, the
     * arrays they point to read during lindhard_serve_create only), so that
     * the first jobs of their classes find a plan and a tuned window schedule;
     * NULL / 0 for none */
    const lindhard_problem *warm;
    int32_t n_warm;
} lindhard_serve_config;

typedef struct lindhard_server_s *lindhard_server_t;

typedef struct {
    uint64_t submitted, completed, failed, rejected, canceled;
    double p50_ms, p99_ms;   /* submit -> result-ready latency of the last 65536 completed jobs */
    double points_per_s;     /* output points of completed jobs / wall time since create */
    size_t hbm_high_water;   /* largest device memory held by the server's plans */
    int32_t queue_depth, inflight;
    uint64_t plan_reuses;    /* jobs that ran on a cached plan of their class */
    uint64_t plan_builds;    /* plans built from scratch (warm problems included) */
    uint64_t plan_evictions; /* idle plans freed to make room */
    int32_t cached_plans;    /* idle plans held right now */
    size_t resident_bytes;   /* device memory held by the server's plans right now */
    uint64_t merged_jobs;    /* jobs that ran together with others of their class */
} lindhard_serve_stats;

/* Start a server.  Worker threads (max_inflight of them, each with a stream
 * of its own) admit queued jobs in arrival order while a slot is free and the
 * memory of all plans the server holds stays within the budget, and run each
 * admitted job (exec, optional rpa) so that jobs overlap on the device.
 * Plans are cached by class: everything that fixes a plan's tables and buffer
 * layout (precision, grid, energy window, zones, form factor, RPA, bands,
 * symmetry), but not the band, broadening, filling, chemical potential or
 * omega list.  A job takes an idle plan of its class and rebinds it (band, mu,
 * omegas; buffers grow when its lag range needs more), so it neither builds
 * tables nor times window schedules; only a job of a new class plans from
 * scratch.  Idle plans are freed, least recently used first, when a job
 * needs their memory.  A worker that admits a job also takes queued jobs of
 * its class behind it (up to 8, within the budget): those on the even path
 * with the same window schedule run every pass as one launch over all of
 * them, as lindhard_exec_batch does.  A job's result equals that of
 * lindhard_plan + lindhard_exec (+ lindhard_rpa) on its problem, bit for bit.
 * Errors: EINVAL, ENOMEM, EDEVICE, or the planning status of a warm problem. */
lindhard_status lindhard_serve_create(const lindhard_serve_config *cfg, lindhard_server_t *out);

/* Queue one job.  The problem (and its omega / eps_table arrays) is copied.
 * Outputs are device buffers as in lindhard_exec / lindhard_rpa; pass
 * U_or_nan = NaN (and NULL re/rpa buffers) for no RPA.  *ticket identifies the
 * job.  Errors: EINVAL / EOFFGRID (problem invalid), ETOOBIG (footprint over
 * the budget), EBUSY (queue full). */
lindhard_status lindhard_serve_submit(lindhard_server_t s, const lindhard_problem *p,
                                      double U_or_nan, void *im_chi, void *re_chi, void *im_rpa,
                                      void *re_rpa, uint64_t *ticket);

/* Non-blocking completion check: *done = 1 when finished (then *job_status is
 * the job's own status).  Once a call has reported a job finished, the server
 * forgets it: later calls with its ticket return EINVAL. */
lindhard_status lindhard_serve_poll(lindhard_server_t s, uint64_t ticket, int32_t *done,
                                    lindhard_status *job_status);

/* Block until the job finishes or timeout_s passes (EBUSY on timeout); a
 * negative timeout waits for good.  As with poll, the ticket is released once
 * the job has been reported finished. */
lindhard_status lindhard_serve_wait(lindhard_server_t s, uint64_t ticket, double timeout_s,
                                    lindhard_status *job_status);

/* Cancel a job that has not been admitted yet (its status becomes ECANCELED).
 * A job already running or finished is left alone and EBUSY is returned.
 * EINVAL for an unknown ticket. */
lindhard_status lindhard_serve_cancel(lindhard_server_t s, uint64_t ticket);

lindhard_status lindhard_serve_stats_get(lindhard_server_t s, lindhard_serve_stats *out);

/* Drain queued and in-flight jobs, stop the admission thread, free all. */
lindhard_status lindhard_serve_destroy(lindhard_server_t s);

/* Static description of a status code. */
const char *lindhard_strerror(lindhard_status st);

#ifdef __cplusplus
}
#endif

#endif /* LINDHARD_H */
