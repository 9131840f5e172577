// lh_internal.h -- plan object and pass launchers shared by the C ABI, the
// batched executor and the server.  Not part of the public interface.
#pragma once
#include <hip/hip_runtime.h>

#include <string>
#include <vector>

#include "../../include/lindhard.h"

namespace lh {

// Geometry of one instance and of its device arrays.
//
// Spectral / real-space arrays ("slices") use a column-tiled layout so that
// every pass streams contiguous memory: element (slice s, rx, ry) of the
// half spectrum rx in [0, L], L = nkx/2, lives at
//   ((s * NT + rx / C) * nky + ry) * C + rx % C,    NT = L / C + 1,
// with C complex values = 32 bytes per tile row (C = 4 in FP32, 2 in FP64).
// A column pass reads one tile (nky * C values) as one contiguous block, a row
// pass reads R rows * C values per tile, the energy-window pass reads RY rows
// * C values per slice.
// Source of one output plane: wa S[a] + wb S[b] over window slots a, b
// (a < 0: the plane is zero; b < 0: no second term).  On-grid omegas have
// a single slot with wa = 1; an omega between lags m and m + 1 blends the two.
struct PlaneSrc {
    int a, b;
    double wa, wb;
};

struct Geo {
    int fp64;
    int nkx, nky, logNx, logNy;
    int L, logL;        // row transform length nkx / 2
    int C, logC, NT;    // tile width (complex values) and tile count
    int nkz, logNz;     // third axis (1, 0 in two dimensions)
    size_t plane_elems; // NT * nky * C: one kz plane of a slice (general path)
    int neps;
    int jA, jB;         // slices that can enter the window: [jA, jB)
    int nS;             // jB - jA
    int j0;             // occupied points (global index)
    int m_lo, m_hi, nL; // lag range of the window pass; nL = 0: nothing to do
    int nslots;         // slices allocated in the spectral array
    size_t slice_elems; // NT * nky * C * nkz
    // launch shapes
    int p1_R, p1_logR, p1_jc;
    int p3_RY, p3_logRY, p3_TR, p3_logTR;
    int p5_R, p5_logR;
    // mirror-symmetric band (eps(kx,ky) = eps(-kx,ky) = eps(kx,-ky)): every
    // real-space function is real and even, so the slices hold real values on
    // the quarter rx in [0, nkx/2], ry in [0, nky/2]:
    //   element (s, rx, ry) at ((s * NTe + rx / Ce) * HyS + ry) * Ce + rx % Ce,
    // Ce = 32 bytes of reals, NTe = ceil((nkx/2 + 1) / Ce), Hy = nky/2 + 1.
    int even;
    int Ce, logCe, NTe, Hy;
    int HyS;                  // row stride of a tile: Hy rounded up to 4 rows (128 bytes)
    size_t slice_e;
    int e1_R, e1_jc;          // row pairs per block, slices per block
    int e3_TR, e3_logTR;      // real-space points per block, even window
    int e3_PL;                // padded length of each reversed / shifted window array
    int e5_R;                 // row pairs per block, even inverse row pass
    // even window on the matrix cores (e3_variant 1): TRm points per block,
    // per point PA reversed occupied values then nHe + 64 unoccupied ones
    // (32 zeros each side), point stride PS; NAG / NMG groups of 256
    // occupied energies / lags
    int e3_variant;
    int e3m_TR, e3m_PA, e3m_nA, e3m_nHe, e3m_PS, e3m_NAG, e3m_NMG;
    int e3m_buf;              // occupied and unoccupied slice ranges each below 4 GiB: buffer loads
    // even window as 4 x 4 rank-1 matrix updates (e3_variant 2, FP32): lag
    // tiles of 16, nT of them; chunk c of tile t reads the B set u = t - c + U0;
    // P' at LDS position 16 + a + offP (a0 + offP = 15), u <= umax, c <= cmax;
    // nAst / nHst values staged, rows of PSP / PSH floats (LP / LH used);
    // e3q_W: the autotuner label TR / 16 (the rank-1 window block shape is fixed)
    int e3q_ok, e3q_nT, e3q_U0, e3q_a0, e3q_offP, e3q_umax, e3q_cmax, e3q_LP, e3q_LH, e3q_PSP, e3q_PSH;
    int e3q_nAst, e3q_nHst, e3q_W;
    int e3q_big;              // offsets past 4 GiB: 64-bit addressing
    // energy-window variant: 0 direct (compensated in FP32), 1 FFT along energy
    int p3_variant;
    int logNE;                // FFT length along energy for variant 1
    int p3f_TR, p3f_logTR;    // real-space points per block for variant 1
    int tuned;                // 1: window schedule chosen by timing, 2: from the tuning cache
    // grids of any size (bs = 1): Bluestein transforms of length 2^logMx,
    // 2^logMy; bs_Rr rows per block in the row passes, bs_Rc columns per
    // block in the column passes, bs_SJ energy slices (or lags) per block in
    // the column passes
    int bs, logMx, logMy, bs_Rr, bs_Rc, bs_SJ;
};

// Elements per thread of the register FFTs in the even builder pass (the
// builder also keeps the band rows of its lines in registers).
constexpr int kE1Elems = 8;
// ... except on 4096-point rows, where eight would take 512 threads per line
constexpr int e1_elems(int logn) { return logn >= 12 ? 16 : kE1Elems; }
// Threads per block of the last even row pass: up to 512 (FP32 rows of 1024
// and 2048 points take four lines per block: with the padded engine the
// block's lines and twiddle table fit twice per CU, sixteen waves against the
// twelve that blocks of two lines give)
constexpr int kE5MaxThreads = 512;
// Threads per block of the column passes: up to 512, 1024 for 4096-point
// columns (one tile of C lines of 256 threads each)
constexpr int col_threads(int logn) { return logn >= 12 ? 1024 : 512; }
// ... and in the general builder pass, for the same reason (with sixteen it
// needs ~220 registers and two waves per SIMD; with eight ~120 and four).
constexpr int kP1Elems = 8;
// Partial sums per output plane of the q-average (plan scratch holds them).
constexpr int kQavgBlocks = 32;
// ... and in the even column passes (sixteen measured faster than eight there).
constexpr int kEcolElems = 16;

constexpr int ilog2_c(int v) { return v <= 1 ? 0 : 1 + ilog2_c(v / 2); }

struct Plan {
    lindhard_problem p{};
    std::vector<double> omega;
    std::vector<int> lag;      // lag m of each requested omega (>= 0)
    std::vector<double> frac;  // omega = (lag + frac) d, 0 <= frac < 1 (0 on the grid)
    std::vector<PlaneSrc> src; // window slots of each omega's plane
    int device = 0;
    Geo g{};
    double mu = 0.0, deps = 0.0, scale = 0.0, ff_s = 0.0;
    int mu_iters = 0;
    int zx = 1, zy = 1, out_nx = 0, out_ny = 0;
    size_t out_elems = 0, elem_bytes = 4;
    // device memory (owned)
    double *xi = nullptr;      // eps(k) - mu, FP64, [band][nky][nkx]
    void *twx = nullptr;       // cx<T>[nkx]
    void *twy = nullptr;       // cx<T>[nky]
    void *twz = nullptr;       // cx<T>[nkz] (three dimensions)
    // grids of any size: per axis chirp b, chirp spectra hf / hi, FFT twiddles of length M
    void *bsx[4] = {nullptr, nullptr, nullptr, nullptr};
    void *bsy[4] = {nullptr, nullptr, nullptr, nullptr};
    void *twe = nullptr;       // cx<T>[2^logNE] (energy-axis FFT)
    bool has_rho = false;
    void *rho = nullptr;       // momentum-density weights rho[band][iy][ix] in T (or none)
    int nb = 1;                // bands (xi and rho hold nb planes)
    bool pairs = false;        // band-pair sum with weights pairw[nu * nb + mu] (else one summed band)
    std::vector<double> pairw;
    // band-pair maps |M^{nu,mu}(Q)|^2 on the extended output grid, in T
    // ([nu][mu][out_ny][out_nx]); m2_pairs: the pairs nu * nb + mu whose map is
    // not all zero (at least one entry)
    bool has_m2 = false;
    void *m2 = nullptr;
    std::vector<int> m2_pairs;
    void *bspec = nullptr;     // pair sum: forward-transformed spectra of every band, nb x nS slices
    void *sacc = nullptr;      // pair sum: the summed window outputs, nL slices
    double2 *ffx = nullptr;    // (exp(-s Qx^2), Qx^2) per extended column
    double2 *ffy = nullptr;    // per extended row
    PlaneSrc *d_src = nullptr; // per omega: window slots and weights
    double *d_frac = nullptr;  // per omega: frac
    int *d_lag = nullptr;      // per omega: lag
    void *spec = nullptr;      // spectral / real-space array, nslots slices
    void *im1 = nullptr;       // RPA: Im chi_1BZ [neps][nky][nkx]
    void *re1 = nullptr;       // RPA: Re chi_1BZ [kk_lags.size()][nky][nkx], one plane per needed lag
    double *kkw = nullptr;     // RPA: Kramers-Kronig weights [kk_ntiles][16 kk_nch][16]
    // RPA: the lags whose Re chi is needed (sorted; the slots of re1), in
    // tiles of 16 lags of one parity ((lag, slot) per row, (-1, -1) padding),
    // and per omega the slots of its lag and of the next one (-1: none)
    std::vector<int> kk_lags;
    std::vector<int2> kk_rows;
    std::vector<int> kk_slot;
    int kk_ntiles = 0, kk_nch = 0;  // tiles, chunks of 32 energies
    int2 *d_kkrow = nullptr;
    int *d_kkslot = nullptr;
    double *scratch = nullptr; // mu-solve partial sums
    size_t ws_bytes = 0;
    std::vector<std::pair<void *, size_t>> allocs;  // pooled device buffers
    bool executed = false;
    std::string schedule;
};

// One instance of a batched launch on the even path: its geometry and the
// arguments its passes take (device memory, read by the batched kernels at
// blockIdx.z).
struct EvenInst {
    Geo g;
    const double *xi;
    const void *rho, *twx, *twy;
    void *spec;
    const PlaneSrc *psrc;
    void *out;
    const double2 *ffx, *ffy;
    double emin, deps, gamma, scale, ffs;
    int zx, zy, ff, onx, ony, nomega;
};

// Validate and derive everything host-side (no device work).  Fills `pl`.
lindhard_status plan_describe(const lindhard_problem *p, Plan &pl);
// One device buffer of a plan: where its pointer lives and its size (0: unused).
struct BufSpec {
    void **ptr;
    size_t bytes;
};
std::vector<BufSpec> plan_buffers(const Plan &pl);
// Plan caching (the server): the class key of a described problem, the key,
// allocated buffer sizes and resident bytes of a built plan, and rebinding a
// built plan to another problem of its class (synchronous on st).
std::string plan_class_key(const Plan &pl);
const std::string &plan_key(lindhard_plan_t plan);
std::vector<size_t> plan_capacity(lindhard_plan_t plan);
size_t plan_resident_bytes(lindhard_plan_t plan);
lindhard_status plan_rebind(lindhard_plan_t plan, const lindhard_problem *p, hipStream_t st);
const Plan &plan_of(lindhard_plan_t plan);
// Allocate device memory, build band / mu / tables.  Synchronous on `st`.
lindhard_status plan_build(Plan &pl, hipStream_t st);
void plan_free(Plan &pl);
// Device footprint of a problem (for admission).  0 if invalid.
size_t plan_footprint(const Plan &pl);

// Pass launchers (asynchronous on `st`).
hipError_t launch_exec(const Plan &pl, void *out, hipStream_t st, hipEvent_t *ev = nullptr);
hipError_t launch_rpa(const Plan &pl, int vkind, double U, void *re, void *imr, void *rer, hipStream_t st);
hipError_t launch_sqw(const Plan &pl, double kT, const void *im, void *s, hipStream_t st);
hipError_t launch_peak(const Plan &pl, const void *im, int32_t *idx, hipStream_t st);
hipError_t launch_qavg(const Plan &pl, const void *im, double *out, hipStream_t st);
// q-average of nw planes of `plane` elements with the partial sums in `part`
// (nw * kQavgBlocks doubles; every entry is written, none is read first).
hipError_t launch_qavg_raw(const void *im, bool fp64, size_t plane, int nw, double *part, double *out,
                           hipStream_t st);
hipError_t launch_window(const Plan &pl, hipStream_t st);  // energy-window pass alone
// The even window as 4 x 4 rank-1 matrix updates (FP32), W waves per block.
size_t e3q_lds_bytes(const Geo &g, int W);
hipError_t launch_e3q(const Plan &pl, int W, hipStream_t st);
hipError_t launch_cut(const Plan &pl, const void *im, const int *xy, int npts, void *out, hipStream_t st);
// res: 3 + 4 * nseg doubles of device memory; im_plane: the plane to cut
hipError_t launch_envelope(const Plan &pl, const void *im_plane, int dir, int W, int nseg, double qstep, double *res,
                           hipStream_t st);

// Batched launches of the even path: plans of one group (same precision,
// grid, momentum-density use and window schedule; one band, no pair sums,
// maps or RPA) run each pass as one launch over all instances.  The key is
// empty for a plan that cannot be batched.
std::string even_group_key(const Plan &pl);
void even_group_fill(const Plan &pl, void *out, EvenInst &d);
hipError_t launch_even_group(const Plan *const *pls, int n, const EvenInst *d_desc, hipStream_t st);
hipError_t launch_e3q_group(const Plan *const *pls, int n, const EvenInst *d_desc, hipStream_t st);
hipError_t plan_exec_group(const lindhard_plan_t *plans, int n, void *const *outs, EvenInst *d_desc,
                           std::vector<EvenInst> &host, hipStream_t st);

// Setup kernels.
hipError_t launch_band(const Plan &pl, const double *d_table, hipStream_t st);
hipError_t launch_occ(const Plan &pl, double mu, double *d_out2, hipStream_t st);
hipError_t launch_tables(const Plan &pl, hipStream_t st);
hipError_t launch_xi_shift(const Plan &pl, double mu, hipStream_t st);

constexpr int kOccBlocks = 512;

}  // namespace lh
