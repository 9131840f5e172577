// lh_window.hip -- energy-window pass of the even path on the matrix cores as
// rank-1 updates of 4 x 4 blocks, one block per real-space point (FP32).
//
// The window of a real-space point r is the real linear convolution
//   S(m) = sum_{a + x = m - 1} P'[a] H'[x],   P'[a] = B(r, j0 - 1 - a) (occupied,
//   reversed), H'[x] = B(r, j0 + x) (unoccupied),
// i.e. the energy integral of Eqs. (9) / (A3) over the product of real-space
// functions (Sec. 3).  v_mfma_f32_4x4x1_16b_f32 multiplies sixteen independent
// 4 x 4 outer products per instruction (block b in lanes 4b .. 4b + 3;
// D[lane 4b + j][r] += A[lane 4b + r] B[lane 4b + j]).  Block b serves point b
// of the wave; a 4 x 4 accumulator holds the sixteen lags
// L = m - 1 = K0 + r + 4 j of one lag tile (K0 = m_lo - 1 + 16 t), and the step
// alpha adds H'[alpha + r] P'[K0 - alpha + 4 j] (both indices sum to L).  Unlike a
// Toeplitz-blocked 16 x 16 product, no block pairs a zero triangle with real
// work: the only extra products are the zero-padded ends of each tile's range.
//
// Steps come in chunks of 16: alpha = 16 c + s - 3 (s = 0..15).  Chunk c of
// tile t needs the sixteen values H'[16 c + s - 3 + r] (set A_c, per lane r) and
// P'[a0 + 16 u + 4 j - s] with u = t - c + U0 (set B_u, per lane j), so that a
// B set serves tile t at chunk c and tile t + 1 at chunk c + 1.  T tiles are
// processed together: each chunk loads one A set (shared by the T tiles) and one
// new B set into a ring of T sets, so LDS delivers 2 / T values per matrix op.
// T = 2 with four waves per block (about 120 registers: four waves per SIMD)
// measured faster than T = 4 with two (half the LDS reads per product, but
// about 220 registers and two waves per SIMD): 1.05 against 1.18 ms at
// 2048^2 x 512 x 256.
// The 4 x 4 x 1 operations share the vector unit's issue: every vector
// instruction in the loop costs matrix-core time, so the loop holds none but
// the folds.
//
// FP32 products are summed by the matrix core over 8 chunks (128 products per
// lag), then folded into a compensated (Kahan) sum per lag.
//
// LDS (per point, point-major): P' at position a + offP (a0 + offP = 15, so
// every B set starts on a 16-byte boundary) in a row of PSP floats, zero outside
// [0, nA); H' at position x + 3 in a row of PSH floats, zero outside [0, nHe).
// PSP = 16 (mod 32) keeps the 16-byte B reads of eight lanes on distinct banks,
// PSH = 4 (mod 32) the 4-byte A reads of 32 lanes.
#include <algorithm>
#include <type_traits>

#include "lh_internal.h"

namespace lh {

namespace {

typedef float f4v __attribute__((ext_vector_type(4)));

__device__ __forceinline__ f4v mfma4x4(float a, float b, f4v c)
{
    return __builtin_amdgcn_mfma_f32_4x4x1f32(a, b, c, 0, 0, 0);
}

constexpr int kPoints = 16;   // real-space points per block (one per MFMA block)
constexpr int kWaves = 4;     // waves per block, sharing the staged points
constexpr int kTiles = 2;     // lag tiles processed together (T), B sets in the ring
constexpr int kFoldChunks = 8;  // chunks (16 products each) summed in FP32 between folds (a multiple of T)
static_assert(kTiles >= 2 && kTiles % 2 == 0 && kFoldChunks % kTiles == 0, "ring phases alternate the A sets");

// f(integral_constant<I>) for I = 0 .. N-1, and for the one I equal to v
template <int N, int I = 0, typename F>
__device__ __forceinline__ void static_for(F &&f)
{
    if constexpr (I < N) {
        f(std::integral_constant<int, I>{});
        static_for<N, I + 1>(f);
    }
}
template <int N, int I = 0, typename F>
__device__ __forceinline__ void static_switch(int v, F &&f)
{
    if constexpr (I < N) {
        if (v == I)
            f(std::integral_constant<int, I>{});
        else
            static_switch<N, I + 1>(v, f);
    }
}

// Launch index -> logical block: the blocks of one XCD (launch index mod 8)
// take one contiguous range, so that neighbouring blocks (whose rows share
// 128-byte lines) meet in one L2 (the ragged tail keeps its index).
__device__ __forceinline__ unsigned xcd_block(unsigned b, unsigned n)
{
    const unsigned per = n >> 3;
    if (b >= (per << 3)) return b;
    return (b & 7) * per + (b >> 3);
}

// (s, c) += x, Kahan's compensated sum: s + c carries the rounding errors of
// the additions (4 operations; on this chip every vector operation in the
// product loop is paid for in matrix-core cycles).
__device__ __forceinline__ void kahan_add(float &s, float &c, float x)
{
    const float y = x - c;
    const float t = s + y;
    c = (t - s) - y;
    s = t;
}

__device__ __forceinline__ f4v buf_load4(__amdgpu_buffer_rsrc_t r, unsigned off)
{
    return __builtin_bit_cast(f4v, __builtin_amdgcn_raw_buffer_load_b128(r, (int)off, 0, 0));
}

// One block: 16 points staged in LDS by all its waves; the tile groups are
// then dealt out to the W waves and back (groups g with g mod 2W = w or
// 2W - 1 - w go to wave w): group g has about T (g + 1) chunks, so the shares
// are equal when the group count is a multiple of 2W.  Several blocks' waves
// share each SIMD, so one block's staging and operand loads overlap another's
// products.
// BIG: the staged slice ranges or the output reach past 4 GiB of byte
// offsets, so the block uses 64-bit addresses (flat loads and stores) instead
// of buffer descriptors.
template <bool BIG>
__device__ __forceinline__ void e3q_body(float *__restrict__ spec, const Geo &g)
{
    extern __shared__ __align__(16) unsigned char smem_raw[];
    const int PSP = g.e3q_PSP, PSH = g.e3q_PSH, LP = g.e3q_LP, LH = g.e3q_LH;
    float *Pl = reinterpret_cast<float *>(smem_raw);  // [16][PSP]
    float *Hl = Pl + (size_t)kPoints * PSP;           // [16][PSH]
    const int tid = threadIdx.x;
    const size_t sl = g.slice_e;
    const unsigned sl4 = (unsigned)(sl * 4);
    const size_t p0 = (size_t)xcd_block(blockIdx.x, gridDim.x) * kPoints;
    const int j0r = g.j0 - g.jA;
    const int nAst = g.e3q_nAst, nHst = g.e3q_nHst;

    // staging with buffer loads: P' row r (position r of the LDS row) holds
    // a = r - 16 - offP from slice j0 - 1 - a, relative slice
    // nAst - 1 + 16 + offP - r of the descriptor starting at slice j0 - nAst;
    // H' row r holds x = r - 3 from slice j0 + x.  Rows with no value fall
    // outside the descriptors' ranges (a negative offset wraps past them) and
    // read 0.  4 lanes per row, 16 bytes = 4 points each.
    {
        constexpr int RPI = 64 * kWaves / 4;  // rows per pass
        constexpr int UNR = 8;
        const int q = tid & 3, r0 = tid >> 2;
        const unsigned pb4 = (unsigned)((p0 + 4 * q) * 4);
        const __amdgpu_buffer_rsrc_t rP = __builtin_amdgcn_make_buffer_rsrc(
            (void *)(spec + (size_t)(j0r - nAst) * sl), 0, (int)((size_t)nAst * sl * 4), 0x00020000);
        const __amdgpu_buffer_rsrc_t rH =
            __builtin_amdgcn_make_buffer_rsrc((void *)(spec + (size_t)j0r * sl), 0, (int)((size_t)nHst * sl * 4), 0x00020000);
        auto stage = [&](__amdgpu_buffer_rsrc_t rs, float *dst0, int npos, unsigned off0, int dir) {
            // row r: offset off0 + dir r sl4 (unsigned wrap for the zero rows)
            for (int rb = r0; rb < npos; rb += UNR * RPI) {
                const unsigned ob = off0 + (unsigned)(dir * rb) * sl4;
                f4v v[UNR];
#pragma unroll
                for (int k = 0; k < UNR; ++k) v[k] = buf_load4(rs, ob + (unsigned)(dir * k * RPI) * sl4);
#pragma unroll
                for (int k = 0; k < UNR; ++k) {
                    if (rb + k * RPI < npos) {
#pragma unroll
                        for (int e = 0; e < 4; ++e) dst0[e * (dir > 0 ? PSH : PSP) + rb + k * RPI] = v[k][e];
                    }
                }
            }
        };
        // 64-bit form: row r of P' is slice j0 - 1 - (r - 16 - offP) when that
        // holds a value, of H' slice j0 + r - 3; other rows read 0
        auto stage64 = [&](float *dst0, int st, int npos, int vlo, int vhi, long slice0, int dir) {
            const float *src0 = spec + p0 + 4 * q;
            for (int rb = r0; rb < npos; rb += UNR * RPI) {
                f4v v[UNR];
#pragma unroll
                for (int k = 0; k < UNR; ++k) {
                    const int r = rb + k * RPI;
                    const bool ok = r >= vlo && r < vhi;
                    const f4v x4 = *reinterpret_cast<const f4v *>(src0 + (ok ? (size_t)(slice0 + (long)dir * r) * sl : 0));
                    v[k] = ok ? x4 : f4v{0.f, 0.f, 0.f, 0.f};
                }
#pragma unroll
                for (int k = 0; k < UNR; ++k) {
                    if (rb + k * RPI < npos) {
#pragma unroll
                        for (int e = 0; e < 4; ++e) dst0[e * st + rb + k * RPI] = v[k][e];
                    }
                }
            }
        };
        const int offP = g.e3q_offP;
        if constexpr (BIG) {
            stage64(Pl + (size_t)(4 * q) * PSP, PSP, LP, 16 + offP, 16 + offP + nAst, (long)j0r - 1 + 16 + offP, -1);
            stage64(Hl + (size_t)(4 * q) * PSH, PSH, LH, 3, 3 + nHst, (long)j0r - 3, 1);
        } else {
            stage(rP, Pl + (size_t)(4 * q) * PSP, LP, pb4 + (unsigned)(nAst - 1 + 16 + offP) * sl4, -1);
            stage(rH, Hl + (size_t)(4 * q) * PSH, LH, pb4 - 3u * sl4, 1);
        }
    }
    __syncthreads();

    const int lane = tid & 63, wave = tid >> 6;
    const int b = lane >> 2, qd = lane & 3;
    const float *Pb = Pl + (size_t)b * PSP + 4 * qd + 16;  // B set u (-1 <= u <= umax + 1) at Pb + 16 u
    const float *Hb = Hl + (size_t)b * PSH + qd;           // A set c: Hb[16 c + s]
    const int nT = g.e3q_nT, U0 = g.e3q_U0, umax = g.e3q_umax, cmax = g.e3q_cmax, nL = g.nL;
    const int G = (nT + kTiles - 1) / kTiles;
    // output slot 16 t + i + 4 qd of point p0 + b
    const __amdgpu_buffer_rsrc_t rO =
        __builtin_amdgcn_make_buffer_rsrc((void *)spec, 0, (int)((size_t)nL * sl * 4), 0x00020000);
    const unsigned ob0 = (unsigned)((p0 + b) * 4) + (unsigned)(4 * qd) * sl4;

    for (int gi = 0; gi < G; ++gi) {
        // groups dealt out and back (0, 1, .., W-1, W-1, .., 0, ...): the work of a
        // group grows with its lags, so every wave gets a balanced share
        const int gm = gi % (2 * kWaves);
        if ((gm < kWaves ? gm : 2 * kWaves - 1 - gm) != wave) continue;
        const int t0 = kTiles * gi;
        float sum[kTiles][4], cmp[kTiles][4];
#pragma unroll
        for (int k = 0; k < kTiles; ++k)
#pragma unroll
            for (int i = 0; i < 4; ++i) sum[k][i] = cmp[k][i] = 0.f;
        f4v ring[kTiles][4];
        // a set out of range reads a zero row (u = -1 or umax + 1)
        auto loadB = [&](int u, f4v(&dst)[4]) {
            const int uc = min(max(u, -1), umax + 1);
            const f4v *src = reinterpret_cast<const f4v *>(Pb + 16 * uc);
#pragma unroll
            for (int e = 0; e < 4; ++e) dst[e] = src[e];
        };
        const int cf = max(0, t0 + U0 - umax), cl = min(cmax, t0 + kTiles - 1 + U0);
        // slots 1 .. T-1 hold the sets of tiles 1 .. T-1 at chunk cf; chunk
        // cc at ring phase R loads the set of tile 0 into slot (-R) mod T and
        // tile k reads slot (k - R) mod T (its set was tile k-1's one chunk ago)
#pragma unroll
        for (int k = 1; k < kTiles; ++k) loadB(t0 + k + U0 - cf, ring[k]);
        f4v acc[kTiles];
#pragma unroll
        for (int k = 0; k < kTiles; ++k) acc[k] = f4v{0.f, 0.f, 0.f, 0.f};
        // tiles k < KLO are past their last chunk (their B set is u < 0): no
        // products.  The A set of the next chunk is loaded while this one is
        // on the matrix cores (two register sets alternating with the phase).
        float Ab[2][16];
        auto loadA = [&](int cc, float(&dst)[16]) {
            const int cq = min(cc, cmax);  // past the last chunk: any row in range
#pragma unroll
            for (int s = 0; s < 16; ++s) dst[s] = Hb[16 * cq + s];
        };
        auto chunk = [&](auto R, int cc, auto KLO) {
            constexpr int r = decltype(R)::value % kTiles;
            constexpr int klo = decltype(KLO)::value;
            constexpr int cur = decltype(R)::value & 1;
            loadB(t0 + U0 - cc, ring[(kTiles - r) % kTiles]);
            loadA(cc + 1, Ab[cur ^ 1]);
            const float(&A)[16] = Ab[cur];
#pragma unroll
            for (int s = 0; s < 16; ++s)
#pragma unroll
                for (int k = klo; k < kTiles; ++k)
                    acc[k] = mfma4x4(A[s], ring[(k - r + kTiles) % kTiles][(15 - s) >> 2][(15 - s) & 3], acc[k]);
        };
        using I0 = std::integral_constant<int, 0>;
        auto fold = [&]() {
#pragma unroll
            for (int k = 0; k < kTiles; ++k) {
#pragma unroll
                for (int i = 0; i < 4; ++i) kahan_add(sum[k][i], cmp[k][i], acc[k][i]);
                acc[k] = f4v{0.f, 0.f, 0.f, 0.f};
            }
        };
        // chunks up to t0 + U0 feed every tile of the group; in the last T - 1
        // chunks after it, tile k < cc - t0 - U0 has no more terms
        const int cm = min(cl, t0 + U0);
        int c = cf, nbody = 0;
        loadA(cf, Ab[0]);  // phase 0 of the first chunk
        for (; c + kTiles - 1 <= cm; c += kTiles) {
            static_for<kTiles>([&](auto R) { chunk(R, c + decltype(R)::value, I0{}); });
            if ((++nbody & (kFoldChunks / kTiles - 1)) == 0) fold();
        }
        // the remaining 0 .. T-1 chunks of the full part (ring phase 0 after
        // whole bodies), then the tail at the phase where they stop
        const int rem = max(0, cm - c + 1);
        static_for<kTiles - 1>([&](auto R) {
            if (rem > decltype(R)::value) chunk(R, c + decltype(R)::value, I0{});
        });
        const int ct = c + rem;  // first tail chunk (t0 + U0 + 1 unless clipped)
        // (cf <= t0 + U0 always, so a tail, if any, starts at t0 + U0 + 1);
        // tail chunk i leaves out the tiles k <= i, which are past their last chunk
        if (ct <= cl) {
            static_switch<kTiles>(rem, [&](auto P) {
                constexpr int ph = decltype(P)::value;
                static_for<kTiles - 1>([&](auto I) {
                    constexpr int i = decltype(I)::value;
                    if (ct + i <= cl) chunk(std::integral_constant<int, ph + i>{}, ct + i, std::integral_constant<int, i + 1>{});
                });
            });
        }
        fold();
        // every input of these points is in LDS, so the slices may be
        // overwritten
#pragma unroll
        for (int k = 0; k < kTiles; ++k) {
            const int t = t0 + k;
            if (t >= nT) break;
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                const int slot = 16 * t + i + 4 * qd;
                if (slot < nL) {
                    if constexpr (BIG)
                        spec[(size_t)slot * sl + p0 + b] = sum[k][i] - cmp[k][i];
                    else
                        __builtin_amdgcn_raw_buffer_store_b32(__builtin_bit_cast(unsigned, sum[k][i] - cmp[k][i]),
                                                              rO, (int)(ob0 + (unsigned)(16 * t + i) * sl4), 0, 0);
                }
            }
        }
    }
}

template <bool BIG>
__global__ void __launch_bounds__(64 * kWaves) k_e3q(float *__restrict__ spec, Geo g)
{
    e3q_body<BIG>(spec, g);
}
// Batched form: instance blockIdx.z of the descriptors
template <bool BIG>
__global__ void __launch_bounds__(64 * kWaves) k_e3q_batch(const EvenInst *__restrict__ in)
{
    const EvenInst &d = in[blockIdx.z];
    const Geo g = d.g;
    e3q_body<BIG>((float *)d.spec, g);
}

}  // namespace

// LDS bytes of one block (16 points).
size_t e3q_lds_bytes(const Geo &g, int)
{
    return (size_t)kPoints * (g.e3q_PSP + g.e3q_PSH) * sizeof(float);
}

hipError_t launch_e3q(const Plan &pl, int, hipStream_t st)
{
    const Geo &g = pl.g;
    const dim3 grid((unsigned)((g.slice_e + kPoints - 1) / kPoints));
    if (g.e3q_big)
        hipLaunchKernelGGL(k_e3q<true>, grid, dim3(64 * kWaves), e3q_lds_bytes(g, 1), st, (float *)pl.spec, g);
    else
        hipLaunchKernelGGL(k_e3q<false>, grid, dim3(64 * kWaves), e3q_lds_bytes(g, 1), st, (float *)pl.spec, g);
    return hipGetLastError();
}

// The window of a batched group (all with this schedule and grid): one launch,
// the LDS of its largest instance, 64-bit addressing if any instance needs it.
hipError_t launch_e3q_group(const Plan *const *pls, int n, const EvenInst *d_desc, hipStream_t st)
{
    size_t lds = 0;
    bool big = false;
    for (int i = 0; i < n; ++i) {
        lds = std::max(lds, e3q_lds_bytes(pls[i]->g, 1));
        big = big || pls[i]->g.e3q_big;
    }
    const dim3 grid((unsigned)((pls[0]->g.slice_e + kPoints - 1) / kPoints), 1, (unsigned)n);
    if (big)
        hipLaunchKernelGGL(k_e3q_batch<true>, grid, dim3(64 * kWaves), lds, st, d_desc);
    else
        hipLaunchKernelGGL(k_e3q_batch<false>, grid, dim3(64 * kWaves), lds, st, d_desc);
    return hipGetLastError();
}

}  // namespace lh
