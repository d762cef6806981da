// HIP kernels of the D3Q39 13-moment DDF lattice Boltzmann step for gfx950.
//
// The hot kernels, step_kernel_f64, step_kernel_f32 and step_kernel_f16 (one
// per storage mode), are the fused pull-stream-and-collide step of Sec. 3 of
// the paper for f and g: each lane gathers the 78 populations of one cell
// from shells up to three cells away, takes the moments, solves the 13
// Lagrange multipliers by warm-started Newton (Sec. 5 table), evaluates the
// Knudsen sensor (Eq. eq:DeltaAvg) and alpha (Eq. eq:alpha), and writes the
// BGK-relaxed populations to the other ping-pong buffer.  diag_kernel
// evaluates the same step up to the sensor, with a gather into registers.
//
// Memory layout (structure of arrays, x fastest): a population buffer is
// [f_0..f_38, g_0..g_38][n]; the multipliers are [13][n].  A wave owns 64
// consecutive cells of one x-row, so every population load and store of a
// wave is one contiguous 64-element run (unaligned by at most three elements
// for the shifted sources).  Work is handed out in blocks of four row
// segments; block b of a launch is mapped onto a contiguous range of segments
// per XCD so that neighbouring rows, which share cache lines at the run ends,
// meet in the same L2.
#include <hip/hip_runtime.h>

#include <mutex>

#include "equilibrium.h"
#include "slot.h"

namespace lbm13 {

template <class S>
struct StoreTraits;
template <>
struct StoreTraits<double> {
    using C = double;
    static constexpr bool kShift = false;
    static constexpr bool kScale = false;
    static constexpr int kWavesPerSimd = 1;  // FP64 arithmetic needs the full register file
    // f_i and g_i of a cell side by side: one 16-byte record per cell and
    // velocity, so that one 16-byte transfer per lane moves both
    static constexpr bool kPaired = true;
};

// Global-memory pointers (address space 1): loads and stores then use a
// uniform 64-bit base in SGPRs plus a 32-bit per-lane byte offset.
using gbyte = char __attribute__((address_space(1)));
using gcbyte = const char __attribute__((address_space(1)));

template <class S>
__device__ __forceinline__ S gload(gcbyte *base, uint32_t off)
{
    return *reinterpret_cast<const S __attribute__((address_space(1))) *>(base + off);
}
template <class S>
__device__ __forceinline__ S gload64(gcbyte *base, uint64_t off)
{
    return *reinterpret_cast<const S __attribute__((address_space(1))) *>(base + off);
}
template <class S>
__device__ __forceinline__ void gstore(gbyte *base, uint32_t off, S v)
{
    *reinterpret_cast<S __attribute__((address_space(1))) *>(base + off) = v;
}

// LDS parking of the gathered populations during the Newton solve: each lane
// owns column threadIdx.x of a [78][256] array (no cross-lane sharing, so no
// barriers).  Values are parked in the arithmetic type of the path.
template <class C>
struct Park {
    C *base;  // &lds[0][threadIdx.x]
    __device__ __forceinline__ void put(int i, C v) const { base[i * kBlockThreads] = v; }
    __device__ __forceinline__ C get(int i) const { return base[i * kBlockThreads]; }
    // f_i and g_i together
    __device__ __forceinline__ void put2(int i, C f, C g) const
    {
        put(i, f);
        put(kQ + i, g);
    }
};

// Running moments of the gathered populations: mass, momentum, and the
// energy sum f |xi|^2 + g (Sec. 3 and the first row of the Sec. 5 table).
template <class C>
struct MomentAcc {
    C rho, j[3], e, sg;
};

template <>
struct StoreTraits<float> {
    using C = float;
    static constexpr bool kShift = true;
    static constexpr bool kScale = false;
    static constexpr int kWavesPerSimd = 2;  // 256 registers per lane, LDS for the parked populations
    static constexpr bool kPaired = false;   // one plane per population
};
template <>
struct StoreTraits<_Float16> {
    using C = float;
    static constexpr bool kShift = true;
    static constexpr bool kScale = true;  // deviations stored divided by a power of two per shell
    static constexpr int kWavesPerSimd = 2;
    static constexpr bool kPaired = true;  // one dword (f_i, g_i) per cell and velocity
};

// Where population pop (0..38 f, 39..77 g) of a cell sits in a population
// buffer of n cells: paired storage keeps [39][n][2] (f_i, g_i), the other
// modes [78][n].
template <class S>
__device__ __forceinline__ int64_t pidx(int pop, int64_t cell, int64_t n)
{
    if constexpr (StoreTraits<S>::kPaired) return (int64_t)(pop % kQ) * 2 * n + 2 * cell + (pop >= kQ ? 1 : 0);
    else return (int64_t)pop * n + cell;
}
// bytes per cell in one velocity's plane, and byte offsets of the f and g
// planes of velocity i from the buffer base
template <class S>
constexpr uint32_t kCellBytes = StoreTraits<S>::kPaired ? 2 * sizeof(S) : sizeof(S);
template <class S>
__device__ __forceinline__ uint64_t fplane(int i, int64_t n)
{
    return (uint64_t)i * (uint64_t)n * kCellBytes<S>;
}
template <class S>
__device__ __forceinline__ uint64_t gplane(int i, int64_t n)
{
    if constexpr (StoreTraits<S>::kPaired) return fplane<S>(i, n) + sizeof(S);
    else return fplane<S>(kQ + i, n);
}

// Coordinate of the pull source along one axis, for a cell at coordinate v
// and velocity component c: periodic axes wrap; Neumann faces read the
// nearest interior layer (index 3 or n - 4); on equilibrium faces the source
// is the frozen layer itself.
__device__ __forceinline__ int source_coord(int v, int c, int n, int periodic, int nlo, int nhi)
{
    int s = v - c;
    if (periodic) {
        s = s < 0 ? s + n : s;
        s = s < 0 ? s + n : s;
        s = s < 0 ? s + n : s;
        s = s >= n ? s - n : s;
        s = s >= n ? s - n : s;
        s = s >= n ? s - n : s;
    } else {
        s = (nlo && s < 3) ? 3 : s;
        s = (nhi && s >= n - 3) ? n - 4 : s;
    }
    return s;
}

__device__ __forceinline__ bool is_fluid_coord(const SlotDesc &d, int x, int y, int z)
{
    const int c[3] = {x, y, z};
    const int n[3] = {d.nx, d.ny, d.nz};
    bool f = true;
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        f = f && !(d.open_lo[a] && c[a] < 3);
        f = f && !(d.open_hi[a] && c[a] >= n[a] - 3);
    }
    return f;
}

// wave-level integer reductions (64 lanes)
__device__ __forceinline__ int32_t wave_sum(int32_t v)
{
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    return v;
}
__device__ __forceinline__ int32_t wave_max(int32_t v)
{
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) {
        const int32_t w = __shfl_xor(v, o, 64);
        v = w > v ? w : v;
    }
    return v;
}

// Gather of one opposite pair p (velocities a = 2p+1 with c_p and b = 2p+2
// with -c_p) into a fluid cell, for read-outs (register loads).  Both
// populations are addressed from the planes of velocity a, so that a half-way
// bounce-back (which reads the cell's own opposite population) is an offset
// from the same base; nP is the byte distance from plane a to plane b:
//   f_a: from x - c_p, or when blocked f_b at the cell  (offset nP + cell)
//   f_b: from x + c_p, or when blocked f_a at the cell  (offset cell)
template <int P, class S, class C>
__device__ __forceinline__ void gather_pair(const SlotDesc &d, gcbyte *srcb, uint64_t nP, uint32_t cellS,
                                            uint64_t links, const uint32_t (&Xo)[7], const uint32_t (&Yo)[7],
                                            const uint32_t (&Zo)[7], const Park<C> &pk, MomentAcc<C> &acc)
{
    constexpr int a = 2 * P + 1, b = 2 * P + 2;
    constexpr int cx = kPairVel[P][0], cy = kPairVel[P][1], cz = kPairVel[P][2];
    uint64_t oa = Xo[cx + 3] + (Yo[cy + 3] + Zo[cz + 3]);
    uint64_t ob = nP + (Xo[3 - cx] + (Yo[3 - cy] + Zo[3 - cz]));
    oa = ((links >> a) & 1ull) ? nP + cellS : oa;
    ob = ((links >> b) & 1ull) ? (uint64_t)cellS : ob;
    gcbyte *bf = srcb + fplane<S>(a, d.n);
    gcbyte *bg = srcb + gplane<S>(a, d.n);
    C fa = C(gload64<S>(bf, oa)), fb = C(gload64<S>(bf, ob));
    C ga = C(gload64<S>(bg, oa)), gb = C(gload64<S>(bg, ob));
    if constexpr (StoreTraits<S>::kScale) {
        const C sf = C(d.shell_scale[0][shell(a)]), sg = C(d.shell_scale[1][shell(a)]);
        fa *= sf;
        fb *= sf;
        ga *= sg;
        gb *= sg;
    }
    if constexpr (StoreTraits<S>::kShift) {
        // a blocked link gathered the opposite velocity's deviation: move it
        // onto this velocity's shift weight (zero for symmetric weights)
        if (d.asym_bounce) {
            const bool ba = (links >> a) & 1ull, bb = (links >> b) & 1ull;
            fa = ba ? fa + C(d.bb_corr[a]) : fa;
            ga = ba ? ga + C(d.bb_corr[kQ + a]) : ga;
            fb = bb ? fb + C(d.bb_corr[b]) : fb;
            gb = bb ? gb + C(d.bb_corr[kQ + b]) : gb;
        }
    }
    pk.put(a, fa);
    pk.put(b, fb);
    pk.put(kQ + a, ga);
    pk.put(kQ + b, gb);
    const C sp = fa + fb, ap = fa - fb;
    acc.rho += sp;
    acc.j[0] = Term<cx>::add(acc.j[0], ap);
    acc.j[1] = Term<cy>::add(acc.j[1], ap);
    acc.j[2] = Term<cz>::add(acc.j[2], ap);
    acc.e = Term<pair_q(P)>::add(acc.e, sp);
    acc.sg += ga + gb;
}

template <class S, class C, int... P>
__device__ __forceinline__ void gather_pairs(const SlotDesc &d, gcbyte *srcb, uint64_t nP, uint32_t cellS,
                                             uint64_t links, const uint32_t (&Xo)[7], const uint32_t (&Yo)[7],
                                             const uint32_t (&Zo)[7], const Park<C> &pk, MomentAcc<C> &acc,
                                             std::integer_sequence<int, P...>)
{
    (gather_pair<P, S, C>(d, srcb, nP, cellS, links, Xo, Yo, Zo, pk, acc), ...);
}

template <int I, class S, class C, class PK>
__device__ __forceinline__ C eps_term(const SlotDesc &d, C rho, C f0, const C *fp, const C *fm, const PK &pk)
{
    const C feq = rho * feq_of<I>(f0, fp, fm);
    const C hf = pk.get(I);
    C diff;
    if constexpr (StoreTraits<S>::kShift) diff = (C(d.shift_w[I]) - feq) + hf;
    else diff = hf - feq;
    return fabs(diff) * recip(feq);
}

template <class S, class C, class PK, int... I>
__device__ __forceinline__ C eps_sum(const SlotDesc &d, C rho, C f0, const C *fp, const C *fm, const PK &pk,
                                     std::integer_sequence<int, I...>)
{
    C e = C(-0.0);
    ((e += eps_term<I, S, C, PK>(d, rho, f0, fp, fm, pk)), ...);
    return e;
}

using VelSeq = std::make_integer_sequence<int, kQ>;

// One fluid cell of the next step up to the sensor: gather, moments, Newton,
// sensor.  Writes eps (NaN where the solve fails) to diag[cell] and the Newton
// iterations to diag[n + cell]; the state is left unchanged.  (y, z) are
// uniform across the wave; x is the lane's coordinate.
template <class S>
__device__ __forceinline__ void diag_cell(const SlotDesc &d, const S *src, int x, int y, int z, uint32_t cell,
                                          const Park<typename StoreTraits<S>::C> &pk, double *diag)
{
    using C = typename StoreTraits<S>::C;
    const uint64_t links = d.has_links ? d.links[cell] : 0ull;
    if (links >> 63) {  // solid
        diag[cell] = __builtin_nan("");
        diag[d.n + cell] = -1.0;
        return;
    }

    // byte offsets of the source coordinates x - c, c = -3..3, per axis,
    // within one velocity's plane
    constexpr uint32_t cb = kCellBytes<S>;
    const uint32_t nx = (uint32_t)d.nx, nxy = (uint32_t)d.nx * (uint32_t)d.ny;
    uint32_t Xo[7], Yo[7], Zo[7];
#pragma unroll
    for (int c = -3; c <= 3; ++c) {
        Xo[c + 3] = (uint32_t)source_coord(x, c, d.nx, d.axis[0] == kAxisPeriodic, d.neumann_lo[0], d.neumann_hi[0]) * cb;
        Yo[c + 3] = (uint32_t)source_coord(y, c, d.ny, d.axis[1] == kAxisPeriodic, d.neumann_lo[1], d.neumann_hi[1]) *
                    nx * cb;
        Zo[c + 3] = (uint32_t)source_coord(z, c, d.nz, d.axis[2] == kAxisPeriodic, d.neumann_lo[2], d.neumann_hi[2]) *
                    nxy * cb;
    }
    const uint64_t nP = (uint64_t)d.n * cb;
    const uint32_t cellS = cell * cb;
    gcbyte *srcb = (gcbyte *)src;

    // moments accumulate while the populations are parked (shifted storage
    // starts from the sums of the shift weights)
    MomentAcc<C> macc;
    if constexpr (StoreTraits<S>::kShift) {
        macc.rho = C(d.ref_mass);
        macc.j[0] = C(d.ref_mom[0]);
        macc.j[1] = C(d.ref_mom[1]);
        macc.j[2] = C(d.ref_mom[2]);
        macc.e = C(d.ref_energy);
    } else {
        macc.rho = C(-0.0);
        macc.j[0] = macc.j[1] = macc.j[2] = C(-0.0);
        macc.e = C(-0.0);
    }
    {
        C f0v = C(gload<S>(srcb + fplane<S>(0, d.n), cellS));
        C g0v = C(gload<S>(srcb + gplane<S>(0, d.n), cellS));
        if constexpr (StoreTraits<S>::kScale) {
            f0v *= C(d.shell_scale[0][0]);
            g0v *= C(d.shell_scale[1][0]);
        }
        pk.put(0, f0v);
        pk.put(kQ, g0v);
        macc.rho += f0v;
        macc.sg = g0v;
    }
    gather_pairs<S, C>(d, srcb, nP, cellS, links, Xo, Yo, Zo, pk, macc, PairSeq{});
    // keep the parked values out of registers across the solve
    __asm__ volatile("" ::: "memory");
    const C rho = macc.rho;
    const C j[3] = {macc.j[0], macc.j[1], macc.j[2]};
    const C e = macc.e + macc.sg;

    C lam[kM];
    gbyte *lamb = (gbyte *)d.lam;
    const uint64_t nC64 = (uint64_t)d.n * sizeof(C);
    const uint32_t cellC = cell * (uint32_t)sizeof(C);
#pragma unroll
    for (int k = 0; k < kM; ++k) lam[k] = gload<C>(lamb + (uint64_t)k * nC64, cellC);

    // correctly rounded divisions (an approximate reciprocal here would bias
    // T, and with it the total energy, by the same sign every step)
    C u[3];
    u[0] = j[0] / rho;
    u[1] = j[1] / rho;
    u[2] = j[2] / rho;
    const C T = (e - rho * (u[0] * u[0] + u[1] * u[1] + u[2] * u[2])) / (C(d.two_cv) * rho);

    C f0, fp[kPairs], fm[kPairs];
    int iters = 0;
    C G[kM];
    // a NaN lambda_0 marks a cell that had no equilibrium in the previous step
    const bool marked = !(lam[0] == lam[0]);
    int status;
    if constexpr (sizeof(C) == 8) {
        status = d.root_finder == 1
                     ? solve_multipliers_secant<C>(u, T, lam, f0, fp, fm, C(d.tol), d.maxit, d.maxit_cold,
                                                   marked ? kStartMarked : kStartWarm, iters, G, d.qn_h, d.qn_T_ref)
                     : solve_multipliers<C>(u, T, lam, f0, fp, fm, C(d.tol), d.maxit, d.maxit_cold,
                                            marked ? kStartMarked : kStartWarm, iters, G);
    } else {
        status = solve_multipliers<C>(u, T, lam, f0, fp, fm, C(d.tol), d.maxit, d.maxit_cold,
                                      marked ? kStartMarked : kStartWarm, iters, G);
    }
    if constexpr (sizeof(C) == 4) {
        // FP32 arithmetic stops at a tolerance far above FP64's; make the
        // collision invariants exact so that the bias of the last Newton
        // step (its mass and energy residuals are positive) does not
        // accumulate over time steps
        project_invariants(f0, fp, fm, u, T, G, status != kFailed);
    }

    // Knudsen sensor over f (Eq. eq:DeltaAvg)
    const C eps = eps_sum<S, C>(d, rho, f0, fp, fm, pk, VelSeq{}) * C(1.0 / kQ);
    // an equilibrium population that underflows makes its term, and eps,
    // infinite (0 * inf gives NaN where the gathered value underflows too)
    diag[cell] = status == kFailed ? __builtin_nan("") : (eps == eps ? (double)eps : __builtin_inf());
    diag[d.n + cell] = (double)iters;
}

// Locate the slot that owns logical block b (uniform across the block).
__device__ __forceinline__ int find_slot(const SlotTable *tab, int b)
{
    int s = 0;
    while (s + 1 < tab->nslots && tab->block_start[s + 1] <= b) ++s;
    return s;
}

// Diagnostics of the next step of one solve (slot 0 of tab, launch index j):
// the Knudsen sensor and the Newton iterations of every cell, from the
// current state, which is left unchanged.  diag: eps[n] then iterations[n]
// (FP64; NaN / -1 outside fluid cells, NaN eps where the solve fails).
template <class S>
__global__ __launch_bounds__(kBlockThreads, StoreTraits<S>::kWavesPerSimd) void diag_kernel(
    const SlotTable *__restrict__ tab, int j, double *__restrict__ diag)
{
    using C = typename StoreTraits<S>::C;
    __shared__ C park[2 * kQ * kBlockThreads];
    const Park<C> pk{park + threadIdx.x};
    const SlotDesc &d = tab->slot[0];
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int lane = threadIdx.x & 63;
    for (int b = blockIdx.x; b < d.blocks; b += gridDim.x) {
        const int64_t seg = (int64_t)b * kWavesPerBlock + wave;
        if (seg >= d.segments) continue;
        const int segx = (int)(seg % d.nsegx);
        const int row = (int)(seg / d.nsegx);
        const int y = row % d.ny;
        const int z = row / d.ny;
        const int x = segx * kSegment + lane;
        if (x >= d.nx) continue;
        const uint32_t cell = (uint32_t)x + (uint32_t)d.nx * ((uint32_t)y + (uint32_t)d.ny * (uint32_t)z);
        if (is_fluid_coord(d, x, y, z)) {
            const int par = (d.parity0 + j) & 1;
            const S *src = static_cast<const S *>(d.buf[par]);
            diag_cell<S>(d, src, x, y, z, cell, pk, diag);
        } else {
            diag[cell] = __builtin_nan("");
            diag[d.n + cell] = -1.0;
        }
    }
}

// ---------------------------------------------------------------------------
// FP32-shifted step: the gather goes global -> LDS directly (no registers,
// per-lane addresses, so wrap, clamps and bounce-back are unchanged), and the
// results leave LDS as 16-byte-per-lane stores of whole 64-cell rows.  Lanes
// of non-fluid cells gather their own values, so that a row can be stored
// whole without changing them.  Two waves per SIMD; each wave touches only
// its own LDS columns, so no barriers are needed.
namespace f32 {

using lds_float = float __attribute__((address_space(3)));
typedef float v4f __attribute__((ext_vector_type(4)));

// s_waitcnt vmcnt(0) (gfx9 encoding, expcnt and lgkmcnt at their maxima): the
// compiler does not track loads into LDS, so reads of gathered rows wait here
__device__ __forceinline__ void wait_vmem() { __builtin_amdgcn_s_waitcnt(0x0F70); }

__device__ __forceinline__ void dma4(gcbyte *gaddr, lds_float *row_base)
{
    __builtin_amdgcn_global_load_lds((const void __attribute__((address_space(1))) *)gaddr,
                                     (void __attribute__((address_space(3))) *)row_base, 4, 0, 0);
}

__device__ __forceinline__ float uniform(float v)
{
    return __builtin_bit_cast(float, __builtin_amdgcn_readfirstlane(__builtin_bit_cast(int, v)));
}

// gather of one cell's 78 FP32 values into the wave's LDS rows (row i at
// rows + i*256, one dword per lane); copy = the cell's own values
__device__ __forceinline__ void gather(const SlotDesc &d, gcbyte *srcb, int x, int y, int z, uint32_t cell,
                                       uint64_t links, bool copy, lds_float *rows)
{
    const uint64_t nS64 = (uint64_t)d.n * 4;
    const uint32_t nS = (uint32_t)nS64;
    const uint32_t cellS = cell * 4u;
    const uint32_t nx = (uint32_t)d.nx, nxy = (uint32_t)d.nx * (uint32_t)d.ny;
    uint32_t Xo[7], Yo[7], Zo[7];
#pragma unroll
    for (int c = -3; c <= 3; ++c) {
        Xo[c + 3] = (uint32_t)source_coord(x, c, d.nx, d.axis[0] == kAxisPeriodic, d.neumann_lo[0], d.neumann_hi[0]) * 4u;
        Yo[c + 3] = (uint32_t)source_coord(y, c, d.ny, d.axis[1] == kAxisPeriodic, d.neumann_lo[1], d.neumann_hi[1]) * nx * 4u;
        Zo[c + 3] = (uint32_t)source_coord(z, c, d.nz, d.axis[2] == kAxisPeriodic, d.neumann_lo[2], d.neumann_hi[2]) * nxy * 4u;
    }
    dma4(srcb + cellS, rows);
    dma4(srcb + (uint64_t)kQ * nS64 + cellS, rows + kQ * kBlockThreads);
#pragma unroll
    for (int p = 0; p < kPairs; ++p) {
        const int a = 2 * p + 1, b = 2 * p + 2;
        const int cx = kPairVel[p][0], cy = kPairVel[p][1], cz = kPairVel[p][2];
        uint32_t oa = Xo[cx + 3] + (Yo[cy + 3] + Zo[cz + 3]);
        uint32_t ob = nS + (Xo[3 - cx] + (Yo[3 - cy] + Zo[3 - cz]));
        oa = ((links >> a) & 1ull) ? nS + cellS : oa;
        ob = ((links >> b) & 1ull) ? cellS : ob;
        oa = copy ? cellS : oa;
        ob = copy ? nS + cellS : ob;
        gcbyte *bf = srcb + (uint64_t)a * nS64;
        gcbyte *bg = srcb + (uint64_t)(kQ + a) * nS64;
        dma4(bf + oa, rows + a * kBlockThreads);
        dma4(bf + ob, rows + b * kBlockThreads);
        dma4(bg + oa, rows + (kQ + a) * kBlockThreads);
        dma4(bg + ob, rows + (kQ + b) * kBlockThreads);
    }
}

// gather of one cell's 39 paired FP16 words (f_i in the low half, g_i in the
// high half) into the wave's LDS rows (row i at rows + i*256, one dword per
// lane); copy = the cell's own words.  A blocked link reads the opposite
// velocity's word at the cell itself, in another plane: waves with such a
// link (linked, uniform) take per-lane addresses, the others a uniform plane
// base plus a 32-bit offset.
__device__ __forceinline__ void gather_paired(const SlotDesc &d, gcbyte *srcb, int x, int y, int z, uint32_t cell,
                                              uint64_t links, bool copy, bool linked, lds_float *rows)
{
    const uint64_t nP = (uint64_t)d.n * 4;
    const uint32_t cellS = cell * 4u;
    const uint32_t nx = (uint32_t)d.nx, nxy = (uint32_t)d.nx * (uint32_t)d.ny;
    uint32_t Xo[7], Yo[7], Zo[7];
#pragma unroll
    for (int c = -3; c <= 3; ++c) {
        Xo[c + 3] = (uint32_t)source_coord(x, c, d.nx, d.axis[0] == kAxisPeriodic, d.neumann_lo[0], d.neumann_hi[0]) * 4u;
        Yo[c + 3] = (uint32_t)source_coord(y, c, d.ny, d.axis[1] == kAxisPeriodic, d.neumann_lo[1], d.neumann_hi[1]) * nx * 4u;
        Zo[c + 3] = (uint32_t)source_coord(z, c, d.nz, d.axis[2] == kAxisPeriodic, d.neumann_lo[2], d.neumann_hi[2]) * nxy * 4u;
    }
    dma4(srcb + cellS, rows);
    const uint64_t lk = copy ? 0ull : links;
#pragma unroll
    for (int p = 0; p < kPairs; ++p) {
        const int a = 2 * p + 1, b = 2 * p + 2;
        const int cx = kPairVel[p][0], cy = kPairVel[p][1], cz = kPairVel[p][2];
        uint32_t oa = Xo[cx + 3] + (Yo[cy + 3] + Zo[cz + 3]);
        uint32_t ob = Xo[3 - cx] + (Yo[3 - cy] + Zo[3 - cz]);
        oa = copy ? cellS : oa;
        ob = copy ? cellS : ob;
        gcbyte *pa = srcb + (uint64_t)a * nP, *pb = srcb + (uint64_t)b * nP;
        if (!linked) {
            dma4(pa + oa, rows + a * kBlockThreads);
            dma4(pb + ob, rows + b * kBlockThreads);
        } else {
            gcbyte *sa = ((lk >> a) & 1ull) ? pb + cellS : pa + oa;
            gcbyte *sb = ((lk >> b) & 1ull) ? pa + cellS : pb + ob;
            dma4(sa, rows + a * kBlockThreads);
            dma4(sb, rows + b * kBlockThreads);
        }
    }
}

// Paired FP16 storage seen through the FP32 park: row word i holds the stored
// halves of f_i (low) and g_i (high); reads decode (times the shell scale),
// writes encode
struct ParkHalf {
    uint32_t *base;  // &lds_words[0][threadIdx.x]
    const float *scale;      // shell scales of f (0..5) then g (6..11)
    const float *inv_scale;
    __device__ __forceinline__ float get(int i) const
    {
        const bool hi = i >= kQ;
        const int v = hi ? i - kQ : i;
        const uint32_t w = base[v * kBlockThreads];
        const uint16_t h = hi ? (uint16_t)(w >> 16) : (uint16_t)w;
        return (float)__builtin_bit_cast(_Float16, h) * scale[(hi ? 6 : 0) + shell(v)];
    }
    __device__ __forceinline__ void put(int i, float v) const
    {
        // a 16-bit write of one half
        const bool hi = i >= kQ;
        const int q = hi ? i - kQ : i;
        *(reinterpret_cast<uint16_t *>(base + q * kBlockThreads) + (hi ? 1 : 0)) =
            __builtin_bit_cast(uint16_t, (_Float16)(v * inv_scale[(hi ? 6 : 0) + shell(q)]));
    }
    __device__ __forceinline__ void put2(int i, float f, float g) const
    {
        const uint32_t lo = __builtin_bit_cast(uint16_t, (_Float16)(f * inv_scale[shell(i)]));
        const uint32_t hi = __builtin_bit_cast(uint16_t, (_Float16)(g * inv_scale[6 + shell(i)]));
        base[i * kBlockThreads] = lo | (hi << 16);
    }
};

// Blocked links of a cell whose opposite velocities have unequal shift
// weights: the gather brought the opposite velocity's stored deviation, which
// moves onto this velocity's weight here (FP16: re-encoded in its shell scale,
// which opposite velocities share)
template <class PK>
__device__ __forceinline__ void bounce_fix(const SlotDesc &d, const PK &pk, uint64_t links)
{
#pragma unroll
    for (int i = 1; i < kQ; ++i) {
        if ((links >> i) & 1ull) {
            pk.put(i, pk.get(i) + d.bb_corr[i]);
            pk.put(kQ + i, pk.get(kQ + i) + d.bb_corr[kQ + i]);
        }
    }
}

// parked values read per group in the sensor and the relaxation (two groups,
// 20 and 19; measured against 8 and 13)
constexpr int kChunk = 20;

// moments, Newton, sensor and relaxation of one fluid cell whose gathered
// values sit in LDS; the results replace them
template <class PK>
__device__ __forceinline__ void collide(const SlotDesc &d, uint32_t cell, const PK &pk, int32_t (&acc)[kStatWords])
{
    using C = float;
    C rho = C(d.ref_mass), j0 = C(d.ref_mom[0]), j1 = C(d.ref_mom[1]), j2 = C(d.ref_mom[2]), e = C(d.ref_energy);
    C sg = pk.get(kQ);
    rho += pk.get(0);
#pragma unroll
    for (int p = 0; p < kPairs; ++p) {
        const C fa = pk.get(2 * p + 1), fb = pk.get(2 * p + 2);
        const C sp = fa + fb, ap = fa - fb;
        rho += sp;
        j0 += C(kPairVel[p][0]) * ap;
        j1 += C(kPairVel[p][1]) * ap;
        j2 += C(kPairVel[p][2]) * ap;
        e += C(pair_q(p)) * sp;
        sg += pk.get(kQ + 2 * p + 1) + pk.get(kQ + 2 * p + 2);
    }
    e += sg;
    // the gathered values are read again after the solve, not kept in registers
    __asm__ volatile("" ::: "memory");
    C u[3];
    u[0] = j0 / rho;
    u[1] = j1 / rho;
    u[2] = j2 / rho;
    const C T = (e - rho * (u[0] * u[0] + u[1] * u[1] + u[2] * u[2])) / (C(d.two_cv) * rho);

    gbyte *lamb = (gbyte *)d.lam;
    const uint64_t nS64 = (uint64_t)d.n * 4;
    const uint32_t cellS = cell * 4u;
    C lam[kM];
#pragma unroll
    for (int k = 0; k < kM; ++k) lam[k] = gload<C>(lamb + (uint64_t)k * nS64, cellS);

    C f0, fp[kPairs], fm[kPairs];
    int iters = 0;
    C G[kM];
    // a NaN lambda_0 marks a cell that had no equilibrium in the previous
    // step: its warm start normalises the other multipliers and it is not
    // restarted cold
    const bool marked = !(lam[0] == lam[0]);
    const int status = solve_multipliers<C>(u, T, lam, f0, fp, fm, C(d.tol), d.maxit, d.maxit_cold,
                                            marked ? kStartMarked : kStartWarm, iters, G);
    const bool failed = status == kFailed;
    // the multipliers leave first (their registers are free for what follows)
    if (!failed) {
#pragma unroll
        for (int k = 0; k < kM; ++k) gstore<C>(lamb + (uint64_t)k * nS64, cellS, lam[k]);
    } else {
        gstore<C>(lamb, cellS, __builtin_nanf(""));  // the failure mark; lambda_1..12 kept
    }
    project_invariants(f0, fp, fm, u, T, G, !failed);

    // the Knudsen sensor with the parked values read kChunk at a time, each
    // group's LDS reads issued together (same terms, same order as eps_sum)
    C eps = C(-0.0);
#pragma unroll
    for (int i0 = 0; i0 < kQ; i0 += kChunk) {
        C hv[kChunk];
#pragma unroll
        for (int k = 0; k < kChunk; ++k)
            if (i0 + k < kQ) hv[k] = pk.get(i0 + k);
        __builtin_amdgcn_sched_barrier(0);
#pragma unroll
        for (int k = 0; k < kChunk; ++k) {
            const int i = i0 + k;
            if (i < kQ) {
                const C e_i = (i == 0) ? f0 : (((i - 1) & 1) == 0 ? fp[(i - 1) >> 1] : fm[(i - 1) >> 1]);
                const C feq = rho * e_i;
                const C diff = (C(d.shift_w[i]) - feq) + hv[k];
                eps += fabs(diff) * recip(feq);
            }
        }
    }
    eps *= C(1.0 / kQ);
    int br = 0;
    if (d.kn_relax) br = (eps < C(1e-2)) ? 0 : (eps < C(1e-1)) ? 1 : (eps < C(1)) ? 2 : 3;
    const C o0 = uniform(C(d.omega[0])), o1 = uniform(C(d.omega[1])), o2 = uniform(C(d.omega[2])),
            o3 = uniform(C(d.omega[3]));
    // a cell whose multipliers were not found is not collided (omega = 0
    // against the finite values the solver leaves): gathered values stored
    // unchanged, multipliers kept for the next warm start
    C omega = o0;
    omega = br == 1 ? o1 : omega;
    omega = br == 2 ? o2 : omega;
    omega = br == 3 ? o3 : omega;
    omega = failed ? C(0) : omega;
    const C dT = C(d.delta) * T;
    __asm__ volatile("" ::: "memory");
#pragma unroll
    for (int i0 = 0; i0 < kQ; i0 += kChunk) {
        C hf[kChunk], hg[kChunk];
#pragma unroll
        for (int k = 0; k < kChunk; ++k) {
            if (i0 + k < kQ) {
                hf[k] = pk.get(i0 + k);
                hg[k] = pk.get(kQ + i0 + k);
            }
        }
        __builtin_amdgcn_sched_barrier(0);
#pragma unroll
        for (int k = 0; k < kChunk; ++k) {
            const int i = i0 + k;
            if (i < kQ) {
                const C e_i = (i == 0) ? f0 : (((i - 1) & 1) == 0 ? fp[(i - 1) >> 1] : fm[(i - 1) >> 1]);
                const C feq = rho * e_i;
                const C geq = dT * feq;
                pk.put2(i, hf[k] + omega * ((feq - C(d.shift_w[i])) - hf[k]),
                        hg[k] + omega * ((geq - C(d.shift_w[kQ + i])) - hg[k]));
            }
        }
    }

    acc[0] += iters;
    acc[1] = iters > acc[1] ? iters : acc[1];
    acc[2] += failed;
    acc[3] += status == kConvergedCold || (failed && !marked);  // cold restarts tried
    acc[4] += !failed && br == 0;
    acc[5] += !failed && br == 1;
    acc[6] += !failed && br == 2;
    acc[7] += !failed && br == 3;
}

}  // namespace f32

// kWide: grids of 2^28 cells or more, whose row stores take 64-bit lane
// addresses (a separate instantiation keeps the common case's registers)
template <bool kWide>
__global__ __launch_bounds__(kBlockThreads, 2) void step_kernel_f32(const SlotTable *__restrict__ tab, int j,
                                                                   int64_t *__restrict__ stats)
{
    __shared__ float park[2 * kQ * kBlockThreads];
    const Park<float> pk{park + threadIdx.x};
    int32_t acc[kStatWords] = {0, 0, 0, 0, 0, 0, 0, 0, 0, 0};
    const int total = tab->total_blocks;
    const int xcd = blockIdx.x & 7;
    const int per_xcd = gridDim.x >> 3;
    const int lo = (int)(((int64_t)total * xcd) >> 3);
    const int hi = (int)(((int64_t)total * (xcd + 1)) >> 3);
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int lane = threadIdx.x & 63;
    f32::lds_float *rows = (f32::lds_float *)park + wave * kSegment;
    for (int b = lo + (int)(blockIdx.x >> 3); b < hi; b += per_xcd) {
        const int s = find_slot(tab, b);
        const SlotDesc &d = tab->slot[s];
        if (j >= d.steps_todo) continue;
        const int64_t seg = (int64_t)(b - tab->block_start[s]) * kWavesPerBlock + wave;
        if (seg >= d.segments) continue;
        const int segx = (int)(seg % d.nsegx);
        const int row = (int)(seg / d.nsegx);
        const int y = row % d.ny;
        const int z = row / d.ny;
        const int x = segx * kSegment + lane;
        const uint32_t cell0 = (uint32_t)(segx * kSegment) + (uint32_t)d.nx * (uint32_t)row;
        const bool full = (segx * kSegment + kSegment <= d.nx) && (d.nx % 4 == 0);
        const bool in_grid = x < d.nx;
        const uint32_t cell = cell0 + (uint32_t)lane;
        const int par = (d.parity0 + j) & 1;
        gcbyte *srcb = (gcbyte *)d.buf[par];
        gbyte *dstb = (gbyte *)d.buf[par ^ 1];
        bool fluid = in_grid && is_fluid_coord(d, x, y, z);
        uint64_t links = 0;
        if (fluid && d.has_links) links = d.links[cell];
        if (links >> 63) fluid = false;  // solid cells pass through unchanged
        // the memory phase (row stores, then the next gather) issues ahead of
        // the other waves' arithmetic
        __builtin_amdgcn_s_setprio(1);
        if (in_grid) f32::gather(d, srcb, x, y, z, cell, links, !fluid, rows);
        __builtin_amdgcn_s_setprio(0);
        f32::wait_vmem();
        int32_t it_cell = 0;
        if (fluid) {
            if (d.asym_bounce && links) f32::bounce_fix(d, pk, links);
            const int32_t before = acc[0];
            f32::collide(d, cell, pk, acc);
            it_cell = acc[0] - before;
        }
        if (stats) {
            const int32_t wmax = wave_max(it_cell);
            acc[8] += lane == 0 ? wmax : 0;
            acc[9] += lane == 0 ? 1 : 0;
        }
        // store the wave's rows
        __builtin_amdgcn_s_setprio(1);
        const uint64_t nS64 = (uint64_t)d.n * 4;
        const float *col = park + wave * kSegment;
        if (full && !kWide) {
            // lanes 16r..16r+15 store row i0 + r, 4 cells each: one uniform
            // base per group of 4 rows and one 32-bit lane offset (4 planes
            // of 4n bytes stay below 2^32 for n < 2^28)
            const int r = lane >> 4, c4 = (lane & 15) * 4;
            uint32_t voff = (uint32_t)r * (uint32_t)nS64 + (cell0 + (uint32_t)c4) * 4u;
            const float *lcol = col + r * kBlockThreads + c4;
            __asm__ volatile("" : "+v"(voff));
#pragma unroll
            for (int i0 = 0; i0 < 2 * kQ; i0 += 4) {
                if (i0 + r < 2 * kQ) {
                    const f32::v4f v = *reinterpret_cast<const f32::v4f *>(lcol + i0 * kBlockThreads);
                    // streaming store: the next step reads these rows long after
                    // the caches have turned over
                    __builtin_nontemporal_store(
                        v, reinterpret_cast<f32::v4f __attribute__((address_space(1))) *>(dstb + (uint64_t)i0 * nS64 + voff));
                }
            }
        } else if (full) {
            // 2^28 cells or more: the same stores from a 64-bit lane address
            const int r = lane >> 4, c4 = (lane & 15) * 4;
            gbyte *lane_base = dstb + (uint64_t)r * nS64 + (uint64_t)(cell0 + (uint32_t)c4) * 4u;
            const float *lcol = col + r * kBlockThreads + c4;
#pragma unroll
            for (int i0 = 0; i0 < 2 * kQ; i0 += 4) {
                if (i0 + r < 2 * kQ) {
                    const f32::v4f v = *reinterpret_cast<const f32::v4f *>(lcol + i0 * kBlockThreads);
                    __builtin_nontemporal_store(
                        v, reinterpret_cast<f32::v4f __attribute__((address_space(1))) *>(lane_base + (uint64_t)i0 * nS64));
                }
            }
        } else if (in_grid) {
#pragma unroll
            for (int i = 0; i < 2 * kQ; ++i) gstore<float>(dstb + (uint64_t)i * nS64, cell * 4u, col[i * kBlockThreads + lane]);
        }
    }
    if (stats) {
        int64_t red[kStatWords];
#pragma unroll
        for (int k = 0; k < kStatWords; ++k) red[k] = (k == 1) ? wave_max(acc[k]) : wave_sum(acc[k]);
        if (lane == 0) {
            int64_t *p = stats + ((int64_t)blockIdx.x * kWavesPerBlock + wave) * kStatWords;
#pragma unroll
            for (int k = 0; k < kStatWords; ++k) p[k] = (k == 1) ? (red[k] > p[k] ? red[k] : p[k]) : p[k] + red[k];
        }
    }
}

// ---------------------------------------------------------------------------
// FP16-shifted step with the FP32 step's structure.  Storage is paired: one
// dword per cell and velocity holds the halves of f_i (low) and g_i (high),
// so the gather is 39 dword transfers global -> LDS per 64-cell segment.
// FP32 arithmetic runs through the decoding park, results are encoded back
// into the row words, and full rows leave as 16-byte-per-lane stores of four
// cells (four rows per instruction).
template <bool kStats, bool kWide>
__global__ __launch_bounds__(kBlockThreads, 2) void step_kernel_f16(const SlotTable *__restrict__ tab, int j,
                                                                   int64_t *__restrict__ stats)
{
    __shared__ uint32_t park[kQ * kBlockThreads];
    int32_t acc[kStatWords] = {0, 0, 0, 0, 0, 0, 0, 0, 0, 0};
    const int total = tab->total_blocks;
    const int xcd = blockIdx.x & 7;
    const int per_xcd = gridDim.x >> 3;
    const int lo = (int)(((int64_t)total * xcd) >> 3);
    const int hi = (int)(((int64_t)total * (xcd + 1)) >> 3);
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int lane = threadIdx.x & 63;
    f32::lds_float *rows = (f32::lds_float *)park + wave * kSegment;
    for (int b = lo + (int)(blockIdx.x >> 3); b < hi; b += per_xcd) {
        const int s = find_slot(tab, b);
        const SlotDesc &d = tab->slot[s];
        if (j >= d.steps_todo) continue;
        const int64_t seg = (int64_t)(b - tab->block_start[s]) * kWavesPerBlock + wave;
        if (seg >= d.segments) continue;
        const int segx = (int)(seg % d.nsegx);
        const int row = (int)(seg / d.nsegx);
        const int y = row % d.ny;
        const int z = row / d.ny;
        const int x = segx * kSegment + lane;
        const uint32_t cell0 = (uint32_t)(segx * kSegment) + (uint32_t)d.nx * (uint32_t)row;
        // 16-byte stores of four cells need a row start on a 4-cell boundary
        const bool full = (segx * kSegment + kSegment <= d.nx) && (d.nx % 4 == 0);
        const bool in_grid = x < d.nx;
        const uint32_t cell = cell0 + (uint32_t)lane;
        const int par = (d.parity0 + j) & 1;
        gcbyte *srcb = (gcbyte *)d.buf[par];
        gbyte *dstb = (gbyte *)d.buf[par ^ 1];
        bool fluid = in_grid && is_fluid_coord(d, x, y, z);
        uint64_t links = 0;
        if (fluid && d.has_links) links = d.links[cell];
        if (links >> 63) fluid = false;  // solid cells pass through unchanged
        const bool linked = __builtin_amdgcn_ballot_w64(fluid && links != 0) != 0;
        // the memory phase (row stores, then the next gather) issues ahead of
        // the other waves' arithmetic
        __builtin_amdgcn_s_setprio(1);
        if (in_grid) f32::gather_paired(d, srcb, x, y, z, cell, links, !fluid, linked, rows);
        __builtin_amdgcn_s_setprio(0);
        f32::wait_vmem();
        int32_t it_cell = 0;
        if (fluid) {
            const f32::ParkHalf pk{park + threadIdx.x, &d.shell_scale[0][0], &d.shell_inv_scale[0][0]};
            if (d.asym_bounce && links) f32::bounce_fix(d, pk, links);
            const int32_t before = acc[0];
            f32::collide(d, cell, pk, acc);
            it_cell = acc[0] - before;
        }
        if constexpr (kStats) {
            const int32_t wmax = wave_max(it_cell);
            acc[8] += lane == 0 ? wmax : 0;
            acc[9] += lane == 0 ? 1 : 0;
        }
        // store the wave's rows
        __builtin_amdgcn_s_setprio(1);
        const uint64_t nP = (uint64_t)d.n * 4;
        const uint32_t *col = park + wave * kSegment;
        typedef uint32_t v4u __attribute__((ext_vector_type(4)));
        if (full && !kWide) {
            // lanes 16r..16r+15 store row i0 + r, four cells each: one uniform
            // base per group of 4 rows and one 32-bit lane offset (4 planes
            // of 4n bytes stay below 2^32 for n < 2^28)
            const int r = lane >> 4, c4 = (lane & 15) * 4;
            uint32_t voff = (uint32_t)r * (uint32_t)nP + (cell0 + (uint32_t)c4) * 4u;
            const uint32_t *lcol = col + r * kBlockThreads + c4;
            __asm__ volatile("" : "+v"(voff));
#pragma unroll
            for (int i0 = 0; i0 < kQ; i0 += 4) {
                if (i0 + r < kQ) {
                    const v4u v = *reinterpret_cast<const v4u *>(lcol + i0 * kBlockThreads);
                    __builtin_nontemporal_store(
                        v, reinterpret_cast<v4u __attribute__((address_space(1))) *>(dstb + (uint64_t)i0 * nP + voff));
                }
            }
        } else if (full) {
            // 2^28 cells or more: the same stores from a 64-bit lane address
            const int r = lane >> 4, c4 = (lane & 15) * 4;
            gbyte *lane_base = dstb + (uint64_t)r * nP + (uint64_t)(cell0 + (uint32_t)c4) * 4u;
            const uint32_t *lcol = col + r * kBlockThreads + c4;
#pragma unroll
            for (int i0 = 0; i0 < kQ; i0 += 4) {
                if (i0 + r < kQ) {
                    const v4u v = *reinterpret_cast<const v4u *>(lcol + i0 * kBlockThreads);
                    __builtin_nontemporal_store(
                        v, reinterpret_cast<v4u __attribute__((address_space(1))) *>(lane_base + (uint64_t)i0 * nP));
                }
            }
        } else if (in_grid) {
#pragma unroll
            for (int i = 0; i < kQ; ++i) gstore<uint32_t>(dstb + (uint64_t)i * nP, cell * 4u, col[i * kBlockThreads + lane]);
        }
    }
    if constexpr (kStats) {
        int64_t red[kStatWords];
#pragma unroll
        for (int k = 0; k < kStatWords; ++k) red[k] = (k == 1) ? wave_max(acc[k]) : wave_sum(acc[k]);
        if (lane == 0) {
            int64_t *p = stats + ((int64_t)blockIdx.x * kWavesPerBlock + wave) * kStatWords;
#pragma unroll
            for (int k = 0; k < kStatWords; ++k) p[k] = (k == 1) ? (red[k] > p[k] ? red[k] : p[k]) : p[k] + red[k];
        }
    }
}

// ---------------------------------------------------------------------------
// FP64 step.  Populations are stored paired, one 16-byte record (f_i, g_i)
// per cell and velocity, so the gather moves a cell's f_i and g_i with one
// 16-byte global -> LDS transfer per lane: 39 transfers of 1 KB per 64-cell
// segment, all in flight together with the 13 multiplier loads (the vector
// memory counter holds 63).  LDS row i of a wave holds the 64 records of
// velocity i; the relaxed records leave from registers as one 16-byte store
// per lane and velocity.  One wave per SIMD (the FP64 solve needs the
// register file).
namespace f64 {

typedef double v2d __attribute__((ext_vector_type(2)));
using lds_v2d = v2d __attribute__((address_space(3)));
constexpr uint32_t kRec = 16;  // bytes of one (f_i, g_i) record

// a uniform plane base forced into SGPRs where it is used: the access is
// then base + 32-bit lane offset, and no per-lane 64-bit address stays live
__device__ __forceinline__ gbyte *splane(gbyte *p)
{
    __asm__ volatile("" : "+s"(p));
    return p;
}
__device__ __forceinline__ gcbyte *splane(gcbyte *p)
{
    __asm__ volatile("" : "+s"(p));
    return p;
}

struct Park {
    lds_v2d *base;  // the lane's record in row 0 of its wave
    __device__ __forceinline__ v2d get(int i) const { return base[i * kSegment]; }
    // f_i alone (an 8-byte read)
    __device__ __forceinline__ double get_f(int i) const
    {
        return *reinterpret_cast<const double __attribute__((address_space(3))) *>(base + i * kSegment);
    }
};

// one 16-byte transfer per lane into LDS row `row` (the hardware places lane
// l's record at row + 16 l): a uniform base plus a 32-bit lane offset, or a
// per-lane address
__device__ __forceinline__ void dma16(gcbyte *base, uint32_t off, lds_v2d *row)
{
    __builtin_amdgcn_global_load_lds((const void __attribute__((address_space(1))) *)(splane(base) + off),
                                     (void __attribute__((address_space(3))) *)row, 16, 0, 0);
}
__device__ __forceinline__ void dma16_at(gcbyte *addr, lds_v2d *row)
{
    __builtin_amdgcn_global_load_lds((const void __attribute__((address_space(1))) *)addr,
                                     (void __attribute__((address_space(3))) *)row, 16, 0, 0);
}

// byte offsets of the pull sources x - c, c = -3..3, along each axis, within
// one velocity's plane of records
__device__ __forceinline__ void source_offsets(const SlotDesc &d, int x, int y, int z, uint32_t (&Xo)[7],
                                               uint32_t (&Yo)[7], uint32_t (&Zo)[7])
{
    const uint32_t nx = (uint32_t)d.nx, nxy = (uint32_t)d.nx * (uint32_t)d.ny;
#pragma unroll
    for (int c = -3; c <= 3; ++c) {
        Xo[c + 3] = (uint32_t)source_coord(x, c, d.nx, d.axis[0] == kAxisPeriodic, d.neumann_lo[0], d.neumann_hi[0]) * kRec;
        Yo[c + 3] = (uint32_t)source_coord(y, c, d.ny, d.axis[1] == kAxisPeriodic, d.neumann_lo[1], d.neumann_hi[1]) * nx * kRec;
        Zo[c + 3] = (uint32_t)source_coord(z, c, d.nz, d.axis[2] == kAxisPeriodic, d.neumann_lo[2], d.neumann_hi[2]) * nxy * kRec;
    }
}

// gather of one cell's 39 records (rows: row 0 of the wave).  copy: the
// cell's own records.  A blocked link (half-way bounce-back) reads the
// opposite velocity's record at the cell itself, in another plane: waves
// with such a link (linked, uniform) take per-lane addresses, the others a
// uniform plane base plus a 32-bit offset.
__device__ __forceinline__ void gather(const SlotDesc &d, gcbyte *srcb, int x, int y, int z, uint32_t cell,
                                       uint64_t links, bool copy, bool linked, lds_v2d *rows)
{
    const uint64_t nP = (uint64_t)d.n * kRec;
    const uint32_t cellR = cell * kRec;
    uint32_t Xo[7], Yo[7], Zo[7];
    source_offsets(d, x, y, z, Xo, Yo, Zo);
    dma16(srcb, cellR, rows);
    if (!linked) {
        // plane bases advance by one plane per transfer (two scalar adds
        // instead of a 64-bit multiply per plane)
        gcbyte *pl = srcb;
#pragma unroll
        for (int p = 0; p < kPairs; ++p) {
            const int a = 2 * p + 1, b = 2 * p + 2;
            const int cx = kPairVel[p][0], cy = kPairVel[p][1], cz = kPairVel[p][2];
            uint32_t oa = Xo[cx + 3] + (Yo[cy + 3] + Zo[cz + 3]);
            uint32_t ob = Xo[3 - cx] + (Yo[3 - cy] + Zo[3 - cz]);
            oa = copy ? cellR : oa;
            ob = copy ? cellR : ob;
            pl = splane(pl + nP);
            dma16(pl, oa, rows + a * kSegment);
            pl = splane(pl + nP);
            dma16(pl, ob, rows + b * kSegment);
        }
    } else {
        const uint64_t lk = copy ? 0ull : links;
#pragma unroll
        for (int p = 0; p < kPairs; ++p) {
            const int a = 2 * p + 1, b = 2 * p + 2;
            const int cx = kPairVel[p][0], cy = kPairVel[p][1], cz = kPairVel[p][2];
            uint32_t oa = Xo[cx + 3] + (Yo[cy + 3] + Zo[cz + 3]);
            uint32_t ob = Xo[3 - cx] + (Yo[3 - cy] + Zo[3 - cz]);
            oa = copy ? cellR : oa;
            ob = copy ? cellR : ob;
            gcbyte *pa = srcb + (uint64_t)a * nP, *pb = srcb + (uint64_t)b * nP;
            gcbyte *sa = ((lk >> a) & 1ull) ? pb + cellR : pa + oa;
            gcbyte *sb = ((lk >> b) & 1ull) ? pa + cellR : pb + ob;
            dma16_at(sa, rows + a * kSegment);
            dma16_at(sb, rows + b * kSegment);
        }
    }
}

// LDS records read per group in the sensor, the relaxation and the stores
// (three groups of 13 measured best against 8, 20 and 39)
constexpr int kChunk = 13;

// The multipliers go out with the gather, except in the variants with
// statistics: those hold more registers through the solve and load them
// after the moments (loading them early there costs scratch).
template <bool kStats>
constexpr bool kLamLoaded = !kStats;

// moments, Newton (kSolver 0; 1: the secant variant), sensor and relaxation
// of one fluid cell whose gathered values sit in LDS; the relaxed records go
// straight to the destination buffer dstb (one 16-byte store per velocity)
template <bool kStats, int kSolver>
__device__ __forceinline__ void collide(const SlotDesc &d, uint32_t cell, const Park &pk, double (&lam)[kM],
                                        gbyte *dstb, int32_t (&acc)[kStatWords])
{
    using C = double;
    C rho = C(-0.0), j0 = C(-0.0), j1 = C(-0.0), j2 = C(-0.0), e = C(-0.0);
    const v2d r0 = pk.get(0);
    C sg = r0.y;
    rho += r0.x;
#pragma unroll
    for (int p = 0; p < kPairs; ++p) {
        const v2d ra = pk.get(2 * p + 1), rb = pk.get(2 * p + 2);
        const C fa = ra.x, fb = rb.x;
        const C sp = fa + fb, ap = fa - fb;
        rho += sp;
        j0 += C(kPairVel[p][0]) * ap;
        j1 += C(kPairVel[p][1]) * ap;
        j2 += C(kPairVel[p][2]) * ap;
        e += C(pair_q(p)) * sp;
        sg += ra.y + rb.y;
        // read the rows a few pairs at a time, not all at once
        if ((p & 1) == 1) __asm__ volatile("" ::: "memory");
    }
    e += sg;
    // the gathered values are read again after the solve, not kept in registers
    __asm__ volatile("" ::: "memory");
    C u[3];
    u[0] = j0 / rho;
    u[1] = j1 / rho;
    u[2] = j2 / rho;
    const C T = (e - rho * (u[0] * u[0] + u[1] * u[1] + u[2] * u[2])) / (C(d.two_cv) * rho);

    gbyte *lamb = (gbyte *)d.lam;
    const uint64_t nL64 = (uint64_t)d.n * 8;
    const uint32_t cellL = cell * 8u;
    if constexpr (!kLamLoaded<kStats>) {
#pragma unroll
        for (int k = 0; k < kM; ++k) lam[k] = gload<C>(splane(lamb + (uint64_t)k * nL64), cellL);
    }

    C f0, fp[kPairs], fm[kPairs];
    int iters = 0;
    C G[kM];
    // a NaN lambda_0 marks a cell that had no equilibrium in the previous
    // step: its warm start normalises the other multipliers and it is not
    // restarted cold
    const bool marked = !(lam[0] == lam[0]);
    int status;
    if constexpr (kSolver == 0)
        status = solve_multipliers<C>(u, T, lam, f0, fp, fm, C(d.tol), d.maxit, d.maxit_cold,
                                      marked ? kStartMarked : kStartWarm, iters, G);
    else
        status = solve_multipliers_secant<C>(u, T, lam, f0, fp, fm, C(d.tol), d.maxit, d.maxit_cold,
                                             marked ? kStartMarked : kStartWarm, iters, G, d.qn_h, d.qn_T_ref);
    const bool failed = status == kFailed;
    if (!failed) {
#pragma unroll
        for (int k = 0; k < kM; ++k) {
            gstore<C>(splane(lamb), cellL, lam[k]);
            lamb += nL64;
        }
    } else {
        gstore<C>(splane(lamb), cellL, __builtin_nan(""));  // the failure mark; lambda_1..12 kept
    }

    // Knudsen sensor over f (Eq. eq:DeltaAvg) and relaxation branch (Eq. eq:alpha).
    // The records are read kChunk at a time, each group's LDS reads issued
    // together (a lone wave has no other wave to cover their latency).
    C eps = C(0);
#pragma unroll
    for (int i0 = 0; i0 < kQ; i0 += kChunk) {
        C hf[kChunk];
#pragma unroll
        for (int k = 0; k < kChunk; ++k)
            if (i0 + k < kQ) hf[k] = pk.get_f(i0 + k);
        __builtin_amdgcn_sched_barrier(0);
#pragma unroll
        for (int k = 0; k < kChunk; ++k) {
            const int i = i0 + k;
            if (i < kQ) {
                const C e_i = (i == 0) ? f0 : (((i - 1) & 1) == 0 ? fp[(i - 1) >> 1] : fm[(i - 1) >> 1]);
                const C feq = rho * e_i;
                eps += fabs(hf[k] - feq) * recip(feq);
            }
        }
    }
    eps *= C(1.0 / kQ);
    int br = 0;
    if (d.kn_relax) br = (eps < C(1e-2)) ? 0 : (eps < C(1e-1)) ? 1 : (eps < C(1)) ? 2 : 3;
    // a cell whose multipliers were not found is not collided (omega = 0
    // against the finite values the solver leaves): gathered values stored
    // unchanged, multipliers kept for the next warm start
    C omega = d.omega[0];
    omega = br == 1 ? d.omega[1] : omega;
    omega = br == 2 ? d.omega[2] : omega;
    omega = br == 3 ? d.omega[3] : omega;
    omega = failed ? C(0) : omega;
    const C dT = C(d.delta) * T;
    __asm__ volatile("" ::: "memory");
    const uint64_t nP = (uint64_t)d.n * kRec;
    const uint32_t cellR = cell * kRec;
    gbyte *pl = splane(dstb);
#pragma unroll
    for (int i0 = 0; i0 < kQ; i0 += kChunk) {
        v2d h[kChunk];
#pragma unroll
        for (int k = 0; k < kChunk; ++k)
            if (i0 + k < kQ) h[k] = pk.get(i0 + k);
        __builtin_amdgcn_sched_barrier(0);
#pragma unroll
        for (int k = 0; k < kChunk; ++k) {
            const int i = i0 + k;
            if (i < kQ) {
                const C e_i = (i == 0) ? f0 : (((i - 1) & 1) == 0 ? fp[(i - 1) >> 1] : fm[(i - 1) >> 1]);
                const C feq = rho * e_i;
                const C geq = dT * feq;
                const C hf = h[k].x, hg = h[k].y;
                __builtin_nontemporal_store(v2d{hf + omega * (feq - hf), hg + omega * (geq - hg)},
                                            reinterpret_cast<v2d __attribute__((address_space(1))) *>(pl + cellR));
                pl = splane(pl + nP);
            }
        }
    }

    if constexpr (kStats) {
        acc[0] += iters;
        acc[1] = iters > acc[1] ? iters : acc[1];
        acc[2] += failed;
        acc[3] += status == kConvergedCold || (failed && !marked);  // cold restarts tried
        acc[4] += !failed && br == 0;
        acc[5] += !failed && br == 1;
        acc[6] += !failed && br == 2;
        acc[7] += !failed && br == 3;
    }
}

}  // namespace f64

// kStats: per-wave statistics (iterations, failures, alpha branches) into
// stats; the variant without them keeps those registers free for the solve.
// kSolver: 0 Newton-Raphson, 1 the secant variant of the root finder.
template <bool kStats, int kSolver>
__global__ __launch_bounds__(kBlockThreads, 1) void step_kernel_f64(const SlotTable *__restrict__ tab, int j,
                                                                   int64_t *__restrict__ stats)
{
    __shared__ f64::v2d park[kWavesPerBlock * kQ * kSegment];
    int32_t acc[kStatWords] = {0, 0, 0, 0, 0, 0, 0, 0, 0, 0};
    const int total = tab->total_blocks;
    const int xcd = blockIdx.x & 7;
    const int per_xcd = gridDim.x >> 3;
    const int lo = (int)(((int64_t)total * xcd) >> 3);
    const int hi = (int)(((int64_t)total * (xcd + 1)) >> 3);
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int lane = threadIdx.x & 63;
    f64::lds_v2d *const rows0 = (f64::lds_v2d *)park + wave * (kQ * kSegment);
    for (int b = lo + (int)(blockIdx.x >> 3); b < hi; b += per_xcd) {
        // the 39 row addresses are cheap to form; keep the compiler from
        // hoisting them out of the loop into registers
        f64::lds_v2d *rows = rows0;
        __asm__ volatile("" : "+s"(rows));
        const f64::Park pk{rows + lane};
        const int s = find_slot(tab, b);
        const SlotDesc &d = tab->slot[s];
        if (j >= d.steps_todo) continue;
        const int64_t seg = (int64_t)(b - tab->block_start[s]) * kWavesPerBlock + wave;
        if (seg >= d.segments) continue;
        const int segx = (int)(seg % d.nsegx);
        const int row = (int)(seg / d.nsegx);
        const int y = row % d.ny;
        const int z = row / d.ny;
        const int x = segx * kSegment + lane;
        const uint32_t cell0 = (uint32_t)(segx * kSegment) + (uint32_t)d.nx * (uint32_t)row;
        const bool in_grid = x < d.nx;
        const uint32_t cell = cell0 + (uint32_t)lane;
        const int par = (d.parity0 + j) & 1;
        gcbyte *srcb = (gcbyte *)d.buf[par];
        gbyte *dstb = (gbyte *)d.buf[par ^ 1];
        bool fluid = in_grid && is_fluid_coord(d, x, y, z);
        uint64_t links = 0;
        if (fluid && d.has_links) links = d.links[cell];
        if (links >> 63) fluid = false;  // solid cells pass through unchanged
        const bool linked = __builtin_amdgcn_ballot_w64(fluid && links != 0) != 0;
        // the gather's 39 transfers and the 13 multiplier loads go out
        // together and are waited for once
        __builtin_amdgcn_s_setprio(1);
        if (in_grid) f64::gather(d, srcb, x, y, z, cell, links, !fluid, linked, rows);
        double lam[kM];
        if (f64::kLamLoaded<kStats> && fluid) {
            gcbyte *lamb = (gcbyte *)d.lam;
            const uint64_t nL64 = (uint64_t)d.n * 8;
#pragma unroll
            for (int k = 0; k < kM; ++k) {
                lam[k] = gload<double>(f64::splane(lamb), cell * 8u);
                lamb += nL64;
            }
        }
        __builtin_amdgcn_s_setprio(0);
        f32::wait_vmem();
        int32_t it_cell = 0;
        if (fluid) {
            const int32_t before = acc[0];
            f64::collide<kStats, kSolver>(d, cell, pk, lam, dstb, acc);
            it_cell = acc[0] - before;
        }
        if constexpr (kStats) {
            const int32_t wmax = wave_max(it_cell);
            acc[8] += lane == 0 ? wmax : 0;
            acc[9] += lane == 0 ? 1 : 0;
        }
        // cells that are not collided (solid, frozen or Neumann layers) pass
        // their gathered records through: one 16-byte store per lane and
        // velocity
        __builtin_amdgcn_s_setprio(1);
        if (in_grid && !fluid) {
            const uint64_t nP = (uint64_t)d.n * f64::kRec;
            const uint32_t cellR = cell * f64::kRec;
            gbyte *pl = f64::splane(dstb);
#pragma unroll
            for (int i0 = 0; i0 < kQ; i0 += f64::kChunk) {
                f64::v2d h[f64::kChunk];
#pragma unroll
                for (int k = 0; k < f64::kChunk; ++k)
                    if (i0 + k < kQ) h[k] = pk.get(i0 + k);
                __builtin_amdgcn_sched_barrier(0);
#pragma unroll
                for (int k = 0; k < f64::kChunk; ++k) {
                    if (i0 + k < kQ) {
                        __builtin_nontemporal_store(
                            h[k], reinterpret_cast<f64::v2d __attribute__((address_space(1))) *>(pl + cellR));
                        pl = f64::splane(pl + nP);
                    }
                }
            }
        }
    }
    if constexpr (kStats) {
        int64_t red[kStatWords];
#pragma unroll
        for (int k = 0; k < kStatWords; ++k) red[k] = (k == 1) ? wave_max(acc[k]) : wave_sum(acc[k]);
        if (lane == 0) {
            int64_t *p = stats + ((int64_t)blockIdx.x * kWavesPerBlock + wave) * kStatWords;
#pragma unroll
            for (int k = 0; k < kStatWords; ++k) p[k] = (k == 1) ? (red[k] > p[k] ? red[k] : p[k]) : p[k] + red[k];
        }
    }
}

// ---------------------------------------------------------------------------
// Initial state: the equilibrium of the given fields, cold-started in FP64.
// fields: rho[n], ux[n], uy[n], uz[n], T[n] (FP64).  Writes both buffers and
// the multipliers.  failed (int64) counts cells whose Newton did not converge.
template <class S>
__global__ __launch_bounds__(256) void init_kernel(SlotDesc d, const double *__restrict__ fields,
                                                   unsigned long long *failed)
{
    using C = typename StoreTraits<S>::C;
    const int64_t cell = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (cell >= d.n) return;
    const double rho = fields[cell];
    const double u[3] = {fields[d.n + cell], fields[2 * d.n + cell], fields[3 * d.n + cell]};
    const double T = fields[4 * d.n + cell];
    double lam[kM], f0, fp[kPairs], fm[kPairs];
    int iters = 0;
    const int maxit = d.maxit_cold;
    double G[kM];
    const int st = solve_multipliers<double>(u, T, lam, f0, fp, fm, d.tol, maxit, maxit, kStartCold, iters, G);
    if (st == kFailed) atomicAdd(failed, 1ull);
    const double dT = d.delta * T;
    S *b0 = static_cast<S *>(d.buf[0]);
    S *b1 = static_cast<S *>(d.buf[1]);
#pragma unroll
    for (int i = 0; i < kQ; ++i) {
        const double e = (i == 0) ? f0 : (((i - 1) & 1) == 0 ? fp[(i - 1) >> 1] : fm[(i - 1) >> 1]);
        const double feq = rho * e;
        const double geq = dT * feq;
        double vf = feq, vg = geq;
        if constexpr (StoreTraits<S>::kShift) {
            vf = (feq - (double)d.shift_w[i]) * (double)d.shell_inv_scale[0][shell(i)];
            vg = (geq - (double)d.shift_w[kQ + i]) * (double)d.shell_inv_scale[1][shell(i)];
        }
        const S sf = static_cast<S>(vf), sg = static_cast<S>(vg);
        b0[pidx<S>(i, cell, d.n)] = sf;
        b1[pidx<S>(i, cell, d.n)] = sf;
        b0[pidx<S>(kQ + i, cell, d.n)] = sg;
        b1[pidx<S>(kQ + i, cell, d.n)] = sg;
    }
    C *lb = static_cast<C *>(d.lam);
#pragma unroll
    for (int k = 0; k < kM; ++k) lb[(int64_t)k * d.n + cell] = static_cast<C>(lam[k]);
}

// Equilibrium of one state (used by the host for shift weights and the shear
// response).  out: feq[39] per unit density followed by lam[13].
__global__ void single_equilibrium_kernel(double rho, double ux, double uy, double uz, double T, double tol,
                                          int maxit, double *out, int *status)
{
    if (blockIdx.x != 0 || threadIdx.x != 0) return;
    const double u[3] = {ux, uy, uz};
    double lam[kM], f0, fp[kPairs], fm[kPairs];
    int iters = 0;
    double G[kM];
    *status = solve_multipliers<double>(u, T, lam, f0, fp, fm, tol, maxit, maxit, kStartCold, iters, G);
    for (int i = 0; i < kQ; ++i)
        out[i] = rho * ((i == 0) ? f0 : (((i - 1) & 1) == 0 ? fp[(i - 1) >> 1] : fm[(i - 1) >> 1]));
    for (int k = 0; k < kM; ++k) out[kQ + k] = lam[k];
    (void)rho;
}

// ---------------------------------------------------------------------------
// Moments of the stored state in FP64 (rho, ux, uy, uz, T per cell) and
// per-block partial totals over fluid cells (mass, momentum, energy).
template <class S>
__global__ __launch_bounds__(256) void moments_kernel(SlotDesc d, int parity, double *__restrict__ out,
                                                      double *__restrict__ partial)
{
    __shared__ double red[5][256];
    const int64_t cell = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    double t[5] = {0.0, 0.0, 0.0, 0.0, 0.0};
    if (cell < d.n) {
        const int x = (int)(cell % d.nx);
        const int y = (int)((cell / d.nx) % d.ny);
        const int z = (int)(cell / ((int64_t)d.nx * d.ny));
        const bool solid = d.has_links && (d.links[cell] >> 63);
        if (solid) {
            for (int k = 0; k < 5; ++k) out[(int64_t)k * d.n + cell] = __builtin_nan("");
        } else {
            // Neumann boundary cells report the interior cell they copy;
            // equilibrium-face cells (which take precedence) report themselves
            int c[3] = {x, y, z};
            const int n[3] = {d.nx, d.ny, d.nz};
            bool in_eq = false;
            for (int a = 0; a < 3; ++a) {
                in_eq = in_eq || (d.open_lo[a] && !d.neumann_lo[a] && c[a] < 3);
                in_eq = in_eq || (d.open_hi[a] && !d.neumann_hi[a] && c[a] >= n[a] - 3);
                if (d.neumann_lo[a] && c[a] < 3) c[a] = 3;
                if (d.neumann_hi[a] && c[a] >= n[a] - 3) c[a] = n[a] - 4;
            }
            const int64_t src =
                in_eq ? cell : (int64_t)c[0] + (int64_t)d.nx * ((int64_t)c[1] + (int64_t)d.ny * c[2]);
            const S *b = static_cast<const S *>(d.buf[parity]);
            double r = 0.0, jx = 0.0, jy = 0.0, jz = 0.0, e = 0.0;
            for (int i = 0; i < kQ; ++i) {
                double vf = (double)b[pidx<S>(i, src, d.n)];
                double vg = (double)b[pidx<S>(kQ + i, src, d.n)];
                if constexpr (StoreTraits<S>::kShift) {
                    vf = (double)d.shift_w[i] + vf * (double)d.shell_scale[0][shell(i)];
                    vg = (double)d.shift_w[kQ + i] + vg * (double)d.shell_scale[1][shell(i)];
                }
                const int cx = vel(i, 0), cy = vel(i, 1), cz = vel(i, 2);
                r += vf;
                jx += vf * cx;
                jy += vf * cy;
                jz += vf * cz;
                e += vf * (double)(cx * cx + cy * cy + cz * cz) + vg;
            }
            const double ux = jx / r, uy = jy / r, uz = jz / r;
            const double T = (e - r * (ux * ux + uy * uy + uz * uz)) / (d.two_cv * r);
            out[cell] = r;
            out[d.n + cell] = ux;
            out[2 * d.n + cell] = uy;
            out[3 * d.n + cell] = uz;
            out[4 * d.n + cell] = T;
            if (is_fluid_coord(d, x, y, z)) {
                t[0] = r;
                t[1] = jx;
                t[2] = jy;
                t[3] = jz;
                t[4] = 0.5 * e;
            }
        }
    }
    for (int k = 0; k < 5; ++k) red[k][threadIdx.x] = t[k];
    __syncthreads();
    for (int s = 128; s > 0; s >>= 1) {
        if ((int)threadIdx.x < s)
            for (int k = 0; k < 5; ++k) red[k][threadIdx.x] += red[k][threadIdx.x + s];
        __syncthreads();
    }
    if (threadIdx.x == 0)
        for (int k = 0; k < 5; ++k) partial[(int64_t)blockIdx.x * 5 + k] = red[k][0];
}

// Fixed-order sum of the per-block partials (one block).  Also flags
// non-finite fluid moments through the totals.
__global__ __launch_bounds__(256) void reduce_partials_kernel(const double *__restrict__ partial, int nblocks,
                                                              double *__restrict__ totals)
{
    __shared__ double red[5][256];
    double t[5] = {0.0, 0.0, 0.0, 0.0, 0.0};
    for (int b = threadIdx.x; b < nblocks; b += blockDim.x)
        for (int k = 0; k < 5; ++k) t[k] += partial[(int64_t)b * 5 + k];
    for (int k = 0; k < 5; ++k) red[k][threadIdx.x] = t[k];
    __syncthreads();
    for (int s = 128; s > 0; s >>= 1) {
        if ((int)threadIdx.x < s)
            for (int k = 0; k < 5; ++k) red[k][threadIdx.x] += red[k][threadIdx.x + s];
        __syncthreads();
    }
    if (threadIdx.x == 0)
        for (int k = 0; k < 5; ++k) totals[k] = red[k][0];
}

// Per-wave statistics partials -> totals (one block).
__global__ __launch_bounds__(256) void reduce_stats_kernel(const int64_t *__restrict__ partial, int nwaves,
                                                           int64_t *__restrict__ out)
{
    __shared__ int64_t red[kStatWords][256];
    int64_t t[kStatWords] = {0, 0, 0, 0, 0, 0, 0, 0, 0, 0};
    for (int w = threadIdx.x; w < nwaves; w += blockDim.x)
        for (int k = 0; k < kStatWords; ++k) {
            const int64_t v = partial[(int64_t)w * kStatWords + k];
            t[k] = (k == 1) ? (v > t[k] ? v : t[k]) : t[k] + v;
        }
    for (int k = 0; k < kStatWords; ++k) red[k][threadIdx.x] = t[k];
    __syncthreads();
    for (int s = 128; s > 0; s >>= 1) {
        if ((int)threadIdx.x < s)
            for (int k = 0; k < kStatWords; ++k) {
                const int64_t a = red[k][threadIdx.x], b = red[k][threadIdx.x + s];
                red[k][threadIdx.x] = (k == 1) ? (a > b ? a : b) : a + b;
            }
        __syncthreads();
    }
    if (threadIdx.x == 0)
        for (int k = 0; k < kStatWords; ++k) out[k] = red[k][0];
}

// Fill with zero (a kernel rather than a memset node, so that the sequence
// can be captured into a graph).
__global__ void zero_kernel(int64_t *p, int64_t count)
{
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < count; i += (int64_t)gridDim.x * blockDim.x)
        p[i] = 0;
}

// Decode population `pop` of buffer `parity` to FP64 (get_state), or encode
// FP64 into both buffers (set_state).
template <class S>
__global__ void decode_pop_kernel(SlotDesc d, int parity, int pop, double *__restrict__ out)
{
    const int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= d.n) return;
    const S *b = static_cast<const S *>(d.buf[parity]);
    double v = (double)b[pidx<S>(pop, c, d.n)];
    if constexpr (StoreTraits<S>::kShift)
        v = (double)d.shift_w[pop] + v * (double)d.shell_scale[pop >= kQ][shell(pop % kQ)];
    out[c] = v;
}

template <class S>
__global__ void encode_pop_kernel(SlotDesc d, int pop, const double *__restrict__ in)
{
    const int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= d.n) return;
    double v = in[c];
    if constexpr (StoreTraits<S>::kShift)
        v = (v - (double)d.shift_w[pop]) * (double)d.shell_inv_scale[pop >= kQ][shell(pop % kQ)];
    const S s = static_cast<S>(v);
    static_cast<S *>(d.buf[0])[pidx<S>(pop, c, d.n)] = s;
    static_cast<S *>(d.buf[1])[pidx<S>(pop, c, d.n)] = s;
}

template <class C>
__global__ void copy_lam_kernel(SlotDesc d, int k, int to_device, double *__restrict__ host_side)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= d.n) return;
    C *l = static_cast<C *>(d.lam) + (int64_t)k * d.n;
    if (to_device) l[i] = static_cast<C>(host_side[i]);
    else host_side[i] = (double)l[i];
}

}  // namespace lbm13

// ---------------------------------------------------------------------------
// Launch wrappers used by the C ABI layer (C++ linkage, internal).
#include "launch.h"

namespace lbm13 {

hipError_t launch_diag(int storage, const SlotTable *tab, int grid, int j, double *diag, hipStream_t st)
{
    switch (storage) {
    case kStoreF64: hipLaunchKernelGGL(diag_kernel<double>, dim3(grid), dim3(kBlockThreads), 0, st, tab, j, diag); break;
    case kStoreF32: hipLaunchKernelGGL(diag_kernel<float>, dim3(grid), dim3(kBlockThreads), 0, st, tab, j, diag); break;
    default: hipLaunchKernelGGL(diag_kernel<_Float16>, dim3(grid), dim3(kBlockThreads), 0, st, tab, j, diag); break;
    }
    return hipGetLastError();
}

hipError_t launch_step(int storage, const SlotTable *tab, int grid, int j, int64_t *stats, hipStream_t st,
                       int solver, bool wide)
{
    const dim3 g(grid), b(kBlockThreads);
    switch (storage) {
    case kStoreF64:
        if (solver == 1) {
            if (stats) hipLaunchKernelGGL((step_kernel_f64<true, 1>), g, b, 0, st, tab, j, stats);
            else hipLaunchKernelGGL((step_kernel_f64<false, 1>), g, b, 0, st, tab, j, stats);
        } else if (stats) {
            hipLaunchKernelGGL((step_kernel_f64<true, 0>), g, b, 0, st, tab, j, stats);
        } else {
            hipLaunchKernelGGL((step_kernel_f64<false, 0>), g, b, 0, st, tab, j, stats);
        }
        break;
    case kStoreF32:
        if (wide) hipLaunchKernelGGL((step_kernel_f32<true>), g, b, 0, st, tab, j, stats);
        else hipLaunchKernelGGL((step_kernel_f32<false>), g, b, 0, st, tab, j, stats);
        break;
    default:
        if (wide) {
            if (stats) hipLaunchKernelGGL((step_kernel_f16<true, true>), g, b, 0, st, tab, j, stats);
            else hipLaunchKernelGGL((step_kernel_f16<false, true>), g, b, 0, st, tab, j, stats);
        } else if (stats) {
            hipLaunchKernelGGL((step_kernel_f16<true, false>), g, b, 0, st, tab, j, stats);
        } else {
            hipLaunchKernelGGL((step_kernel_f16<false, false>), g, b, 0, st, tab, j, stats);
        }
        break;
    }
    return hipGetLastError();
}

const void *step_kernel_symbol(int storage)
{
    switch (storage) {
    case kStoreF64: return reinterpret_cast<const void *>(&step_kernel_f64<false, 0>);
    case kStoreF32: return reinterpret_cast<const void *>(&step_kernel_f32<false>);
    default: return reinterpret_cast<const void *>(&step_kernel_f16<false, false>);
    }
}

hipError_t launch_init(int storage, const SlotDesc &d, const double *fields, unsigned long long *failed,
                       hipStream_t st)
{
    const int grid = (int)((d.n + 255) / 256);
    switch (storage) {
    case kStoreF64: hipLaunchKernelGGL(init_kernel<double>, dim3(grid), dim3(256), 0, st, d, fields, failed); break;
    case kStoreF32: hipLaunchKernelGGL(init_kernel<float>, dim3(grid), dim3(256), 0, st, d, fields, failed); break;
    default: hipLaunchKernelGGL(init_kernel<_Float16>, dim3(grid), dim3(256), 0, st, d, fields, failed); break;
    }
    return hipGetLastError();
}

hipError_t launch_single_equilibrium(double rho, const double u[3], double T, double tol, int maxit, double *out,
                                     int *status, hipStream_t st)
{
    hipLaunchKernelGGL(single_equilibrium_kernel, dim3(1), dim3(64), 0, st, rho, u[0], u[1], u[2], T, tol, maxit,
                       out, status);
    return hipGetLastError();
}

hipError_t launch_moments(int storage, const SlotDesc &d, int parity, double *out, double *partial, double *totals,
                          hipStream_t st)
{
    const int grid = (int)((d.n + 255) / 256);
    switch (storage) {
    case kStoreF64:
        hipLaunchKernelGGL(moments_kernel<double>, dim3(grid), dim3(256), 0, st, d, parity, out, partial);
        break;
    case kStoreF32:
        hipLaunchKernelGGL(moments_kernel<float>, dim3(grid), dim3(256), 0, st, d, parity, out, partial);
        break;
    default:
        hipLaunchKernelGGL(moments_kernel<_Float16>, dim3(grid), dim3(256), 0, st, d, parity, out, partial);
        break;
    }
    hipLaunchKernelGGL(reduce_partials_kernel, dim3(1), dim3(256), 0, st, partial, grid, totals);
    return hipGetLastError();
}

int moments_partial_blocks(int64_t n) { return (int)((n + 255) / 256); }

// Scratch of lbm_moments_noalloc: the per-block partial totals of
// moments_kernel (one block per 256 cells) followed by the reduced totals,
// for grids of up to kNoallocMaxCells cells.  Each GPU the library runs on
// holds its own copy until the process ends.  In host code the name is a
// host-side stand-in, never a device address: host code uses only the
// address noalloc_scratch() looks up per device.
__device__ __align__(256) static double scratch[(kNoallocMaxCells / 256) * 5 + 8];

hipError_t noalloc_scratch(double **ptr)
{
    static std::mutex mu;
    static void *addr[kNoallocMaxDevices] = {};
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return e;
    if (dev < 0 || dev >= kNoallocMaxDevices) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lock(mu);
    if (!addr[dev]) {
        void *p = nullptr;
        e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return e;
        addr[dev] = p;
    }
    *ptr = static_cast<double *>(addr[dev]);
    return hipSuccess;
}

hipError_t launch_zero(int64_t *p, int64_t count, hipStream_t st)
{
    if (count <= 0) return hipSuccess;
    int grid = (int)((count + 255) / 256);
    grid = grid > 1024 ? 1024 : grid;
    hipLaunchKernelGGL(zero_kernel, dim3(grid), dim3(256), 0, st, p, count);
    return hipGetLastError();
}

hipError_t launch_reduce_stats(const int64_t *partial, int nwaves, int64_t *out, hipStream_t st)
{
    hipLaunchKernelGGL(reduce_stats_kernel, dim3(1), dim3(256), 0, st, partial, nwaves, out);
    return hipGetLastError();
}

hipError_t launch_decode_pop(int storage, const SlotDesc &d, int parity, int pop, double *out, hipStream_t st)
{
    const int grid = (int)((d.n + 255) / 256);
    switch (storage) {
    case kStoreF64: hipLaunchKernelGGL(decode_pop_kernel<double>, dim3(grid), dim3(256), 0, st, d, parity, pop, out); break;
    case kStoreF32: hipLaunchKernelGGL(decode_pop_kernel<float>, dim3(grid), dim3(256), 0, st, d, parity, pop, out); break;
    default: hipLaunchKernelGGL(decode_pop_kernel<_Float16>, dim3(grid), dim3(256), 0, st, d, parity, pop, out); break;
    }
    return hipGetLastError();
}

hipError_t launch_encode_pop(int storage, const SlotDesc &d, int pop, const double *in, hipStream_t st)
{
    const int grid = (int)((d.n + 255) / 256);
    switch (storage) {
    case kStoreF64: hipLaunchKernelGGL(encode_pop_kernel<double>, dim3(grid), dim3(256), 0, st, d, pop, in); break;
    case kStoreF32: hipLaunchKernelGGL(encode_pop_kernel<float>, dim3(grid), dim3(256), 0, st, d, pop, in); break;
    default: hipLaunchKernelGGL(encode_pop_kernel<_Float16>, dim3(grid), dim3(256), 0, st, d, pop, in); break;
    }
    return hipGetLastError();
}

hipError_t launch_copy_lam(int storage, const SlotDesc &d, int k, int to_device, double *host_side, hipStream_t st)
{
    const int grid = (int)((d.n + 255) / 256);
    if (storage == kStoreF64)
        hipLaunchKernelGGL(copy_lam_kernel<double>, dim3(grid), dim3(256), 0, st, d, k, to_device, host_side);
    else
        hipLaunchKernelGGL(copy_lam_kernel<float>, dim3(grid), dim3(256), 0, st, d, k, to_device, host_side);
    return hipGetLastError();
}

}  // namespace lbm13
