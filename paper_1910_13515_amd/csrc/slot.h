// Descriptor of one solve ("slot") as the device kernels see it, and the
// table of slots that one batched launch advances.  A single lbm_ctx is a
// table with one slot; the serving pool packs many slots into one table.
#pragma once

#include <cstdint>

namespace lbm13 {

constexpr int kSegment = 64;        // cells per wave: one row segment along x
constexpr int kWavesPerBlock = 4;   // 256 threads per block
constexpr int kBlockThreads = kSegment * kWavesPerBlock;
constexpr int kMaxSlots = 256;

enum StorageKind : int32_t { kStoreF64 = 0, kStoreF32 = 1, kStoreF16 = 2 };

// per-axis boundary handling
enum AxisKind : int32_t { kAxisPeriodic = 0, kAxisOpen = 1 };

struct SlotDesc {
    int32_t nx, ny, nz;
    int32_t nsegx;           // ceil(nx / 64)
    int64_t n;               // cells
    int64_t segments;        // nsegx * ny * nz
    int32_t blocks;          // ceil(segments / 4)
    int32_t axis[3];         // AxisKind per axis
    int32_t neumann_lo[3];   // 1 if the low face of the axis is Neumann
    int32_t neumann_hi[3];
    int32_t open_lo[3];      // 1 if the low face is non-periodic (equilibrium or Neumann)
    int32_t open_hi[3];
    int32_t has_links;       // obstacle present: links[] valid
    int32_t kn_relax;
    int32_t maxit, maxit_cold;
    int32_t parity0;         // buffer holding the state at step index 0 of a launch sequence
    int32_t steps_todo;      // launches with step index j < steps_todo advance this slot
    int32_t storage;         // StorageKind (informational; kernels are instantiated per storage)
    int32_t pad0;
    double tol;
    double omega[4];         // 1/(tau alpha) per branch of the relaxation table
    double delta;            // 2 C_v - D
    double two_cv;           // 2 C_v
    void *buf[2];            // ping-pong populations: [f 39][g 39][n] of the storage type
    void *lam;               // multipliers [13][n] in the arithmetic type
    const uint64_t *links;   // per cell: bit i = link i blocked (half-way bounce-back), bit 63 = solid
    int64_t *stats;          // per-wave partial statistics (8 x int64 per wave of the launch grid)
    // shifted storage: h_i = w_i + scale * stored_i (f: 0..38, g: 39..77);
    // FP16 only: scale is a power of two per velocity shell |xi|^2 in
    // {0, 1, 3, 4, 8, 9} (index 0..5), for f (row 0) and g (row 1)
    float shift_w[78];
    float shell_scale[2][6];
    float shell_inv_scale[2][6];
    // sums of the shift weights: mass, momentum (3), energy sum f|xi|^2 + g
    float ref_mass, ref_mom[3], ref_energy;
    // shifted storage with unequal shift weights of opposite velocities
    // (a stream-shifted solve with obstacles): a half-way bounce-back gathers
    // the stored deviation of the opposite velocity, which becomes the
    // population once bb_corr[i] = w_opp(i) - w_i is added (f: 0..38, g: 39..77)
    int32_t asym_bounce;
    float bb_corr[78];
    // root finder of the multipliers: 0 Newton-Raphson, 1 the secant variant
    // (FP64 only), whose model Jacobian is built on the rest equilibrium at
    // qn_T_ref; qn_h holds the inverse of that rest Jacobian in its cubic-
    // symmetric blocks: h00, h0s, hss, hst over (1, xi_a^2); h11, h1q, hqq
    // over (xi_a, xi_a |xi|^2) of one axis; hp for xi_a xi_b, a != b
    int32_t root_finder;
    int32_t pad1;
    double qn_T_ref;
    double qn_h[8];
};

struct SlotTable {
    int32_t nslots;
    int32_t total_blocks;
    int32_t block_start[kMaxSlots + 1];
    SlotDesc slot[1];  // nslots entries follow (allocated with room for nslots)
};

inline constexpr std::size_t slot_table_bytes(int nslots)
{
    return sizeof(SlotTable) + sizeof(SlotDesc) * (nslots > 1 ? nslots - 1 : 0);
}

constexpr int kStatWords = 10;  // iterations, max, failed, cold, hist[4], wave iterations, waves

// outcome of a cell's Newton solve
enum NewtonStatus : int { kConverged = 0, kConvergedCold = 1, kFailed = 2 };

}  // namespace lbm13
