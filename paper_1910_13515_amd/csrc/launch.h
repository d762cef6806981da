// Launch wrappers of the device kernels (internal C++ interface between the
// kernel translation unit and the C ABI layer).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

#include "slot.h"

namespace lbm13 {

// solver: 0 Newton-Raphson, 1 the secant variant (FP64 storage only);
// wide: a reduced-precision slot of kWideCells cells or more (row stores from
// 64-bit lane addresses)
constexpr int64_t kWideCells = (int64_t)1 << 28;
hipError_t launch_step(int storage, const SlotTable *tab, int grid, int j, int64_t *stats, hipStream_t st,
                       int solver = 0, bool wide = false);
// the kernel the pool's graph launches (Newton, slots below kWideCells cells)
const void *step_kernel_symbol(int storage);
hipError_t launch_diag(int storage, const SlotTable *tab, int grid, int j, double *diag, hipStream_t st);
hipError_t launch_init(int storage, const SlotDesc &d, const double *fields, unsigned long long *failed,
                       hipStream_t st);
hipError_t launch_single_equilibrium(double rho, const double u[3], double T, double tol, int maxit, double *out,
                                     int *status, hipStream_t st);
hipError_t launch_moments(int storage, const SlotDesc &d, int parity, double *out, double *partial, double *totals,
                          hipStream_t st);
int moments_partial_blocks(int64_t n);

// lbm_moments_noalloc: grids up to this many cells (the partials of one
// moments_kernel block per 256 cells fit the static scratch), on up to this
// many devices
constexpr int64_t kNoallocMaxCells = 524288;
constexpr int kNoallocMaxDevices = 64;
// device address of the static scratch on the current device: kNoallocMaxCells
// / 256 * 5 partials, then 5 totals
hipError_t noalloc_scratch(double **ptr);
hipError_t launch_zero(int64_t *p, int64_t count, hipStream_t st);
hipError_t launch_reduce_stats(const int64_t *partial, int nwaves, int64_t *out, hipStream_t st);
hipError_t launch_decode_pop(int storage, const SlotDesc &d, int parity, int pop, double *out, hipStream_t st);
hipError_t launch_encode_pop(int storage, const SlotDesc &d, int pop, const double *in, hipStream_t st);
hipError_t launch_copy_lam(int storage, const SlotDesc &d, int k, int to_device, double *host_side, hipStream_t st);

}  // namespace lbm13
