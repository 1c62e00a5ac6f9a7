// Host-side launch interface between the C ABI layer and the kernels.
#pragma once

#include "common.hpp"

namespace cmlb {

GridArgs make_grid(uint32_t nx, uint32_t ny, uint32_t nz);

// Each returns 0, or -1 for an unsupported lattice/storage/model combination.
int launch_step(int lattice, int storage, int model, const StepArgs& a, hipStream_t s);
int launch_init(int lattice, int storage, const StepArgs& a, const FieldArgs& f, hipStream_t s);
int launch_moments(int lattice, int storage, const StepArgs& a, const FieldArgs& f, hipStream_t s);
int launch_codec(int lattice, int storage, bool decode, void* stor, double* full, const StepArgs& a,
                 const double* w, hipStream_t s);

// Reduction: uf holds 3 * plane doubles of scratch, p1 and p2 reduce_blocks(plane) * 8
// doubles each, out 8 doubles (drho, jx, jy, jz, sum h|e|^2, ke, enstrophy, nonfinite).
int reduce_blocks(uint64_t plane);
int launch_reduce(int lattice, int storage, const StepArgs& a, double* uf, double* p1, double* p2, double* out,
                  hipStream_t s);

}  // namespace cmlb
