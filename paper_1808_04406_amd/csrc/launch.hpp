// Host-side launch interface between the C ABI layer and the kernels.
#pragma once

#include "common.hpp"

namespace cmlb {

GridArgs make_grid(uint32_t nx, uint32_t ny, uint32_t nz, uint64_t plane);

// Step-kernel launch shape: one block per x-segment of each of `rows` rows,
// segments of up to max_block nodes (a whole row when it fits, so that the
// x-shifted reads of a row stay in one block and one L2), and the matching
// chunk count written to a.g.nchunks.
inline void step_shape(StepArgs& a, dim3& grid, dim3& block, uint32_t rows, uint32_t max_block) {
    uint32_t bs = ((a.g.nx + 63u) / 64u) * 64u;
    if (bs > max_block) bs = max_block;
    a.g.nchunks = (a.g.nx + bs - 1) / bs;
    block = dim3(bs);
    grid = dim3(a.g.nchunks * rows);
}

// Block index -> logical block: blocks are dealt round-robin to the 8 XCDs;
// give each XCD a contiguous run of logical blocks, so that the chunks of one
// row, which share cache lines at their edges, meet in one L2.
__device__ __forceinline__ uint32_t xcd_block(uint32_t nchunks) {
    const uint32_t b = blockIdx.x, nb = gridDim.x;
    if (nchunks == 1 || nb % 8 != 0) return b;
    return (b % 8) * (nb / 8) + b / 8;
}

// Each returns 0, or -1 for an unsupported lattice/storage/model combination.
int launch_step(int lattice, int storage, int model, const StepArgs& a, hipStream_t s);
int launch_step_tp(int lattice, int storage, const StepArgs& a, hipStream_t s);     // step_tp.hip
// 2D Hermite rules (step_d37.hip): D2Q37 with every storage and model, the
// other rules with FP64/FP32 storage and the central-moment kernel.
int launch_step_h2(int lattice, int storage, int model, const StepArgs& a, hipStream_t s);
// One step of `count` lattices (A.l[0..count)) in one launch.
int launch_step_batch(int lattice, int storage, int model, const BatchArgs& A, int count, hipStream_t s);
int launch_step_tp_batch(int lattice, int storage, const BatchArgs& A, int count, hipStream_t s);
int launch_step_d37_batch(int storage, int model, const BatchArgs& A, int count, hipStream_t s);
// Steps-per-launch modes of cmlb_set_step_fusion.
enum { kFuseAuto = 0, kFuseOne = 1, kFuseTwo = 2, kFuseTwoAcc = 3 };
// Two steps in one launch (step_tp2.hip, D3Q27 with FP32 storage); -1 if the
// configuration is not supported or, unless force is set, if two single-step
// launches are expected to be faster.
int launch_step2_tp(int lattice, int storage, const StepArgs& a, bool force, hipStream_t s);
// Two steps in one launch on D2Q37 with FP32 storage (step2_d37.hip): mode
// kFuseTwoAcc runs the row-accumulating kernel, kFuseTwo the bitwise one,
// kFuseAuto the bitwise one unless two single steps are expected faster.
int launch_step2_d37(int storage, int model, const StepArgs& a, int mode, hipStream_t s);
// Two steps in one launch where supported (either of the above); mode as
// above (kFuseTwoAcc is kFuseTwo on the tensor-product lattices).
int launch_step2(int lattice, int storage, int model, const StepArgs& a, int mode, hipStream_t s);
int launch_init(int lattice, int storage, const StepArgs& a, const FieldArgs& f, hipStream_t s);
int launch_moments(int lattice, int storage, const StepArgs& a, const FieldArgs& f, hipStream_t s);
int launch_encode_deviations(int lattice, int storage, void* stor, const float* dev, const StepArgs& a,
                             hipStream_t s);
int launch_codec(int lattice, int storage, bool decode, void* stor, double* full, const StepArgs& a,
                 const double* w, hipStream_t s);

// Reduction: uf holds 3 * plane doubles of scratch, p1 and p2 reduce_blocks(plane) * 8
// doubles each, out 8 doubles (drho, jx, jy, jz, sum h|e|^2, ke, enstrophy, nonfinite).
int reduce_blocks(uint64_t plane);
// Copy of `planes` (1 or 27) FP32 planes of `plane` values, one element of
// each plane per thread (kernels.hip).
int launch_stream_copy(int planes, const float* src, float* dst, uint64_t plane, hipStream_t s);
// Values per partial row of the FP64 reductions (8 sums, 3 maxima).
constexpr int kRedVals = 11;
int launch_reduce(int lattice, int storage, const StepArgs& a, double* uf, double* p1, double* p2, double* out,
                  hipStream_t s);

// Learned closure (kernels_closure.hip).
size_t closure_net_bytes();
int closure_partial_stride();
void launch_closure_pack(const float* params, const float* norm, int tie_even, void* net, hipStream_t s);
void launch_step_closure(const StepArgs& a, const void* net, hipStream_t s);
// mode 0: population objective against target [pair][27][nodes]; mode 1:
// momentum objective, target = the field D of launch_closure_momentum.
void launch_closure_train(const float* state, const float* target, int64_t n_pairs, const GridArgs& g, float rho0,
                          float omega2, const void* net, float* partials, int nblocks, float* grad, int mode,
                          hipStream_t s);
// D = (2/N)(j2 - jbar) [pair][3][nodes]: j2 the momentum of f1 [pair][27][nodes]
// after one more streaming, jbar that of target [pair][27][nodes].
void launch_closure_momentum(const float* f1, const float* target, int64_t n_pairs, const GridArgs& g, float* D,
                             hipStream_t s);
void launch_closure_adam(float* params, float* m1, float* m2, const float* grad, float lr, float beta1, float beta2,
                         float eps, int frozen, int step, hipStream_t s);

// Box filter of a D3Q27 state to FP32 deviations on the coarse grid.
int launch_box_filter(int storage, const StepArgs& a, int factor, float* dst, hipStream_t s);

}  // namespace cmlb
