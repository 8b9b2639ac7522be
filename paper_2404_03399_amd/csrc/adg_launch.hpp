// Internal launch interface between the C ABI layer and the HIP kernels.
#pragma once

#include "adg_common.hpp"

namespace adg {

struct StepArgs {
  const DevProblem* probs;   // device descriptors
  const WorkItem* work;      // device work list, one item per workgroup
  int32_t n_work;
  double* ring;              // delay ring (fluxes), may be null when no PE faces
  int64_t* ctr;              // ctr[0] = steps completed by earlier batches, ctr[2] = non-finite flag
  double* atsum;             // fused kernel: AT sums of past levels, [kRecSlots][P][S] per problem
  RecWord* atk;              // fused kernel: clamped delays, [kRecSlots][P] words per problem (byte s = stage s)
  int32_t group[9];          // fused kernel: work-item ranges per degree and form (below)
  int32_t grid[8];           // fused kernel: workgroups per range
  int32_t single[8];         // fused kernel: the only problem of a range, or -1
  int32_t lane_elems;        // fused kernel: elements per lane (1, 2 or 4)
  int32_t steps;             // fused kernel: time steps per launch (1 or 2)
  double* qbuf;              // local DG: q = u_x of the current stage input (state layout)
  double* umid;              // fused kernel, two steps per launch: also write the state after
                             // the first step here (state layout), or null
  int32_t mode[8];           // fused kernel: fused_mode of each range (FUSED_SPLIT ranges mark
                             // their window items by tile index -(window group + 1))
  int32_t one_launch;        // fused kernel: one launch over every range (two elements per lane,
                             // every range FUSED_FULL), else one launch per range
};

// Work items of the fused kernel are sorted by descending np and, within a
// degree, by form: range g = 2 (5 - np) + v, [group[g], group[g + 1]), holds
// the items of degree np - 1 that take the a > 0 upwind form (v = 0: upwind
// advection with a positive speed, whose interior right-face flux is folded
// into the volume operator) or the general form of the context's equation
// (v = 1).  Each problem therefore runs the same kernel in a batch as in a
// context of its own.
constexpr int kFusedRanges = 8;

// Fused step kernel geometry: one wave64 per work item, R in {1, 2, 4}
// consecutive elements per lane, K in {1, 2} time steps per launch, halo of
// ceil(K S / R) lanes per side; owned elements per work item:
constexpr int kWave = 64;
constexpr int kWavesPerBlock = kBlock / kWave;
__host__ __device__ constexpr int fused_halo(int rk, int R, int K) { return (K * rk_stages(rk) + R - 1) / R; }
__host__ __device__ constexpr int fused_tile(int rk, int R, int K) { return R * (kWave - 2 * fused_halo(rk, R, K)); }

// Fused kernel modes, per work range: FUSED_FULL handles PE faces in every
// tile; FUSED_NOPE has every PE-face path compiled out (ranges without
// asynchronous problems); FUSED_SPLIT (the PE-face split) runs two kinds of
// wave in one launch: window waves (one element per lane, windows of
// fused_window elements centred on PE faces, each owning the 2 K S elements
// that the face's delayed flux reaches in K S stages, with every PE-face
// path) and tile waves with the PE-face paths compiled out that store only
// the elements outside those windows.
enum fused_mode { FUSED_FULL = 0, FUSED_NOPE = 1, FUSED_SPLIT = 2 };
__host__ __device__ constexpr int fused_window(int rk, int K) { return 4 * K * rk_stages(rk); }
__host__ __device__ constexpr int fused_windows_per_wave(int rk, int K) { return kWave / fused_window(rk, K); }

// Workgroups of the fused kernel for n_work items (kWavesPerBlock per group).
inline int fused_grid(int n_work) { return n_work < 1 ? 1 : (n_work + kWavesPerBlock - 1) / kWavesPerBlock; }

// a.steps full RK steps (1 or 2), all stages on chip: state uin -> uout
// (distinct buffers).  The first step's index is ctr[0] + step_offset.
hipError_t launch_fused_step(int rk, int phys, const StepArgs& a, const double* uin, double* uout,
                             int32_t step_offset, hipStream_t stream);
// Its per-integrator part (one translation unit per RK scheme).
template <int RK>
hipError_t launch_fused_rk(int phys, const StepArgs& a, const double* uin, double* uout, int32_t step_offset,
                           hipStream_t stream);

// One RK stage with the RK registers in HBM.  Stage 0 reads its input from U;
// the last stage writes U in place.  yin/yout alternate between two buffers.
hipError_t launch_stage(int rk, int phys, int stage, const StepArgs& a, const double* yin, double* yout,
                        double* U, double* A, int32_t step_offset, hipStream_t stream);

// Local DG, first pass of stage `stage`: q = u_x of the stage input yin into
// a.qbuf, with the u-hat face values (AT-combined at PE faces, level-n raw
// values written to the u-hat ring).
hipError_t launch_ldg_q(int rk, int stage, const StepArgs& a, const double* yin, int32_t step_offset,
                        hipStream_t stream);

// Reverse of RK stage `stage` of step n (absolute index) for all problems:
// lamu += mu, Q_i += a_{stage,i} mu, adjoint-ring deposits for delayed AT
// levels, cpart[workgroup] += dJ/da share.  Stage work list (kBlock per item).
hipError_t launch_adj_stage(int rk, int phys, int stage, const StepArgs& a, const double* Y, const double* lam,
                            double* lamu, double* Q, int64_t qstride, const double* ring, double* adjring,
                            double* cpart, int32_t n, hipStream_t stream);

// Fused adjoint geometry: one element per lane, halo of S lanes per side for
// a constant Jacobian (linear advection) and 2S - 1 when the Jacobian depends
// on the stage inputs (Burgers).  Work items are grouped by descending np
// like the fused step's list.
__host__ __device__ constexpr int adj_halo(int rk, bool nonlinear) {
  return nonlinear ? 2 * rk_stages(rk) - 1 : rk_stages(rk);
}
__host__ __device__ constexpr int adj_tile_elems(int rk, bool nonlinear) { return kWave - 2 * adj_halo(rk, nonlinear); }
struct AdjArgs {
  const DevProblem* probs;
  const WorkItem* work;
  int32_t group[5];
  int32_t grid[4];
  int32_t lane_elems;  // two-step reverse: elements per lane (1 or 2)
};

// Reverse of the whole RK step n (absolute index) for all problems in one
// launch per degree group: lamo = lambda^n from lam = lambda^{n+1} and the
// forward state u = u^n (stages recomputed on chip); adjoint-ring deposits for
// delayed AT levels; cpart[work item] += dJ/da share (advection).
hipError_t launch_adj_fused(int rk, int phys, const AdjArgs& a, const double* u, const double* lam, double* lamo,
                            const double* ring, double* adjring, double* cpart, int32_t n, hipStream_t stream);

// Reverse of steps n + 1 and n (absolute indices) for linear advection without
// the forward states (dJ/du0 only): lamo = lambda^n from lam = lambda^{n+2},
// R = a.lane_elems consecutive elements per lane, halo of 2S elements per
// side (work list of adj_tile_elems2(rk, R) elements per item).
hipError_t launch_adj_fused2(int rk, int phys, const AdjArgs& a, const double* lam, double* lamo, double* adjring,
                             int32_t n, hipStream_t stream);
__host__ __device__ constexpr int adj_halo2(int rk, int R) { return (2 * adj_halo(rk, false) + R - 1) / R; }
__host__ __device__ constexpr int adj_tile_elems2(int rk, int R) { return R * (kWave - 2 * adj_halo2(rk, R)); }

// Zero fill of `bytes` bytes at p (8-byte aligned, a multiple of 8).
hipError_t launch_zero(void* p, int64_t bytes, hipStream_t stream);

// ctr[0] := value (one lane).
hipError_t launch_set_counter(int64_t* ctr, int64_t value, hipStream_t stream);

// ctr[0] += n_steps (one lane), closing a batch of launches.
hipError_t launch_advance(int64_t* ctr, int64_t n_steps, hipStream_t stream);

// Per-workgroup partial error sums (work list with kBlock elements per item),
// then per-problem reduction in a fixed order.
hipError_t launch_stats(const StepArgs& a, const double* u, const double* ref, double* partials,
                        const int32_t* first_item, int32_t n_probs, double* out, hipStream_t stream);

// Per-group mean / variance of the per-problem statistics (3 doubles per
// problem: mean |u-ref|, max |u-ref|, integral) -> 4 doubles per group.
hipError_t launch_group_stats(const double* pstats, const int32_t* gstart, const int32_t* gmembers, int32_t n_groups,
                              double* out, hipStream_t stream);

// Sets ctr[2] = 1 if any owned state entry is NaN or Inf.
hipError_t launch_check_finite(const StepArgs& a, const double* u, hipStream_t stream);

}  // namespace adg
