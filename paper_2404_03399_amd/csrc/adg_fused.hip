// Fused step kernel: one wave64 per tile, all RK stages of one or two time
// steps on chip.  Compiled once per integrator (-DADG_RK=0 .. 4) so that the
// instantiations build in parallel.
#include "adg_device.hpp"

#ifndef ADG_RK
#error "compile once per integrator with -DADG_RK=0, 1, 2, 3 or 4"
#endif

namespace adg {

// One wave64 = one tile of T owned elements plus HL halo lanes per side,
// R consecutive elements per lane (16- or 32-byte accesses per plane), and
// K time steps per launch.  Each stage shrinks the valid range by one element
// per side, so after K*S stages the owned lanes are exact.  Halo elements are
// recomputed with the same instructions as by their owners, so a face shared
// by two waves gets a bitwise-identical flux on both sides.  Each lane
// computes the fluxes of the left faces of its elements; the right face of
// its last element is the next lane's first left face, received by a lane
// shift.  No workgroup barrier: the waves of a workgroup are independent.
//
// PE faces (Secs. 3-5): at step m the lane owning the element right of PE
// face b writes the level-m flux of every stage into the ring.  Before a
// launch at step n the records hold, per face and stage, the delay and AT sum
// of step n over its past levels and, for step n + 1, the delay and the part
// of its AT sum over the levels up to n - 1; a two-step launch adds the
// level-n term of step n + 1 itself (delay 1), from the raw flux the lane
// computed in the first step.  So the PE faces of a launch read two records and nothing
// else; no lane reads what another wave writes in the same launch.  The owner
// wave writes the records of steps n + K and n + K + 1 (levels up to
// n + K - 1) into slots that no wave of the launch reads (slot = step mod 4),
// one lane per (face, step, stage): the delays and the sums over the levels
// before n are formed at the start of the launch, where their ring loads
// overlap the state loads, and the levels of the launch are added at the end
// from the owner's raw fluxes kept on chip.  A delay of 0 selects the
// synchronous flux.  AT sums add the oldest level first in every path.
//
// MODE: TILE_FULL as above; TILE_NOPE compiles every PE-face path out (all
// faces synchronous: exact for problems without asynchronous faces, and away
// from PE faces for the others); TILE_MAIN is TILE_NOPE storing only the
// elements farther than K S from a PE face of an asynchronous problem;
// TILE_WINDOW runs the full PE logic on windows of 4 K S elements centred on
// PE faces (one element per lane), owning the 2 K S elements around each
// face that its delayed flux can reach in K S stages.  TILE_MAIN waves over
// every tile and TILE_WINDOW waves over every PE face compute each element
// with the same instructions as TILE_FULL, so the result is bitwise the same.
enum TileMode : int { TILE_FULL = 0, TILE_NOPE = 1, TILE_MAIN = 2, TILE_WINDOW = 3 };

template <int NP, int RK, int PHYS, int R, int K, int MODE>
__device__ __forceinline__ void wave_tile(const DevProblem& P, const WorkItem wi, const FusedPtrs& A, int64_t n,
                                          const double* __restrict__ uin, double* __restrict__ uout,
                                          double* __restrict__ umid, WaveSmemK<K, rk_stages(RK)>& sm, int wv,
                                          int lane) {
#pragma clang fp contract(off)  // explicit FMAs only: rounding independent of the launch shape
  constexpr int S = rk_stages(RK);
  constexpr bool PEF = MODE == TILE_FULL || MODE == TILE_WINDOW;  // PE-face paths compiled in
  constexpr bool WIN = MODE == TILE_WINDOW;
  static_assert(!WIN || R == 1, "windows take one element per lane");
  constexpr int HL = fused_halo(RK, R, K);
  constexpr int T = fused_tile(RK, R, K);
  const int N = (int)P.n_elem;
  // With N a multiple of R a lane's R elements never straddle the periodic
  // wrap, so its planes can move as 16-byte pieces.
  const bool grouped = R > 1 && (N % R) == 0;
  const int64_t ld = P.ld;
  const double* __restrict__ u = uin + P.u_off;

  int e[R];
  bool owned[R];
  if constexpr (WIN) {
    // window w of the wave covers elements f - 2KS .. f + 2KS - 1 of face
    // f = (tile * FW + w) pe_size and owns f - KS .. f + KS - 1; lanes past
    // the last window, and windows past the last face, own nothing
    constexpr int WW = fused_window(RK, K), FW = kWave / WW;
    const int w = lane / WW, l = lane - w * WW;
    const int fi = wi.tile * FW + (w < FW ? w : FW - 1);
    const int n_pe = (int)P.n_pe;
    const int x = (fi < n_pe ? fi : n_pe - 1) * (int)P.pe_size - 2 * K * S + l;
    e[0] = wrap_once(x, N);
    owned[0] = w < FW && fi < n_pe && l >= K * S && l < 3 * K * S;
  } else {
    const int e0 = wi.tile * T;
    const int teff = (N - e0) < T ? (N - e0) : T;
    const int xb = e0 - R * HL;  // element position of lane 0, element 0 (a multiple of R)
    const bool lane_owned = lane >= HL && lane < kWave - HL;
    const bool tiny = N < kWave * R;  // the wave's extent may wrap more than once
#pragma unroll
    for (int r = 0; r < R; ++r) {
      const int x = xb + R * lane + r;
      e[r] = tiny ? wrap_elem(x, N) : wrap_once(x, N);
      owned[r] = lane_owned && (x - e0) < teff;
    }
    if constexpr (MODE == TILE_MAIN) {
      if (P.async_faces) {  // the window waves own the elements near PE faces
        const uint32_t pes = P.pe_div.d;
#pragma unroll
        for (int r = 0; r < R; ++r) {
          const uint32_t d = (uint32_t)e[r] - fast_div((uint32_t)e[r], P.pe_div) * pes;
          owned[r] = owned[r] && d >= (uint32_t)(K * S) && d < pes - (uint32_t)(K * S);
        }
      }
    }
  }
  double u0[R][NP];
  // A grouped lane reads and writes its R elements of every plane as 16-byte
  // pieces through a buffer resource: the lane's byte offset sits in one
  // VGPR and each plane's offset in an SGPR, so no 64-bit address is formed
  // per plane (the problem's planes must span less than 2 GiB).
  const bool buffered = grouped && (int64_t)P.np * ld < (int64_t)1 << 28;
  const int voff = e[0] * 8;
  if (buffered) {
    const __amdgpu_buffer_rsrc_t rs = plane_rsrc(u);
#pragma unroll
    for (int j = 0; j < NP; ++j)
#pragma unroll
      for (int r = 0; r < R; r += 2) {
        const double2 v = __builtin_bit_cast(double2,
                                             __builtin_amdgcn_raw_buffer_load_b128(rs, voff + 8 * r, (int)(8 * j * ld), 0));
        u0[r][j] = v.x;
        u0[r + 1 < R ? r + 1 : r][j] = v.y;  // R >= 2 here
      }
  } else {
#pragma unroll
    for (int r = 0; r < R; ++r)
#pragma unroll
      for (int j = 0; j < NP; ++j) u0[r][j] = u[j * ld + e[r]];
  }

  // the PE face among this lane's left faces (if any) and its records
  bool pe[R];           // element r's left face is a PE face (at most one r)
  bool pe_right = false;  // the right face of element R-1 is a PE face
  bool any_pe = false;
  uint32_t b = 0;       // its boundary index
  RecWord kp[K];        // delays of step n + kk, byte s = stage s
  int depth = 1, slot_n = 0;
#pragma unroll
  for (int kk = 0; kk < K; ++kk) kp[kk] = 0;
#pragma unroll
  for (int r = 0; r < R; ++r) pe[r] = false;
  if (PEF && P.async_faces) {
    depth = P.depth;
    const uint32_t n32 = (uint32_t)n;  // step indices stay below 2^31
    slot_n = (int)(n32 - fast_div(n32, P.depth_div) * (uint32_t)depth);
    const uint32_t pes = P.pe_div.d;
#pragma unroll
    for (int r = 0; r < R; ++r) {
      const uint32_t br = fast_div((uint32_t)e[r], P.pe_div);
      pe[r] = (uint32_t)e[r] == br * pes;
      if (pe[r]) b = br;
      any_pe = any_pe || pe[r];
    }
    const uint32_t e1 = (e[R - 1] + 1 == N) ? 0u : (uint32_t)(e[R - 1] + 1);
    pe_right = e1 == fast_div(e1, P.pe_div) * pes;
  }
  // the records of this lane's PE face, into registers first: their loads,
  // the state loads and the record jobs' ring loads below are all issued
  // before the wave waits for any of them
  double rec[K][S];
  if (any_pe) {
#pragma unroll
    for (int kk = 0; kk < K; ++kk) {
      const int64_t rs = rec_slot(n + kk);
      kp[kk] = A.atk[P.atk_off + rs * P.n_pe + b];
      const double* __restrict__ src = A.atsum + P.at_off + (rs * P.n_pe + b) * S;
#pragma unroll
      for (int s = 0; s < S; ++s) rec[kk][s] = src[s];
    }
  }

  bool own_pe = false;  // this lane owns the element right of its PE face
#pragma unroll
  for (int r = 0; r < R; ++r) own_pe = own_pe || (pe[r] && owned[r]);
  // record jobs of the owner wave: g = face * 2S + t * S + s for the t-th
  // next record step n + K + t; one pass when they fit the wave
  constexpr int NJ = 2 * S;
  const uint64_t owners = __ballot(own_pe);
  const int n_jobs = NJ * __builtin_popcountll(owners);
  const bool one_pass = n_jobs <= kWave;
  const bool job_now = owners != 0 && one_pass;
  int job_kd = 0;
  AtLevels job_lv;
  if (job_now) {  // uniform: every lane takes part in the lane shuffle
    const int fi = lane / NJ, jj = lane - fi * NJ, t = jj / S, s = jj - t * S;
    const uint32_t bo = (uint32_t)__shfl((int)b, nth_set_lane(owners, fi));
    if (lane < n_jobs) {
      const int64_t m = n + K + t;
      job_kd = pe_delay(P, m, s, bo);
      at_old_levels_load(P, A.ring + P.ring_off + ((int64_t)bo * S + s) * depth, K + t, job_kd, slot_n, depth,
                         job_lv);
    }
  }
  if (any_pe) {
#pragma unroll
    for (int kk = 0; kk < K; ++kk)
#pragma unroll
      for (int s = 0; s < S; ++s) sm.at[kk][wv][s][lane] = rec[kk][s];
    if constexpr (K == 2) {
      if (n == 0) {  // no launch has written the records of step 1: its delays, no past levels
        kp[1] = 0;
#pragma unroll
        for (int s = 0; s < S; ++s) {
          kp[1] |= (RecWord)pe_delay(P, 1, s, b) << (8 * s);
          sm.at[1][wv][s][lane] = 0.0;
        }
      }
    }
  }
  if (job_now && lane < n_jobs) {
    sm.kdj[wv][lane] = job_kd;
    sm.part[wv][lane] = at_old_levels_sum(job_lv);
  }

  // write the owned elements of the tile
  bool all_owned = true;
#pragma unroll
  for (int r = 0; r < R; ++r) all_owned = all_owned && owned[r];
  double y[R][NP], ks[R][NP], k[NP];
  auto store = [&](double* __restrict__ dst) {
    double* __restrict__ uo = dst + P.u_off;
    if (buffered && all_owned) {
      const __amdgpu_buffer_rsrc_t rs = plane_rsrc(uo);
#pragma unroll
      for (int j = 0; j < NP; ++j)
#pragma unroll
        for (int r = 0; r < R; r += 2) {
          double2 v;
          v.x = y[r][j];
          v.y = y[r + 1 < R ? r + 1 : r][j];
          __builtin_amdgcn_raw_buffer_store_b128(__builtin_bit_cast(BufWord4, v), rs, voff + 8 * r, (int)(8 * j * ld), 0);
        }
    } else {
#pragma unroll
      for (int r = 0; r < R; ++r)
        if (owned[r])
#pragma unroll
          for (int j = 0; j < NP; ++j) uo[j * ld + e[r]] = y[r][j];
    }
  };
#pragma unroll
  for (int r = 0; r < R; ++r)
#pragma unroll
    for (int j = 0; j < NP; ++j) y[r][j] = u0[r][j];
  const double a = P.speed;
  const double dt = P.dt;

  // upwind, a > 0: the interior right-face flux a u_p is part of Kdu; only a
  // PE face on the right adds -Kr (F_right - a u_p).  rpe[r]: the right face
  // of element r is a PE face; wave_rpe[r] (uniform): it is on some lane.
  bool rpe[R], wave_rpe[R];
#pragma unroll
  for (int r = 0; r < R; ++r) {
    rpe[r] = r + 1 < R ? pe[r + 1] : pe_right;
    wave_rpe[r] = PHYS == PHYS_ADV_UPWIND_POS && __ballot(rpe[r]) != 0;
  }

  int slot_m = slot_n;
#pragma unroll
  for (int kk = 0; kk < K; ++kk) {
    if (kk > 0) {
      // after 2S stages of halo the owned lanes are exact after the first step too
      if (umid != nullptr) store(umid);
      slot_m = slot_m + 1 == depth ? 0 : slot_m + 1;
#pragma unroll
      for (int r = 0; r < R; ++r)
#pragma unroll
        for (int j = 0; j < NP; ++j) u0[r][j] = y[r][j];
    }
#pragma unroll
    for (int s = 0; s < S; ++s) {
      double F[R];
      const double um = lane_from_left(y[R - 1][NP - 1]);
      F[0] = Physics<PHYS>::fhat(um, y[0][0], a);
#pragma unroll
      for (int r = 1; r < R; ++r) F[r] = Physics<PHYS>::fhat(y[r - 1][NP - 1], y[r][0], a);
#pragma unroll
      for (int r = 0; r < R; ++r) {
        if (pe[r]) {
          const double raw = F[r];
          if (owned[r]) A.ring[P.ring_off + ((int64_t)b * S + s) * depth + slot_m] = raw;
          const int kd = (int)((kp[kk] >> (8 * s)) & 0xff);
          if (kd) {
            double at = sm.at[kk][wv][s][lane];
            if constexpr (K == 2) {  // delay 1 at step n+1: level n, this lane's raw flux of step n, completes the sum
              if (kk == 1 && kd == 1) at = fma(P.atc[1][0], sm.at[0][wv][s][lane], at);
            }
            F[r] = at;
          }
          sm.at[kk][wv][s][lane] = raw;  // level n + kk, for the records formed at the end
        }
      }
      if constexpr (PHYS == PHYS_ADV_UPWIND_POS) {
        double f_last = 0.0;
        if (wave_rpe[R - 1]) f_last = lane_from_right(F[0]);
#pragma unroll
        for (int r = 0; r < R; ++r) {
#pragma unroll
          for (int i = 0; i < NP; ++i) {
            double v = P.Kl[i] * F[r];
#pragma unroll
            for (int j = 0; j < NP; ++j) v = fma(P.Kdu[i * kMaxNp + j], y[r][j], v);
            k[i] = v;
          }
          if (wave_rpe[r]) {
            const double fr = r + 1 < R ? F[r + 1] : f_last;
            // 0 at an interior face; at a PE face the applied flux minus the
            // exact a u_p (for a synchronous one the rounding error of a u_p)
            const double corr = rpe[r] ? fma(-a, y[r][NP - 1], fr) : 0.0;
#pragma unroll
            for (int i = 0; i < NP; ++i) k[i] = fma(-P.Kr[i], corr, k[i]);
          }
          rk_update<NP, RK>(s, dt, u0[r], y[r], ks[r], k);
        }
      } else {
        const double f_last = lane_from_right(F[0]);
#pragma unroll
        for (int r = 0; r < R; ++r) {
          folded_rhs<NP, PHYS>(P, y[r], F[r], r + 1 < R ? F[r + 1] : f_last, k);
          rk_update<NP, RK>(s, dt, u0[r], y[r], ks[r], k);
        }
      }
    }
  }

  store(uout);

  // records of steps n + K and n + K + 1 over the levels up to n + K - 1:
  // the part before n and the delay from the start of the launch (formed here
  // when the jobs need more than one pass), the levels of the launch from the
  // owners' raw fluxes
  for (int g0 = 0; g0 < n_jobs; g0 += kWave) {
    const int g = g0 + lane;
    const int fi = g / NJ, jj = g - fi * NJ, t = jj / S, s = jj - t * S;
    const int src = nth_set_lane(owners, fi);
    const uint32_t bo = (uint32_t)__shfl((int)b, src);  // outside the branch: every lane active
    if (g < n_jobs) {
      const int64_t m = n + K + t;
      int kd;
      double acc;
      if (one_pass) {
        kd = sm.kdj[wv][lane];
        acc = sm.part[wv][lane];
      } else {
        kd = pe_delay(P, m, s, bo);
        acc = at_old_levels(P, A.ring + P.ring_off + ((int64_t)bo * S + s) * depth, K + t, kd, slot_n, depth);
      }
#pragma unroll
      for (int j = kMaxQ - 1; j >= 0; --j) {
        const int rel = K + t - kd - j;  // level n + rel of this launch
        if (kd > 0 && j < P.q && rel >= 0 && rel < K) acc = fma(P.atc[kd][j], sm.at[rel][wv][s][src], acc);
      }
      const int64_t rs = rec_slot(m);
      A.atsum[P.at_off + (rs * P.n_pe + bo) * S + s] = acc;
      reinterpret_cast<uint8_t*>(A.atk + P.atk_off + rs * P.n_pe + bo)[s] = (uint8_t)kd;
    }
  }
}

// MODE: fused_mode of the range.  Under FUSED_SPLIT the range interleaves
// window items (tile index -(g + 1) for window group g) with tile items in
// order of position along the mesh, so that the workgroups of one XCD hold
// the windows and the tiles of one stretch of elements (balanced work, and
// the windows' reads meet the tiles' in that XCD's L2); a wave takes one of
// the two paths as a whole, so the kernel's registers are those of the
// larger path, not of both.
template <int NP, int RK, int PHYS, int R, int K, int MODE>
__global__ __launch_bounds__(kBlock) void k_fused_step(const DevProblem* __restrict__ probs,
                                                       const WorkItem* __restrict__ work,
                                                       const int64_t* __restrict__ ctr, double* __restrict__ ring,
                                                       double* __restrict__ atsum, RecWord* __restrict__ atk,
                                                       int32_t w_begin, int32_t w_end,
                                                       const double* __restrict__ uin, double* __restrict__ uout,
                                                       double* __restrict__ umid, int32_t step_offset,
                                                       int32_t single_prob) {
  __shared__ WaveSmemK<K, rk_stages(RK)> sm;
  const int wv = __builtin_amdgcn_readfirstlane((int)(threadIdx.x / kWave));
  const int lane = (int)(threadIdx.x % kWave);
  const int w = w_begin + xcd_block((int)blockIdx.x, (int)gridDim.x) * kWavesPerBlock + wv;
  if (w >= w_end) return;  // whole wave
  const int64_t n = ctr[0] + step_offset;
  const FusedPtrs A{ring, atsum, atk};
  if constexpr (MODE == FUSED_SPLIT) {
    const WorkItem wi = work[w];
    if (wi.tile < 0)
      wave_tile<NP, RK, PHYS, 1, K, TILE_WINDOW>(probs[wi.prob], WorkItem{wi.prob, -wi.tile - 1}, A, n, uin, uout,
                                                 umid, sm, wv, lane);
    else
      wave_tile<NP, RK, PHYS, R, K, TILE_MAIN>(probs[wi.prob], wi, A, n, uin, uout, umid, sm, wv, lane);
  } else {
    // a range holding one problem lists its tiles in order: no work-list load
    const WorkItem wi = single_prob >= 0 ? WorkItem{single_prob, w - w_begin} : work[w];
    wave_tile<NP, RK, PHYS, R, K, MODE == FUSED_NOPE ? TILE_NOPE : TILE_FULL>(probs[wi.prob], wi, A, n, uin, uout,
                                                                             umid, sm, wv, lane);
  }
}

// One launch over every degree range (ADG_OPT_ONE_LAUNCH): wave w finds its
// range from the range table (ranges are contiguous in the work list, in the
// order of the per-range launches) and runs that range's tile with every
// PE-face path compiled in, as a FUSED_FULL range does.  A kernel's registers
// are those of its largest body, so every range runs at the occupancy of the
// degree-4 tile; one launch per range (the default) lets each degree keep its
// own.  The per-element arithmetic is that of the per-range kernels: the
// results are bitwise the same.
struct FusedRangeTable {
  int32_t group[kFusedRanges + 1];
};

template <int RK, int PHYS, int R, int K>
__global__ __launch_bounds__(kBlock) void k_fused_all(const DevProblem* __restrict__ probs,
                                                      const WorkItem* __restrict__ work,
                                                      const int64_t* __restrict__ ctr, double* __restrict__ ring,
                                                      double* __restrict__ atsum, RecWord* __restrict__ atk,
                                                      const FusedRangeTable rt, const double* __restrict__ uin,
                                                      double* __restrict__ uout, double* __restrict__ umid,
                                                      int32_t step_offset) {
  __shared__ WaveSmemK<K, rk_stages(RK)> sm;
  const int wv = __builtin_amdgcn_readfirstlane((int)(threadIdx.x / kWave));
  const int lane = (int)(threadIdx.x % kWave);
  const int w = xcd_block((int)blockIdx.x, (int)gridDim.x) * kWavesPerBlock + wv;
  if (w >= rt.group[kFusedRanges]) return;  // whole wave
  const int64_t n = ctr[0] + step_offset;
  const FusedPtrs A{ring, atsum, atk};
  const WorkItem wi = work[w];
  const DevProblem& P = probs[wi.prob];
  int gi = 0;  // uniform
#pragma unroll
  for (int g = 1; g < kFusedRanges; ++g) gi += w >= rt.group[g] ? 1 : 0;
  // even ranges hold the a > 0 upwind form, which exists for upwind advection only
  constexpr bool kPos = PHYS == PHYS_ADV_UPWIND;
  constexpr int PH0 = kPos ? PHYS_ADV_UPWIND_POS : PHYS;
  if (kPos && (gi & 1) == 0) {
    switch (gi) {
      case 0: wave_tile<5, RK, PH0, R, K, TILE_FULL>(P, wi, A, n, uin, uout, umid, sm, wv, lane); break;
      case 2: wave_tile<4, RK, PH0, R, K, TILE_FULL>(P, wi, A, n, uin, uout, umid, sm, wv, lane); break;
      case 4: wave_tile<3, RK, PH0, R, K, TILE_FULL>(P, wi, A, n, uin, uout, umid, sm, wv, lane); break;
      default: wave_tile<2, RK, PH0, R, K, TILE_FULL>(P, wi, A, n, uin, uout, umid, sm, wv, lane); break;
    }
  } else {
    switch (gi / 2) {
      case 0: wave_tile<5, RK, PHYS, R, K, TILE_FULL>(P, wi, A, n, uin, uout, umid, sm, wv, lane); break;
      case 1: wave_tile<4, RK, PHYS, R, K, TILE_FULL>(P, wi, A, n, uin, uout, umid, sm, wv, lane); break;
      case 2: wave_tile<3, RK, PHYS, R, K, TILE_FULL>(P, wi, A, n, uin, uout, umid, sm, wv, lane); break;
      default: wave_tile<2, RK, PHYS, R, K, TILE_FULL>(P, wi, A, n, uin, uout, umid, sm, wv, lane); break;
    }
  }
}

// Viscous Burgers in local DG form (Sec. 7): K in {1, 2} time steps per
// launch, R in {1, 2, 4} consecutive elements per lane, halo of K S elements
// per side.  Per stage: u-hat at a face is the trace of the element on its
// left (alternating flux); q = Kr u-hat_right - Kl u-hat_left - Kd u; the
// total flux at a face is G = LLF(u-, u+) - nu q+ with q+ from the element on
// its right; the element update is Kl G_left - Kr G_right + Kd (u^2/2 - nu q).
// u-hat_left comes from the element on the left (the left lane's last element
// by a lane shift) and u-hat_right is the element's own trace, so q needs no
// data from the right; G_right comes from the element on the right.  Each
// stage then depends on one element to either side, as the inviscid update
// does, and every element takes the same operations whatever R.  At a PE
// face the element right of it writes the raw level-m u-hat and G to their
// rings; the element holding the face as its left face takes the AT
// combinations of past levels of both, and the element holding it as its
// right face the u-hat combination.  The levels before n were written by
// earlier launches, so these sums are formed at the start of the launch; for
// the second step a delay of 1 also needs level n, which each lane adds from
// its own raw values (the left-face u-hat and G it computes, and for the
// right face its own trace, which is that face's u-hat).  A PE size of at
// least R gives a lane at most one PE face as some element's left face and
// at most one as some element's right face, so the per-lane LDS slots below
// hold each kind once.
template <int S, int K>
struct LdgSmem {
  double atu[K][kWavesPerBlock][S][kWave];   // left face: u-hat
  double atg[K][kWavesPerBlock][S][kWave];   // left face: G
  double atur[K][kWavesPerBlock][S][kWave];  // right face: u-hat
  uint8_t kl[K][kWavesPerBlock][S][kWave];   // delays of the left face
  uint8_t kr[K][kWavesPerBlock][S][kWave];   // delays of the right face
};

template <int NP, int RK, int K, int R>
__device__ __forceinline__ void wave_tile_ldg(const DevProblem& P, const WorkItem wi, double* __restrict__ ring,
                                              int64_t n, const double* __restrict__ uin, double* __restrict__ uout,
                                              LdgSmem<rk_stages(RK), K>& sm, int wv, int lane) {
#pragma clang fp contract(off)  // explicit FMAs only
  constexpr int S = rk_stages(RK);
  constexpr int HL = fused_halo(RK, R, K);
  constexpr int T = fused_tile(RK, R, K);
  const int N = (int)P.n_elem;
  const int e0 = wi.tile * T;
  const int teff = (N - e0) < T ? (N - e0) : T;
  const int xb = e0 - R * HL;  // element position of lane 0, element 0 (a multiple of R)
  const bool lane_owned = lane >= HL && lane < kWave - HL;
  const bool tiny = N < kWave * R;  // the wave's extent may wrap more than once
  int e[R];
  bool owned[R];
#pragma unroll
  for (int r = 0; r < R; ++r) {
    const int x = xb + R * lane + r;
    e[r] = tiny ? wrap_elem(x, N) : wrap_once(x, N);
    owned[r] = lane_owned && (x - e0) < teff;
  }
  // with N a multiple of R a lane's elements never straddle the periodic
  // wrap: its planes move as 16-byte pieces through a buffer resource
  const bool buffered = R > 1 && (N % R) == 0 && (int64_t)P.np * P.ld < (int64_t)1 << 28;
  const int voff = e[0] * 8;
  const int64_t ld = P.ld;
  const double* __restrict__ u = uin + P.u_off;
  double u0[R][NP];
  if (buffered) {
    const __amdgpu_buffer_rsrc_t rs = plane_rsrc(u);
#pragma unroll
    for (int j = 0; j < NP; ++j)
#pragma unroll
      for (int r = 0; r < R; r += 2) {
        const double2 v = __builtin_bit_cast(double2,
                                             __builtin_amdgcn_raw_buffer_load_b128(rs, voff + 8 * r, (int)(8 * j * ld), 0));
        u0[r][j] = v.x;
        u0[r + 1 < R ? r + 1 : r][j] = v.y;  // R >= 2 here
      }
  } else {
#pragma unroll
    for (int r = 0; r < R; ++r)
#pragma unroll
      for (int j = 0; j < NP; ++j) u0[r][j] = u[j * ld + e[r]];
  }

  bool pe[R];    // the left face of element r is a PE face
  bool per[R];   // the right face of element r is a PE face
  bool pe_any = false, per_any = false;
  uint32_t b = 0, br = 0;  // the lane's PE face of each kind
  int depth = 1, slot_n = 0;
#pragma unroll
  for (int r = 0; r < R; ++r) pe[r] = per[r] = false;
  if (P.async_faces) {
    depth = P.depth;
    const uint32_t n32 = (uint32_t)n;  // step indices stay below 2^31
    slot_n = (int)(n32 - fast_div(n32, P.depth_div) * (uint32_t)depth);
    const uint32_t pes = P.pe_div.d;
#pragma unroll
    for (int r = 0; r < R; ++r) {
      const uint32_t bl = fast_div((uint32_t)e[r], P.pe_div);
      pe[r] = (uint32_t)e[r] == bl * pes;
      if (pe[r]) b = bl;
      const uint32_t e1 = (e[r] + 1 == N) ? 0u : (uint32_t)(e[r] + 1);
      const uint32_t b1 = fast_div(e1, P.pe_div);
      per[r] = e1 == b1 * pes;
      if (per[r]) br = b1;
      pe_any = pe_any || pe[r];
      per_any = per_any || per[r];
    }
  }
  // The delays and the AT sums over the levels before n, one job lane per
  // (PE lane, step, stage, value): the left-face u-hat and G of each lane with
  // a PE left face, the right-face u-hat of each lane with a PE right face.
  // Each job draws its delay and sums its past levels; the target lane reads
  // both from LDS.
  constexpr int KS = K * S;
  const uint64_t m_l = __ballot(pe_any), m_r = __ballot(per_any);
  const int n_l = 2 * KS * __builtin_popcountll(m_l);
  const int n_jobs = n_l + KS * __builtin_popcountll(m_r);
  for (int g0 = 0; g0 < n_jobs; g0 += kWave) {  // uniform
    const int g = g0 + lane;
    const bool left = g < n_l;
    const int h = left ? g : g - n_l;
    const int per_face = left ? 2 * KS : KS;
    const int i = h / per_face, r = h - i * per_face;
    const int v = left ? r / KS : 2;  // 0: u-hat, 1: G (left face); 2: u-hat (right face)
    const int rr = r - (left ? v * KS : 0);
    const int kk = rr / S, s = rr - kk * S;
    const int tl = nth_set_lane(m_l, i), tr = nth_set_lane(m_r, i);
    const uint32_t fl = (uint32_t)__shfl((int)b, tl), fr = (uint32_t)__shfl((int)br, tr);  // every lane active
    if (g < n_jobs) {
      const int tgt = left ? tl : tr;
      const uint32_t face = left ? fl : fr;
      const int kd = pe_delay(P, n + kk, s, face);
      const double* __restrict__ rb = ring + (v == 1 ? P.ring_off : P.ring2_off) + ((int64_t)face * S + s) * depth;
      const double val = at_old_levels(P, rb, kk, kd, slot_n, depth);
      if (v == 0) {
        sm.atu[kk][wv][s][tgt] = val;
        sm.kl[kk][wv][s][tgt] = (uint8_t)kd;
      } else if (v == 1) {
        sm.atg[kk][wv][s][tgt] = val;
      } else {
        sm.atur[kk][wv][s][tgt] = val;
        sm.kr[kk][wv][s][tgt] = (uint8_t)kd;
      }
    }
  }

  double y[R][NP], ks[R][NP], k[NP], q[R][NP];
#pragma unroll
  for (int r = 0; r < R; ++r)
#pragma unroll
    for (int j = 0; j < NP; ++j) y[r][j] = u0[r][j];
  const double nu = P.nu;
  const double dt = P.dt;
  int slot_m = slot_n;
#pragma unroll
  for (int kk = 0; kk < K; ++kk) {
    if (kk > 0) {
      slot_m = slot_m + 1 == depth ? 0 : slot_m + 1;
#pragma unroll
      for (int r = 0; r < R; ++r)
#pragma unroll
        for (int j = 0; j < NP; ++j) u0[r][j] = y[r][j];
    }
#pragma unroll
    for (int s = 0; s < S; ++s) {
      const int64_t rs = ((int64_t)b * S + s) * depth + slot_m;
      double um[R], G[R];
      const double um0 = lane_from_left(y[R - 1][NP - 1]);
#pragma unroll
      for (int r = 0; r < R; ++r) {
        um[r] = r == 0 ? um0 : y[r - 1][NP - 1];  // u- at the left face, and its u-hat
        double hl = um[r];
        if (pe[r]) {
          if (owned[r]) ring[P.ring2_off + rs] = um[r];
          if constexpr (K == 2) {  // level n completes step n+1's u-hat sum when its delay is 1
            if (kk == 0 && sm.kl[1][wv][s][lane] == 1)
              sm.atu[1][wv][s][lane] = fma(P.atc[1][0], um[r], sm.atu[1][wv][s][lane]);
          }
          if (sm.kl[kk][wv][s][lane] != 0) hl = sm.atu[kk][wv][s][lane];
        }
        double hr = y[r][NP - 1];  // u-hat at the right face: this element's own trace
        if (per[r]) {
          if constexpr (K == 2) {
            if (kk == 0 && sm.kr[1][wv][s][lane] == 1)
              sm.atur[1][wv][s][lane] = fma(P.atc[1][0], hr, sm.atur[1][wv][s][lane]);
          }
          if (sm.kr[kk][wv][s][lane] != 0) hr = sm.atur[kk][wv][s][lane];
        }
#pragma unroll
        for (int i = 0; i < NP; ++i) {
          double v = fma(-P.Kl[i], hl, P.Kr[i] * hr);
#pragma unroll
          for (int j = 0; j < NP; ++j) v = fma(-P.Kd[i * kMaxNp + j], y[r][j], v);
          q[r][i] = v;
        }
      }
#pragma unroll
      for (int r = 0; r < R; ++r) {
        G[r] = fma(-nu, q[r][0], Physics<PHYS_BURGERS_LLF>::fhat(um[r], y[r][0], 1.0));
        if (pe[r]) {
          if (owned[r]) ring[P.ring_off + rs] = G[r];
          if constexpr (K == 2) {
            if (kk == 0 && sm.kl[1][wv][s][lane] == 1)
              sm.atg[1][wv][s][lane] = fma(P.atc[1][0], G[r], sm.atg[1][wv][s][lane]);
          }
          if (sm.kl[kk][wv][s][lane] != 0) G[r] = sm.atg[kk][wv][s][lane];
        }
      }
      const double Gr_last = lane_from_right(G[0]);
#pragma unroll
      for (int r = 0; r < R; ++r) {
        const double Gr = r + 1 < R ? G[r + 1] : Gr_last;
        double g[NP];
#pragma unroll
        for (int j = 0; j < NP; ++j) g[j] = fma(0.5 * y[r][j], y[r][j], -nu * q[r][j]);
#pragma unroll
        for (int i = 0; i < NP; ++i) {
          double v = fma(-P.Kr[i], Gr, P.Kl[i] * G[r]);
#pragma unroll
          for (int j = 0; j < NP; ++j) v = fma(P.Kd[i * kMaxNp + j], g[j], v);
          k[i] = v;
        }
        rk_update<NP, RK>(s, dt, u0[r], y[r], ks[r], k);
      }
    }
  }
  bool all_owned = true;
#pragma unroll
  for (int r = 0; r < R; ++r) all_owned = all_owned && owned[r];
  double* __restrict__ uo = uout + P.u_off;
  if (buffered && all_owned) {
    const __amdgpu_buffer_rsrc_t rs = plane_rsrc(uo);
#pragma unroll
    for (int j = 0; j < NP; ++j)
#pragma unroll
      for (int r = 0; r < R; r += 2) {
        double2 v;
        v.x = y[r][j];
        v.y = y[r + 1 < R ? r + 1 : r][j];
        __builtin_amdgcn_raw_buffer_store_b128(__builtin_bit_cast(BufWord4, v), rs, voff + 8 * r, (int)(8 * j * ld), 0);
      }
  } else {
#pragma unroll
    for (int r = 0; r < R; ++r)
      if (owned[r])
#pragma unroll
        for (int j = 0; j < NP; ++j) uo[j * ld + e[r]] = y[r][j];
  }
}

template <int NP, int RK, int K, int R>
__global__ __launch_bounds__(kBlock) void k_fused_ldg(const DevProblem* __restrict__ probs,
                                                      const WorkItem* __restrict__ work,
                                                      const int64_t* __restrict__ ctr, double* __restrict__ ring,
                                                      int32_t w_begin, int32_t w_end, const double* __restrict__ uin,
                                                      double* __restrict__ uout, int32_t step_offset,
                                                      int32_t single_prob) {
  __shared__ LdgSmem<rk_stages(RK), K> sm;
  const int wv = __builtin_amdgcn_readfirstlane((int)(threadIdx.x / kWave));
  const int lane = (int)(threadIdx.x % kWave);
  const int w = w_begin + xcd_block((int)blockIdx.x, (int)gridDim.x) * kWavesPerBlock + wv;
  if (w >= w_end) return;  // whole wave
  const int64_t n = ctr[0] + step_offset;
  const WorkItem wi = single_prob >= 0 ? WorkItem{single_prob, w - w_begin} : work[w];
  wave_tile_ldg<NP, RK, K, R>(probs[wi.prob], wi, ring, n, uin, uout, sm, wv, lane);
}

template <int NP, int RK, int R>
static void fused_ldg_go_r(const StepArgs& a, int gi, const double* uin, double* uout, int32_t off, hipStream_t st) {
  if (a.steps == 2)
    hipLaunchKernelGGL((k_fused_ldg<NP, RK, 2, R>), dim3(a.grid[gi]), dim3(kBlock), 0, st, a.probs, a.work, a.ctr,
                       a.ring, a.group[gi], a.group[gi + 1], uin, uout, off, a.single[gi]);
  else
    hipLaunchKernelGGL((k_fused_ldg<NP, RK, 1, R>), dim3(a.grid[gi]), dim3(kBlock), 0, st, a.probs, a.work, a.ctr,
                       a.ring, a.group[gi], a.group[gi + 1], uin, uout, off, a.single[gi]);
}

template <int NP, int RK>
static void fused_ldg_go(const StepArgs& a, int gi, const double* uin, double* uout, int32_t off, hipStream_t st) {
  switch (a.lane_elems) {
    case 2: fused_ldg_go_r<NP, RK, 2>(a, gi, uin, uout, off, st); break;
    case 4: fused_ldg_go_r<NP, RK, 4>(a, gi, uin, uout, off, st); break;
    default: fused_ldg_go_r<NP, RK, 1>(a, gi, uin, uout, off, st); break;
  }
}

template <int RK>
static void fused_ldg_np(const StepArgs& a, const double* uin, double* uout, int32_t off, hipStream_t st) {
  for (int gi = 0; gi < kFusedRanges; ++gi) {
    if (a.group[gi + 1] <= a.group[gi]) continue;
    switch (gi / 2) {  // np = 5, 4, 3, 2
      case 0: fused_ldg_go<5, RK>(a, gi, uin, uout, off, st); break;
      case 1: fused_ldg_go<4, RK>(a, gi, uin, uout, off, st); break;
      case 2: fused_ldg_go<3, RK>(a, gi, uin, uout, off, st); break;
      default: fused_ldg_go<2, RK>(a, gi, uin, uout, off, st); break;
    }
  }
}

template <int NP, int RK, int PHYS, int R, int MODE>
static void fused_go_m(const StepArgs& a, int gi, const double* uin, double* uout, int32_t off, hipStream_t st) {
  const dim3 g(a.grid[gi]), b(kBlock);
  if (a.steps == 2)
    hipLaunchKernelGGL((k_fused_step<NP, RK, PHYS, R, 2, MODE>), g, b, 0, st, a.probs, a.work, a.ctr, a.ring, a.atsum,
                       a.atk, a.group[gi], a.group[gi + 1], uin, uout, a.umid, off, a.single[gi]);
  else
    hipLaunchKernelGGL((k_fused_step<NP, RK, PHYS, R, 1, MODE>), g, b, 0, st, a.probs, a.work, a.ctr, a.ring, a.atsum,
                       a.atk, a.group[gi], a.group[gi + 1], uin, uout, nullptr, off, a.single[gi]);
}

template <int NP, int RK, int PHYS, int R>
static void fused_go_r(const StepArgs& a, int gi, const double* uin, double* uout, int32_t off, hipStream_t st) {
  switch (a.mode[gi]) {
    case FUSED_NOPE: fused_go_m<NP, RK, PHYS, R, FUSED_NOPE>(a, gi, uin, uout, off, st); break;
    case FUSED_SPLIT: fused_go_m<NP, RK, PHYS, R, FUSED_SPLIT>(a, gi, uin, uout, off, st); break;
    default: fused_go_m<NP, RK, PHYS, R, FUSED_FULL>(a, gi, uin, uout, off, st); break;
  }
}

template <int NP, int RK, int PHYS>
static void fused_go(const StepArgs& a, int gi, const double* uin, double* uout, int32_t off, hipStream_t st) {
  switch (a.lane_elems) {
    case 1: fused_go_r<NP, RK, PHYS, 1>(a, gi, uin, uout, off, st); break;
    case 4: fused_go_r<NP, RK, PHYS, 4>(a, gi, uin, uout, off, st); break;
    default: fused_go_r<NP, RK, PHYS, 2>(a, gi, uin, uout, off, st); break;
  }
}

template <int NP, int RK, int PHYS>
static void fused_form(const StepArgs& a, int gi, const double* uin, double* uout, int32_t off, hipStream_t st) {
  if constexpr (PHYS == PHYS_ADV_UPWIND) {
    if ((gi & 1) == 0) {  // the problems with a > 0
      fused_go<NP, RK, PHYS_ADV_UPWIND_POS>(a, gi, uin, uout, off, st);
      return;
    }
  }
  fused_go<NP, RK, PHYS>(a, gi, uin, uout, off, st);
}

template <int RK, int PHYS>
static void fused_np(const StepArgs& a, const double* uin, double* uout, int32_t off, hipStream_t st) {
  for (int gi = 0; gi < kFusedRanges; ++gi) {
    if (a.group[gi + 1] <= a.group[gi]) continue;
    switch (gi / 2) {  // np = 5, 4, 3, 2
      case 0: fused_form<5, RK, PHYS>(a, gi, uin, uout, off, st); break;
      case 1: fused_form<4, RK, PHYS>(a, gi, uin, uout, off, st); break;
      case 2: fused_form<3, RK, PHYS>(a, gi, uin, uout, off, st); break;
      default: fused_form<2, RK, PHYS>(a, gi, uin, uout, off, st); break;
    }
  }
}

template <int RK>
static void fused_phys(int phys, const StepArgs& a, const double* uin, double* uout, int32_t off, hipStream_t st) {
  switch (phys) {
    case PHYS_ADV_UPWIND: fused_np<RK, PHYS_ADV_UPWIND>(a, uin, uout, off, st); break;
    case PHYS_ADV_CENTRAL: fused_np<RK, PHYS_ADV_CENTRAL>(a, uin, uout, off, st); break;
    case PHYS_BURGERS_LDG: fused_ldg_np<RK>(a, uin, uout, off, st); break;  // one element per lane
    default: fused_np<RK, PHYS_BURGERS_LLF>(a, uin, uout, off, st); break;
  }
}

// ADG_OPT_ONE_LAUNCH: one launch over every range (two elements per lane).
template <int RK, int PHYS>
static void fused_all_go(const StepArgs& a, const double* uin, double* uout, int32_t off, hipStream_t st) {
  FusedRangeTable rt;
  for (int i = 0; i <= kFusedRanges; ++i) rt.group[i] = a.group[i];
  const dim3 g(fused_grid(a.group[kFusedRanges])), b(kBlock);
  if (a.steps == 2)
    hipLaunchKernelGGL((k_fused_all<RK, PHYS, 2, 2>), g, b, 0, st, a.probs, a.work, a.ctr, a.ring, a.atsum, a.atk, rt,
                       uin, uout, a.umid, off);
  else
    hipLaunchKernelGGL((k_fused_all<RK, PHYS, 2, 1>), g, b, 0, st, a.probs, a.work, a.ctr, a.ring, a.atsum, a.atk, rt,
                       uin, uout, nullptr, off);
}

template <int RK>
hipError_t launch_fused_rk(int phys, const StepArgs& a, const double* uin, double* uout, int32_t step_offset,
                           hipStream_t stream) {
  if (a.one_launch) {
    if (a.lane_elems != 2 || phys == PHYS_BURGERS_LDG) return hipErrorInvalidValue;
    switch (phys) {
      case PHYS_ADV_UPWIND: fused_all_go<RK, PHYS_ADV_UPWIND>(a, uin, uout, step_offset, stream); break;
      case PHYS_ADV_CENTRAL: fused_all_go<RK, PHYS_ADV_CENTRAL>(a, uin, uout, step_offset, stream); break;
      default: fused_all_go<RK, PHYS_BURGERS_LLF>(a, uin, uout, step_offset, stream); break;
    }
    return hipGetLastError();
  }
  fused_phys<RK>(phys, a, uin, uout, step_offset, stream);
  return hipGetLastError();
}

template hipError_t launch_fused_rk<ADG_RK>(int, const StepArgs&, const double*, double*, int32_t, hipStream_t);

}  // namespace adg
