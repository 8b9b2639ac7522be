// HIP kernels (gfx950, FP64) of the asynchronous DG stepper with AT fluxes.
//
// Element update of the reference-element weak form (paper Sec. 2):
//   du^e/dt = (2/dx) ( D f(u^e) + l_l F_e - l_r F_{e+1} ),  D = M^-1 S,
//   l_l = M^-1 phi(-1), l_r = M^-1 phi(1),
// with one numerical flux per face shared by both neighbours (conservation,
// Sec. 4.1).  At PE faces the flux is the AT combination of delayed levels
// (Sec. 5): F = sum_{j<q} c_j(k) F^{n-k-j}, read from a per-(boundary, stage)
// ring of past face fluxes.
//
// Layout: structure of arrays, u[off + j*ld + e]; lane = element, so every
// node-plane load/store of a wave64 is one contiguous 512-byte segment.
// Neighbour traces come through LDS (fused kernel) or through the cache
// from the neighbouring lanes' own loads (stage kernel).  No MFMA: the
// per-element operators are at most 5x5.
#include "adg_launch.hpp"

namespace adg {

// ---------------------------------------------------------------- physics ---
template <int PHYS>
struct Physics;

template <>
struct Physics<PHYS_ADV_UPWIND> {
  __device__ static double f(double u, double a) { return a * u; }
  __device__ static double fhat(double um, double up, double a) { return a >= 0.0 ? a * um : a * up; }
};

template <>
struct Physics<PHYS_ADV_UPWIND_POS> {
  __device__ static double f(double u, double a) { return a * u; }
  __device__ static double fhat(double um, double, double a) { return a * um; }
};

template <>
struct Physics<PHYS_ADV_CENTRAL> {
  __device__ static double f(double u, double a) { return a * u; }
  __device__ static double fhat(double um, double up, double a) { return a * (0.5 * um + 0.5 * up); }
};

template <>
struct Physics<PHYS_BURGERS_LLF> {
  __device__ static double f(double u, double) { return 0.5 * u * u; }
  __device__ static double fhat(double um, double up, double) {
    const double lam = fmax(fabs(um), fabs(up));
    return 0.5 * (0.5 * um * um + 0.5 * up * up) - 0.5 * lam * (up - um);
  }
};

// ------------------------------------------------------- PE-face AT flux ---
// Slot of level n - back (0 <= back < depth) given slot_n = n mod depth.
__device__ __forceinline__ int ring_slot(int slot_n, int back, int depth) {
  const int s = slot_n - back;
  return s < 0 ? s + depth : s;
}

// Clamped delay of boundary b at (step n, stage s).
__device__ __forceinline__ int pe_delay(const DevProblem& P, int64_t n, int s, uint32_t b) {
  const int key = P.per_stage ? s : 0;
  return clamp_delay(draw_delay(P.seed, n, key, (int64_t)b, P.thr, P.n_delays), n, P.q);
}

// sum_{j<q} c_j(k) F^{n-k-j} over the ring of (boundary, stage); k >= 1, so
// every level is a past one.
__device__ __forceinline__ double at_past_sum(const DevProblem& P, const double* __restrict__ r, int k,
                                              int slot_n) {
  double acc = 0.0;
  for (int j = 0; j < P.q; ++j) acc += P.atc[k][j] * r[ring_slot(slot_n, k + j, P.depth)];
  return acc;
}

// (2/dx) ( D f(y) + l_l fl - l_r fr ) with the operators held in registers.
template <int NP, int PHYS>
__device__ __forceinline__ void element_rhs(const double (&Dm)[NP][NP], const double (&ll)[NP],
                                            const double (&lr)[NP], double two_dx, double a,
                                            const double (&y)[NP], double fl, double fr, double (&k)[NP]) {
  double fy[NP];
#pragma unroll
  for (int j = 0; j < NP; ++j) fy[j] = Physics<PHYS>::f(y[j], a);
#pragma unroll
  for (int i = 0; i < NP; ++i) {
    double v = 0.0;
#pragma unroll
    for (int j = 0; j < NP; ++j) v += Dm[i][j] * fy[j];
    k[i] = two_dx * (v + ll[i] * fl - lr[i] * fr);
  }
}

template <int NP>
__device__ __forceinline__ void load_operators(const DevProblem& P, double (&Dm)[NP][NP], double (&ll)[NP],
                                               double (&lr)[NP]) {
#pragma unroll
  for (int i = 0; i < NP; ++i) {
#pragma unroll
    for (int j = 0; j < NP; ++j) Dm[i][j] = P.D[i * kMaxNp + j];
    ll[i] = P.lift_l[i];
    lr[i] = P.lift_r[i];
  }
}

// RK update after the stage-s operator value k (oracle's algebraic forms).
// u0: u^n; y: stage input (in) -> next stage input or u^{n+1} (out);
// ks: RK4 running sum k1 + 2k2 + 2k3, Heun k1 = dt L(u^n).
template <int NP, int RK>
__device__ __forceinline__ void rk_update(int s, double dt, const double (&u0)[NP], double (&y)[NP],
                                          double (&ks)[NP], const double (&k)[NP]) {
  if constexpr (RK == RK_RK4) {
    if (s == 0) {
#pragma unroll
      for (int j = 0; j < NP; ++j) { ks[j] = k[j]; y[j] = u0[j] + (0.5 * dt) * k[j]; }
    } else if (s == 1) {
#pragma unroll
      for (int j = 0; j < NP; ++j) { ks[j] = ks[j] + 2.0 * k[j]; y[j] = u0[j] + (0.5 * dt) * k[j]; }
    } else if (s == 2) {
#pragma unroll
      for (int j = 0; j < NP; ++j) { ks[j] = ks[j] + 2.0 * k[j]; y[j] = u0[j] + dt * k[j]; }
    } else {
#pragma unroll
      for (int j = 0; j < NP; ++j) y[j] = u0[j] + (dt / 6.0) * (ks[j] + k[j]);
    }
  } else if constexpr (RK == RK_SSP3) {
    if (s == 0) {
#pragma unroll
      for (int j = 0; j < NP; ++j) y[j] = u0[j] + dt * k[j];
    } else if (s == 1) {
#pragma unroll
      for (int j = 0; j < NP; ++j) y[j] = 0.75 * u0[j] + 0.25 * (y[j] + dt * k[j]);
    } else {
#pragma unroll
      for (int j = 0; j < NP; ++j) y[j] = u0[j] / 3.0 + (2.0 / 3.0) * (y[j] + dt * k[j]);
    }
  } else {  // Heun
    if (s == 0) {
#pragma unroll
      for (int j = 0; j < NP; ++j) { ks[j] = dt * k[j]; y[j] = u0[j] + ks[j]; }
    } else {
#pragma unroll
      for (int j = 0; j < NP; ++j) y[j] = u0[j] + 0.5 * (ks[j] + dt * k[j]);
    }
  }
}

// The absolute step index of a launch is ctr[0] + step_offset: launches of
// one batch (or one captured graph) carry offsets 0, 1, 2, ... and a single
// k_advance at the end of the batch adds the batch length to ctr[0].  No
// workgroup ever writes the counter while others read it.
__global__ void k_advance(int64_t* __restrict__ ctr, int64_t n_steps) {
  if (threadIdx.x == 0 && blockIdx.x == 0) ctr[0] = ctr[0] + n_steps;
}

// Element index of virtual position x on the periodic mesh of N elements.
__device__ __forceinline__ int wrap_elem(int x, int N) {
  while (x < 0) x += N;
  while (x >= N) x -= N;
  return x;
}

// Same for -N <= x < 2N (one correction at most).
__device__ __forceinline__ int wrap_once(int x, int N) {
  const int y = x < 0 ? x + N : x;
  return y >= N ? y - N : y;
}

// ------------------------------------------------------ fused step kernel ---
constexpr int kMaxStages = 4;

// Lane shifts across the whole wave64 (DPP wave_shr:1 / wave_shl:1): lane l
// receives lane l-1 (resp. l+1); the lane without a source receives 0
// (bound_ctrl).
__device__ __forceinline__ double lane_from_left(double v) {
  const int lo = __builtin_amdgcn_mov_dpp(__double2loint(v), 0x138, 0xf, 0xf, true);
  const int hi = __builtin_amdgcn_mov_dpp(__double2hiint(v), 0x138, 0xf, 0xf, true);
  return __hiloint2double(hi, lo);
}
__device__ __forceinline__ double lane_from_right(double v) {
  const int lo = __builtin_amdgcn_mov_dpp(__double2loint(v), 0x130, 0xf, 0xf, true);
  const int hi = __builtin_amdgcn_mov_dpp(__double2hiint(v), 0x130, 0xf, 0xf, true);
  return __hiloint2double(hi, lo);
}

// Per-lane PE-face record of the current step (written and read by the same
// lane only).  With R <= PE size a lane's R left faces hold at most one PE face.
struct WaveSmem {
  double at[kWavesPerBlock][kMaxStages][kWave];
};

template <int NP, int PHYS>
__device__ __forceinline__ void folded_rhs(const DevProblem& P, const double (&y)[NP], double fl, double fr,
                                           double (&k)[NP]) {
  double g[NP];
#pragma unroll
  for (int j = 0; j < NP; ++j) g[j] = PHYS == PHYS_BURGERS_LLF ? y[j] * y[j] : y[j];
#pragma unroll
  for (int i = 0; i < NP; ++i) {
    double v = P.Kl[i] * fl - P.Kr[i] * fr;
#pragma unroll
    for (int j = 0; j < NP; ++j) v += P.Kd[i * kMaxNp + j] * g[j];
    k[i] = v;
  }
}

struct FusedPtrs {
  double* __restrict__ ring;
  double* __restrict__ atsum;
  int32_t* __restrict__ atk;
};

// One wave64 = one tile of T owned elements plus HL halo lanes per side,
// R consecutive elements per lane (16- or 32-byte accesses per plane).  Each
// stage shrinks the valid range by one element per side, so after S stages
// the owned lanes are exact.  Halo elements are recomputed with the same
// instructions as by their owners, so a face shared by two waves gets a
// bitwise-identical flux on both sides.  Each lane computes the fluxes of
// the left faces of its elements; the right face of its last element is the
// next lane's first left face, received by a lane shift.  No workgroup
// barrier: the waves of a workgroup are independent.
//
// PE faces (Secs. 3-5): at step n the lane owning the element right of PE
// face b writes the level-n flux of every stage into the ring, and at the end
// of the step computes the delays of step n+1 and the AT sums
// sum_j c_j(k) F^{n+1-k-j} over past levels (all <= n when k >= 1) into record
// parity (n+1)&1.  Both neighbours of the face read parity n&1 at step n; a
// delay of 0 selects the synchronous level-n flux.
template <int NP, int RK, int PHYS, int R>
__device__ __forceinline__ void wave_tile(const DevProblem& P, const WorkItem wi, const FusedPtrs& A, int64_t n,
                                          const double* __restrict__ uin, double* __restrict__ uout, WaveSmem& sm,
                                          int wv, int lane) {
  constexpr int S = rk_stages(RK);
  constexpr int HL = halo_lanes(RK, R);
  constexpr int T = fused_tile(RK, R);
  const int N = (int)P.n_elem;
  const int e0 = wi.tile * T;
  const int teff = (N - e0) < T ? (N - e0) : T;
  const int xb = e0 - R * HL;  // element position of lane 0, element 0 (a multiple of R)
  // With N a multiple of R a lane's R elements never straddle the periodic
  // wrap, so one R*8-byte access per plane serves them all.
  const bool grouped = R > 1 && (N % R) == 0;
  const int64_t ld = P.ld;
  const double* __restrict__ u = uin + P.u_off;
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
  double u0[R][NP];
  if (grouped) {
    const double2* __restrict__ u2 = reinterpret_cast<const double2*>(__builtin_assume_aligned(u, 16));
#pragma unroll
    for (int j = 0; j < NP; ++j)
#pragma unroll
      for (int r = 0; r < R; r += 2) {
        const double2 v = u2[(j * ld + e[0] + r) >> 1];
        u0[r][j] = v.x;
        u0[r + 1 < R ? r + 1 : r][j] = R > 1 ? v.y : v.x;
      }
  } else {
#pragma unroll
    for (int r = 0; r < R; ++r)
#pragma unroll
      for (int j = 0; j < NP; ++j) u0[r][j] = u[j * ld + e[r]];
  }

  // the PE face among this lane's left faces (if any) and its step-n record
  const int par = (int)(n & 1);
  bool pe[R];           // element r's left face is a PE face (at most one r)
  bool pe_right = false;  // the right face of element R-1 is a PE face
  bool any_pe = false;
  uint32_t b = 0;       // its boundary index
  int32_t kp = 0;       // delays of step n, byte s = stage s
  int depth = 1, slot_n = 0;
#pragma unroll
  for (int r = 0; r < R; ++r) pe[r] = false;
  if (P.async_faces) {
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
    if (any_pe) {
      kp = A.atk[P.atk_off + (int64_t)par * P.n_pe + b];
      const double* __restrict__ src = A.atsum + P.at_off + ((int64_t)par * P.n_pe + b) * S;
#pragma unroll
      for (int s = 0; s < S; ++s) sm.at[wv][s][lane] = src[s];
    }
  }

  double y[R][NP], ks[R][NP], k[NP];
#pragma unroll
  for (int r = 0; r < R; ++r)
#pragma unroll
    for (int j = 0; j < NP; ++j) y[r][j] = u0[r][j];
  const double a = P.speed;
  const double dt = P.dt;

  // upwind, a > 0: the interior right-face flux a u_p is part of Kdu; only a
  // delayed PE face on the right adds -Kr (F_right - a u_p)
  const bool wave_pe_right = PHYS == PHYS_ADV_UPWIND_POS && __ballot(pe_right) != 0;

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
        if (owned[r]) A.ring[P.ring_off + ((int64_t)b * S + s) * depth + slot_n] = F[r];
        if ((kp >> (8 * s)) & 0xff) F[r] = sm.at[wv][s][lane];
      }
    }
    if constexpr (PHYS == PHYS_ADV_UPWIND_POS) {
      double f_last = 0.0;
      if (wave_pe_right) f_last = lane_from_right(F[0]);
#pragma unroll
      for (int r = 0; r < R; ++r) {
#pragma unroll
        for (int i = 0; i < NP; ++i) {
          double v = P.Kl[i] * F[r];
#pragma unroll
          for (int j = 0; j < NP; ++j) v += P.Kdu[i * kMaxNp + j] * y[r][j];
          k[i] = v;
        }
        const bool right_pe = r + 1 < R ? pe[r + 1] : pe_right;
        if (right_pe) {
          const double fr = r + 1 < R ? F[r + 1] : f_last;
          const double corr = fr - a * y[r][NP - 1];  // exactly 0 unless the face is delayed
#pragma unroll
          for (int i = 0; i < NP; ++i) k[i] -= P.Kr[i] * corr;
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

  double* __restrict__ uo = uout + P.u_off;
  bool all_owned = true;
#pragma unroll
  for (int r = 0; r < R; ++r) all_owned = all_owned && owned[r];
  if (grouped && all_owned) {
    double2* __restrict__ uo2 = reinterpret_cast<double2*>(__builtin_assume_aligned(uo, 16));
#pragma unroll
    for (int j = 0; j < NP; ++j)
#pragma unroll
      for (int r = 0; r < R; r += 2) {
        double2 v;
        v.x = y[r][j];
        v.y = y[r + 1 < R ? r + 1 : r][j];
        uo2[(j * ld + e[0] + r) >> 1] = v;
      }
  } else {
#pragma unroll
    for (int r = 0; r < R; ++r)
      if (owned[r])
#pragma unroll
        for (int j = 0; j < NP; ++j) uo[j * ld + e[r]] = y[r][j];
  }

  // owners of PE faces: records of step n+1, one lane per (face, stage).
  // For each owned PE face of this wave (uniform loop over the owner mask),
  // lanes 0..S-1 draw the stage's delay and sum the AT weights over the
  // past levels, independently of each other.
  bool own = false;
#pragma unroll
  for (int r = 0; r < R; ++r) own = own || (pe[r] && owned[r]);
  uint64_t owners = __ballot(own);
  while (owners) {
    const int src = __builtin_ctzll(owners);
    owners &= owners - 1;
    const uint32_t bo = (uint32_t)__builtin_amdgcn_readlane((int)b, src);
    if (lane < S) {
      const int s = lane;
      const int64_t n1 = n + 1;
      const uint64_t pre = delay_prefix(P.seed, n1, P.per_stage ? s : 0);
      const int kd = clamp_delay(delay_from_prefix(pre, bo, P.thr, P.n_delays), n1, P.q);
      const double* __restrict__ rb = A.ring + P.ring_off + ((int64_t)bo * S + s) * depth;
      double acc = 0.0;
      for (int j = 0; kd > 0 && j < P.q; ++j)  // level n1 - kd - j = n - (kd + j - 1)
        acc += P.atc[kd][j] * rb[ring_slot(slot_n, kd + j - 1, depth)];
      A.atsum[P.at_off + ((int64_t)(par ^ 1) * P.n_pe + bo) * S + s] = acc;
      reinterpret_cast<uint8_t*>(A.atk + P.atk_off + (int64_t)(par ^ 1) * P.n_pe + bo)[s] = (uint8_t)kd;
    }
  }
}

template <int NP, int RK, int PHYS, int R>
__global__ __launch_bounds__(kBlock) void k_fused_step(const DevProblem* __restrict__ probs,
                                                       const WorkItem* __restrict__ work,
                                                       const int64_t* __restrict__ ctr, double* __restrict__ ring,
                                                       double* __restrict__ atsum, int32_t* __restrict__ atk,
                                                       int32_t w_begin, int32_t w_end, const double* __restrict__ uin,
                                                       double* __restrict__ uout, int32_t step_offset) {
  __shared__ WaveSmem sm;
  const int wv = __builtin_amdgcn_readfirstlane((int)(threadIdx.x / kWave));
  const int lane = (int)(threadIdx.x % kWave);
  const int w = w_begin + (int)blockIdx.x * kWavesPerBlock + wv;
  if (w >= w_end) return;  // whole wave
  const int64_t n = ctr[0] + step_offset;
  const WorkItem wi = work[w];
  const FusedPtrs A{ring, atsum, atk};
  wave_tile<NP, RK, PHYS, R>(probs[wi.prob], wi, A, n, uin, uout, sm, wv, lane);
}

// ------------------------------------------------------ per-stage kernel ---
// One lane per element; the neighbours' traces are read from global memory
// (the same cache lines the neighbouring lanes load).  RK registers in HBM:
//   RK4:     A = k1 + 2k2 + 2k3 (accumulated), Y = next stage input
//   SSP-RK3: Y = u1, then u2
//   Heun:    A = k1 = dt L(u), Y = u + k1
template <int NP, int RK, int PHYS, int SI>
__device__ __forceinline__ void stage_elem(const DevProblem& P, int tile, const double* __restrict__ yin,
                                           double* __restrict__ yout, double* __restrict__ U,
                                           double* __restrict__ A, double* __restrict__ ring, int64_t n) {
  constexpr int S = rk_stages(RK);
  const int N = (int)P.n_elem;
  const int e = tile * kBlock + (int)threadIdx.x;
  if (e >= N) return;
  const int64_t ld = P.ld;
  const int64_t off = P.u_off;
  const double a = P.speed;
  const double dt = P.dt;
  const int em = e == 0 ? N - 1 : e - 1;
  const int e1 = e + 1 == N ? 0 : e + 1;
  double Dm[NP][NP], ll[NP], lr[NP];
  load_operators<NP>(P, Dm, ll, lr);
  double y[NP], k[NP];
#pragma unroll
  for (int j = 0; j < NP; ++j) y[j] = yin[off + j * ld + e];
  const double um = yin[off + (NP - 1) * ld + em];
  const double upr = yin[off + e1];
  double fl = Physics<PHYS>::fhat(um, y[0], a);
  double fr = Physics<PHYS>::fhat(y[NP - 1], upr, a);
  if (P.async_faces) {
    const uint32_t pes = P.pe_div.d;
    const int slot_n = (int)(n % (int64_t)P.depth);
    const uint32_t bl = fast_div((uint32_t)e, P.pe_div);
    if ((uint32_t)e == bl * pes) {
      const double* r = ring + P.ring_off + ((int64_t)bl * S + SI) * P.depth;
      const int kd = pe_delay(P, n, SI, bl);
      ring[P.ring_off + ((int64_t)bl * S + SI) * P.depth + slot_n] = fl;
      if (kd > 0) fl = at_past_sum(P, r, kd, slot_n);
    }
    const uint32_t br = fast_div((uint32_t)e1, P.pe_div);
    if ((uint32_t)e1 == br * pes) {
      const double* r = ring + P.ring_off + ((int64_t)br * S + SI) * P.depth;
      const int kd = pe_delay(P, n, SI, br);
      if (kd > 0) fr = at_past_sum(P, r, kd, slot_n);
    }
  }
  element_rhs<NP, PHYS>(Dm, ll, lr, P.two_over_dx, a, y, fl, fr, k);

  double* __restrict__ Uo = U + off;
  double* __restrict__ Ao = A + off;
  double* __restrict__ Yo = yout + off;
  if constexpr (RK == RK_RK4) {
#pragma unroll
    for (int j = 0; j < NP; ++j) {
      const int64_t i = j * ld + e;
      if constexpr (SI == 0) {
        Ao[i] = k[j];
        Yo[i] = y[j] + (0.5 * dt) * k[j];  // stage-0 input is u
      } else if constexpr (SI == 1) {
        Ao[i] = Ao[i] + 2.0 * k[j];
        Yo[i] = Uo[i] + (0.5 * dt) * k[j];
      } else if constexpr (SI == 2) {
        Ao[i] = Ao[i] + 2.0 * k[j];
        Yo[i] = Uo[i] + dt * k[j];
      } else {
        Uo[i] = Uo[i] + (dt / 6.0) * (Ao[i] + k[j]);
      }
    }
  } else if constexpr (RK == RK_SSP3) {
#pragma unroll
    for (int j = 0; j < NP; ++j) {
      const int64_t i = j * ld + e;
      if constexpr (SI == 0) {
        Yo[i] = y[j] + dt * k[j];
      } else if constexpr (SI == 1) {
        Yo[i] = 0.75 * Uo[i] + 0.25 * (y[j] + dt * k[j]);
      } else {
        Uo[i] = Uo[i] / 3.0 + (2.0 / 3.0) * (y[j] + dt * k[j]);
      }
    }
  } else {
#pragma unroll
    for (int j = 0; j < NP; ++j) {
      const int64_t i = j * ld + e;
      if constexpr (SI == 0) {
        const double k1 = dt * k[j];
        Ao[i] = k1;
        Yo[i] = y[j] + k1;
      } else {
        Uo[i] = Uo[i] + 0.5 * (Ao[i] + dt * k[j]);
      }
    }
  }
}

template <int RK, int PHYS, int SI>
__global__ __launch_bounds__(kBlock) void k_stage(const DevProblem* __restrict__ probs,
                                                  const WorkItem* __restrict__ work, const double* yin,
                                                  double* yout, double* U, double* A, double* __restrict__ ring,
                                                  const int64_t* __restrict__ ctr, int32_t step_offset) {
  const WorkItem wi = work[blockIdx.x];
  const DevProblem& P = probs[wi.prob];
  const int64_t n = ctr[0] + step_offset;
  switch (P.np) {
    case 2: stage_elem<2, RK, PHYS, SI>(P, wi.tile, yin, yout, U, A, ring, n); break;
    case 3: stage_elem<3, RK, PHYS, SI>(P, wi.tile, yin, yout, U, A, ring, n); break;
    case 4: stage_elem<4, RK, PHYS, SI>(P, wi.tile, yin, yout, U, A, ring, n); break;
    default: stage_elem<5, RK, PHYS, SI>(P, wi.tile, yin, yout, U, A, ring, n); break;
  }
}

// --------------------------------------------------------------- adjoint ---
// Butcher form of the three integrators (the same maps as the forward
// algebraic forms): Y_i = U + dt sum_{j<i} a_ij K_j, U' = U + dt sum_i b_i K_i.
template <int RK>
__device__ constexpr double bt_a(int i, int j) {
  if constexpr (RK == RK_RK4) return (j == i - 1) ? (i == 3 ? 1.0 : 0.5) : 0.0;
  else if constexpr (RK == RK_SSP3) return i == 1 ? (j == 0 ? 1.0 : 0.0) : (i == 2 && j < 2 ? 0.25 : 0.0);
  else return (i == 1 && j == 0) ? 1.0 : 0.0;
}
template <int RK>
__device__ constexpr double bt_b(int i) {
  if constexpr (RK == RK_RK4) return (i == 0 || i == 3) ? 1.0 / 6.0 : 1.0 / 3.0;
  else if constexpr (RK == RK_SSP3) return i == 2 ? 2.0 / 3.0 : 1.0 / 6.0;
  else return 0.5;
}

// (d fhat / d u-, d fhat / d u+); local Lax-Friedrichs on the branch taken
// (ties pick u-), d|u|/du = sign(u) with sign(0) = +1.
template <int PHYS>
__device__ __forceinline__ void flux_partials(double um, double up, double a, double& dm, double& dp) {
  if constexpr (PHYS == PHYS_ADV_UPWIND) {
    dm = a >= 0.0 ? a : 0.0;
    dp = a >= 0.0 ? 0.0 : a;
  } else if constexpr (PHYS == PHYS_ADV_CENTRAL) {
    dm = 0.5 * a;
    dp = 0.5 * a;
  } else {
    const bool pick_m = fabs(um) >= fabs(up);
    const double lam = pick_m ? fabs(um) : fabs(up);
    const double dl_m = pick_m ? (um >= 0.0 ? 1.0 : -1.0) : 0.0;
    const double dl_p = pick_m ? 0.0 : (up >= 0.0 ? 1.0 : -1.0);
    const double jump = up - um;
    dm = 0.5 * um - 0.5 * dl_m * jump + 0.5 * lam;
    dp = 0.5 * up - 0.5 * dl_p * jump - 0.5 * lam;
  }
}

struct AdjPtrs {
  const double* __restrict__ Y;   // forward input of this stage
  const double* __restrict__ lam; // lambda_{n+1}
  double* __restrict__ lamu;      // lambda_n accumulator (starts as lambda_{n+1})
  double* __restrict__ Q;         // Q_i = sum_{j>i} a_ji mu_j, i < S-1, stride qstride
  int64_t qstride;
  const double* __restrict__ ring;  // forward raw PE fluxes (full history)
  double* __restrict__ adjring;     // their sensitivities (full history)
  double* __restrict__ cpart;       // per-workgroup dJ/da partial sums
};

// Reverse of stage SI of step n for one element: lambda_K = dt (b_SI lam + Q_SI),
// mu = (dK/dY)^T lambda_K with the transposed volume term, transposed face
// fluxes (both neighbours' lifts), and for PE faces the transposed AT
// combination: the delayed levels' share goes to the adjoint ring, the
// level-n raw flux collects its share plus what later steps deposited.
template <int NP, int RK, int PHYS, int SI>
__device__ __forceinline__ double adj_elem(const DevProblem& P, int tile, const AdjPtrs& A, int64_t n) {
  constexpr int S = rk_stages(RK);
  const int N = (int)P.n_elem;
  const int e = tile * kBlock + (int)threadIdx.x;
  if (e >= N) return 0.0;
  const int64_t ld = P.ld, off = P.u_off;
  const double a = P.speed, dt = P.dt;
  const int em = e == 0 ? N - 1 : e - 1;
  const int e1 = e + 1 == N ? 0 : e + 1;
  const double* __restrict__ Y = A.Y + off;
  double y[NP];
#pragma unroll
  for (int j = 0; j < NP; ++j) y[j] = Y[j * ld + e];
  const double um = Y[(NP - 1) * ld + em];
  const double upr = Y[e1];

  const double bs = dt * bt_b<RK>(SI);
  const double* __restrict__ lam = A.lam + off;
  const double* __restrict__ qs = A.Q + SI * A.qstride + off;
  auto lk = [&](int x, int i) {
    double v = bs * lam[i * ld + x];
    if constexpr (SI < S - 1) v += dt * qs[i * ld + x];
    return v;
  };
  double lke[NP];
  double lf_l = 0.0, lf_r = 0.0;
#pragma unroll
  for (int i = 0; i < NP; ++i) {
    lke[i] = lk(e, i);
    lf_l += P.Kl[i] * lke[i] - P.Kr[i] * lk(em, i);
    lf_r += P.Kl[i] * lk(e1, i) - P.Kr[i] * lke[i];
  }
  double mu[NP];
#pragma unroll
  for (int j = 0; j < NP; ++j) {
    double v = 0.0;
#pragma unroll
    for (int i = 0; i < NP; ++i) v += P.Kd[i * kMaxNp + j] * lke[i];
    mu[j] = PHYS == PHYS_BURGERS_LLF ? 2.0 * y[j] * v : v;
  }
  double dm_l, dp_l, dm_r, dp_r;
  flux_partials<PHYS>(um, y[0], a, dm_l, dp_l);
  flux_partials<PHYS>(y[NP - 1], upr, a, dm_r, dp_r);
  double raw_l = lf_l, raw_r = lf_r;
  // forward face fluxes (for the speed gradient)
  double fl = Physics<PHYS>::fhat(um, y[0], a);
  double fr = Physics<PHYS>::fhat(y[NP - 1], upr, a);
  if (P.async_faces) {
    const uint32_t pes = P.pe_div.d;
    const int depth = P.depth;
    const int slot_n = (int)(n % (int64_t)depth);
    const uint32_t bl = fast_div((uint32_t)e, P.pe_div);
    if ((uint32_t)e == bl * pes) {
      const int64_t rb = P.ring_off + ((int64_t)bl * S + SI) * depth;
      const int kd = pe_delay(P, n, SI, bl);
      raw_l = (kd == 0 ? lf_l : 0.0) + A.adjring[rb + slot_n];
      if (kd > 0) {
        fl = at_past_sum(P, A.ring + rb, kd, slot_n);
        for (int j = 0; j < P.q; ++j) A.adjring[rb + ring_slot(slot_n, kd + j, depth)] += P.atc[kd][j] * lf_l;
      }
    }
    const uint32_t br = fast_div((uint32_t)e1, P.pe_div);
    if ((uint32_t)e1 == br * pes) {
      const int64_t rb = P.ring_off + ((int64_t)br * S + SI) * depth;
      const int kd = pe_delay(P, n, SI, br);
      raw_r = (kd == 0 ? lf_r : 0.0) + A.adjring[rb + slot_n];
      if (kd > 0) fr = at_past_sum(P, A.ring + rb, kd, slot_n);
    }
  }
  mu[0] += raw_l * dp_l;
  mu[NP - 1] += raw_r * dm_r;

  double* __restrict__ lu = A.lamu + off;
#pragma unroll
  for (int j = 0; j < NP; ++j) lu[j * ld + e] += mu[j];
#pragma unroll
  for (int i = 0; i < SI; ++i) {
    const double c = bt_a<RK>(SI, i);
    if (c != 0.0) {
      double* __restrict__ qi = A.Q + i * A.qstride + off;
#pragma unroll
      for (int j = 0; j < NP; ++j) qi[j * ld + e] += c * mu[j];
    }
  }
  // dJ/da through this stage with its inputs held fixed: every term of K is
  // proportional to a for linear advection, so dK/da = K / a.
  double ca = 0.0;
  if constexpr (PHYS != PHYS_BURGERS_LLF) {
    double kf[NP];
    folded_rhs<NP, PHYS>(P, y, fl, fr, kf);
#pragma unroll
    for (int i = 0; i < NP; ++i) ca += lke[i] * kf[i];
    ca /= a;
  }
  return ca;
}

template <int RK, int PHYS, int SI>
__global__ __launch_bounds__(kBlock) void k_adj_stage(const DevProblem* __restrict__ probs,
                                                      const WorkItem* __restrict__ work, AdjPtrs A, int32_t n) {
  __shared__ double red[kBlock];
  const WorkItem wi = work[blockIdx.x];
  const DevProblem& P = probs[wi.prob];
  double ca;
  switch (P.np) {
    case 2: ca = adj_elem<2, RK, PHYS, SI>(P, wi.tile, A, n); break;
    case 3: ca = adj_elem<3, RK, PHYS, SI>(P, wi.tile, A, n); break;
    case 4: ca = adj_elem<4, RK, PHYS, SI>(P, wi.tile, A, n); break;
    default: ca = adj_elem<5, RK, PHYS, SI>(P, wi.tile, A, n); break;
  }
  if constexpr (PHYS != PHYS_BURGERS_LLF) {
    red[threadIdx.x] = ca;
    __syncthreads();
    for (int w = kBlock / 2; w > 0; w >>= 1) {
      if ((int)threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
      __syncthreads();
    }
    if (threadIdx.x == 0) A.cpart[blockIdx.x] += red[0];
  }
}

// ------------------------------------------------------ fused adjoint step ---
// Reverse of one whole RK step n in one launch: one wave64 per tile of
// T = 64 - 2H owned elements with H halo lanes per side, one element per lane.
// The forward stages are recomputed on chip from u^n (keeping what the reverse
// needs: the stage operator values K_i for the speed gradient of advection,
// the stage inputs Y_i for the Burgers Jacobian), then the stages are reversed
// in Butcher form with the face terms exchanged between lanes:
//   lambda_K,i = dt (b_i lambda^{n+1} + sum_{j>i} a_ji mu_j),
//   mu_i = (dK_i/dY_i)^T lambda_K,i,   lambda^n = lambda^{n+1} + sum_i mu_i.
// Each reverse stage widens the dependence by one element per side, so after
// S stages the owned lanes are exact when the Jacobian is constant (linear
// advection, H = S).  For Burgers reverse stage s also reads the stage input
// Y_s one lane further out, which is exact only s lanes in from the wave's
// edge: H = 2S - 1.  PE faces take the transposed AT
// combination: the delayed levels' weights go to the adjoint ring (levels
// below n, deposited by the owner lane only), the raw level-n flux collects
// its synchronous share plus what later steps deposited at level n.
template <int NP, int RK, int PHYS, bool FWD>
__device__ __forceinline__ void adj_tile(const DevProblem& P, const WorkItem wi, int w, int lane, int32_t n,
                                         const double* __restrict__ uin, const double* __restrict__ lam,
                                         double* __restrict__ lamo, const double* __restrict__ ring,
                                         double* __restrict__ adjring, double* __restrict__ cpart) {
  constexpr int S = rk_stages(RK);
  constexpr int HL = adj_halo(RK, PHYS == PHYS_BURGERS_LLF);
  constexpr int T = kWave - 2 * HL;
  const int N = (int)P.n_elem;
  const int e0 = wi.tile * T;
  const int teff = (N - e0) < T ? (N - e0) : T;
  const int x = e0 - HL + lane;
  const int e = N < kWave ? wrap_elem(x, N) : wrap_once(x, N);
  const bool owned = lane >= HL && lane < kWave - HL && (x - e0) < teff;
  const int64_t ld = P.ld;
  const double* __restrict__ lp = lam + P.u_off;
  double u0[NP], lamp[NP];
#pragma unroll
  for (int j = 0; j < NP; ++j) {
    if constexpr (FWD) u0[j] = uin[P.u_off + j * ld + e];
    lamp[j] = lp[j * ld + e];
  }

  // PE face on this lane's left face: delays of step n, the applied AT sums of
  // past levels and the adjoint already collected for the level-n raw fluxes
  bool pe = false;
  uint32_t b = 0;
  int depth = 1, slot_n = 0;
  int kd[S];
  double atf[S], adjn[S];
#pragma unroll
  for (int s = 0; s < S; ++s) { kd[s] = 0; atf[s] = 0.0; adjn[s] = 0.0; }
  if (P.async_faces) {
    depth = P.depth;
    slot_n = (int)((uint32_t)n - fast_div((uint32_t)n, P.depth_div) * (uint32_t)depth);
    const uint32_t bl = fast_div((uint32_t)e, P.pe_div);
    pe = (uint32_t)e == bl * P.pe_div.d;
    if (pe) {
      b = bl;
      const uint64_t pre0 = delay_prefix(P.seed, n, 0);
#pragma unroll
      for (int s = 0; s < S; ++s) {
        const uint64_t pre = P.per_stage ? delay_prefix(P.seed, n, s) : pre0;
        kd[s] = clamp_delay(delay_from_prefix(pre, b, P.thr, P.n_delays), n, P.q);
        const int64_t rb = P.ring_off + ((int64_t)b * S + s) * depth;
        adjn[s] = adjring[rb + slot_n];
        if (FWD && kd[s] > 0) atf[s] = at_past_sum(P, ring + rb, kd[s], slot_n);
      }
    }
  }

  // forward stages, keeping K_s (advection) or Y_s (Burgers) in registers
  // (a per-lane LDS copy lowers the occupancy further and measured slower)
  const double a = P.speed, dt = P.dt;
  double keep[S][NP];
  auto kept = [&](int s, int j) -> double& { return keep[s][j]; };
  if constexpr (FWD) {
    double y[NP], ks[NP], k[NP];
#pragma unroll
    for (int j = 0; j < NP; ++j) y[j] = u0[j];
#pragma unroll
    for (int s = 0; s < S; ++s) {
      double F = Physics<PHYS>::fhat(lane_from_left(y[NP - 1]), y[0], a);
      if (pe && kd[s] > 0) F = atf[s];
      folded_rhs<NP, PHYS>(P, y, F, lane_from_right(F), k);
#pragma unroll
      for (int j = 0; j < NP; ++j) kept(s, j) = PHYS == PHYS_BURGERS_LLF ? y[j] : k[j];
      if (s + 1 < S) rk_update<NP, RK>(s, dt, u0, y, ks, k);
    }
  }

  // reverse stages
  double lu[NP], Q[S][NP];
#pragma unroll
  for (int j = 0; j < NP; ++j) lu[j] = lamp[j];
#pragma unroll
  for (int s = 0; s < S; ++s)
#pragma unroll
    for (int j = 0; j < NP; ++j) Q[s][j] = 0.0;
  double ca = 0.0;
#pragma unroll
  for (int s = S - 1; s >= 0; --s) {
    double lk[NP];
    const double bs = dt * bt_b<RK>(s);
#pragma unroll
    for (int i = 0; i < NP; ++i) lk[i] = s < S - 1 ? bs * lamp[i] + dt * Q[s][i] : bs * lamp[i];
    double cl = 0.0, cr = 0.0;
#pragma unroll
    for (int i = 0; i < NP; ++i) {
      cl += P.Kl[i] * lk[i];
      cr += P.Kr[i] * lk[i];
    }
    // sensitivity of the flux applied at the left face (both neighbours' lifts)
    const double lf = cl - lane_from_left(cr);
    double dm, dp;
    if constexpr (PHYS == PHYS_BURGERS_LLF)
      flux_partials<PHYS>(lane_from_left(kept(s, NP - 1)), kept(s, 0), a, dm, dp);
    else
      flux_partials<PHYS>(0.0, 0.0, a, dm, dp);
    double raw = lf;
    if (pe) {
      const int kk = kd[s];
      raw = (kk == 0 ? lf : 0.0) + adjn[s];
      if (owned && kk > 0) {
        double* __restrict__ rb = adjring + P.ring_off + ((int64_t)b * S + s) * depth;
        for (int j = 0; j < P.q; ++j) rb[ring_slot(slot_n, kk + j, depth)] += P.atc[kk][j] * lf;
      }
    }
    double mu[NP];
#pragma unroll
    for (int j = 0; j < NP; ++j) {
      double v = 0.0;
#pragma unroll
      for (int i = 0; i < NP; ++i) v += P.Kd[i * kMaxNp + j] * lk[i];
      if constexpr (PHYS == PHYS_BURGERS_LLF)
        mu[j] = 2.0 * kept(s, j) * v;
      else
        mu[j] = v;
    }
    mu[0] += raw * dp;
    mu[NP - 1] += lane_from_right(raw * dm);  // the right face is the next lane's left face
#pragma unroll
    for (int j = 0; j < NP; ++j) lu[j] += mu[j];
#pragma unroll
    for (int i = 0; i < s; ++i) {
      const double c = bt_a<RK>(s, i);
      if (c != 0.0)
#pragma unroll
        for (int j = 0; j < NP; ++j) Q[i][j] += c * mu[j];
    }
    if constexpr (FWD && PHYS != PHYS_BURGERS_LLF) {
      if (owned)
#pragma unroll
        for (int i = 0; i < NP; ++i) ca += lk[i] * kept(s, i);
    }
  }

  double* __restrict__ lo = lamo + P.u_off;
  if (owned)
#pragma unroll
    for (int j = 0; j < NP; ++j) lo[j * ld + e] = lu[j];

  // dJ/da share of this tile: every term of K is proportional to a for linear
  // advection, so dK/da = K / a with the stage inputs held fixed.  Fixed
  // butterfly order: deterministic.
  if constexpr (FWD && PHYS != PHYS_BURGERS_LLF) {
#pragma unroll
    for (int o = kWave / 2; o > 0; o >>= 1) ca += __shfl_xor(ca, o, kWave);
    if (lane == 0) cpart[w] += ca / a;
  }
}

template <int NP, int RK, int PHYS, bool FWD>
__global__ __launch_bounds__(kBlock) void k_adj_fused(const DevProblem* __restrict__ probs,
                                                      const WorkItem* __restrict__ work, int32_t w_begin,
                                                      int32_t w_end, const double* __restrict__ u,
                                                      const double* __restrict__ lam, double* __restrict__ lamo,
                                                      const double* __restrict__ ring,
                                                      double* __restrict__ adjring, double* __restrict__ cpart,
                                                      int32_t n) {
  const int wv = __builtin_amdgcn_readfirstlane((int)(threadIdx.x / kWave));
  const int lane = (int)(threadIdx.x % kWave);
  const int w = w_begin + (int)blockIdx.x * kWavesPerBlock + wv;
  if (w >= w_end) return;  // whole wave
  const WorkItem wi = work[w];
  adj_tile<NP, RK, PHYS, FWD>(probs[wi.prob], wi, w, lane, n, u, lam, lamo, ring, adjring, cpart);
}

// ----------------------------------------------------------- statistics ---
__global__ __launch_bounds__(kBlock) void k_stats_partial(const DevProblem* __restrict__ probs,
                                                          const WorkItem* __restrict__ work,
                                                          const double* __restrict__ u,
                                                          const double* __restrict__ ref,
                                                          double* __restrict__ part) {
  __shared__ double red[3][kBlock];
  const WorkItem wi = work[blockIdx.x];
  const DevProblem& P = probs[wi.prob];
  const int64_t e = (int64_t)wi.tile * kBlock + threadIdx.x;
  double sabs = 0.0, mabs = 0.0, integ = 0.0;
  if (e < P.n_elem) {
    for (int j = 0; j < P.np; ++j) {
      const int64_t i = P.u_off + j * P.ld + e;
      const double d = fabs(u[i] - ref[i]);
      sabs += d;
      mabs = fmax(mabs, d);
      integ += P.wq[j] * u[i];
    }
  }
  red[0][threadIdx.x] = sabs;
  red[1][threadIdx.x] = mabs;
  red[2][threadIdx.x] = integ;
  __syncthreads();
  for (int w = kBlock / 2; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) {
      red[0][threadIdx.x] += red[0][threadIdx.x + w];
      red[1][threadIdx.x] = fmax(red[1][threadIdx.x], red[1][threadIdx.x + w]);
      red[2][threadIdx.x] += red[2][threadIdx.x + w];
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    part[3 * blockIdx.x + 0] = red[0][0];
    part[3 * blockIdx.x + 1] = red[1][0];
    part[3 * blockIdx.x + 2] = red[2][0];
  }
}

// One workgroup per problem: lane l sums items first+l, first+l+256, ... in
// order, then a fixed tree.
__global__ __launch_bounds__(kBlock) void k_stats_final(const DevProblem* __restrict__ probs,
                                                        const int32_t* __restrict__ first_item,
                                                        const double* __restrict__ part, double* __restrict__ out) {
  __shared__ double red[3][kBlock];
  const int p = blockIdx.x;
  const DevProblem& P = probs[p];
  const int32_t i0 = first_item[p], i1 = first_item[p + 1];
  double s0 = 0.0, s1 = 0.0, s2 = 0.0;
  for (int32_t i = i0 + threadIdx.x; i < i1; i += kBlock) {
    s0 += part[3 * i];
    s1 = fmax(s1, part[3 * i + 1]);
    s2 += part[3 * i + 2];
  }
  red[0][threadIdx.x] = s0;
  red[1][threadIdx.x] = s1;
  red[2][threadIdx.x] = s2;
  __syncthreads();
  for (int w = kBlock / 2; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) {
      red[0][threadIdx.x] += red[0][threadIdx.x + w];
      red[1][threadIdx.x] = fmax(red[1][threadIdx.x], red[1][threadIdx.x + w]);
      red[2][threadIdx.x] += red[2][threadIdx.x + w];
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    out[3 * p + 0] = red[0][0] / (double)(P.n_elem * P.np);
    out[3 * p + 1] = red[1][0];
    out[3 * p + 2] = P.half_dx * red[2][0];
  }
}

// One workgroup per group: two passes over the group's problems in list
// order (mean, then mean squared deviation) of <E> and of max|u - ref|.
__global__ void k_group_stats(const double* __restrict__ pstats, const int32_t* __restrict__ gstart,
                              const int32_t* __restrict__ gmembers, double* __restrict__ out) {
  if (threadIdx.x != 0) return;
  const int g = blockIdx.x;
  const int32_t b = gstart[g], e = gstart[g + 1];
  const double m = (double)(e - b);
  double s0 = 0.0, s1 = 0.0;
  for (int32_t i = b; i < e; ++i) {
    s0 += pstats[3 * gmembers[i] + 0];
    s1 += pstats[3 * gmembers[i] + 1];
  }
  const double mean0 = e > b ? s0 / m : 0.0, mean1 = e > b ? s1 / m : 0.0;
  double v0 = 0.0, v1 = 0.0;
  for (int32_t i = b; i < e; ++i) {
    const double d0 = pstats[3 * gmembers[i] + 0] - mean0;
    const double d1 = pstats[3 * gmembers[i] + 1] - mean1;
    v0 += d0 * d0;
    v1 += d1 * d1;
  }
  out[4 * g + 0] = mean0;
  out[4 * g + 1] = e > b ? v0 / m : 0.0;
  out[4 * g + 2] = mean1;
  out[4 * g + 3] = e > b ? v1 / m : 0.0;
}

hipError_t launch_group_stats(const double* pstats, const int32_t* gstart, const int32_t* gmembers, int32_t n_groups,
                              double* out, hipStream_t stream) {
  hipLaunchKernelGGL(k_group_stats, dim3(n_groups), dim3(64), 0, stream, pstats, gstart, gmembers, out);
  return hipGetLastError();
}

__global__ __launch_bounds__(kBlock) void k_check_finite(const DevProblem* __restrict__ probs,
                                                         const WorkItem* __restrict__ work,
                                                         const double* __restrict__ u, int64_t* __restrict__ ctr) {
  const WorkItem wi = work[blockIdx.x];
  const DevProblem& P = probs[wi.prob];
  const int64_t e = (int64_t)wi.tile * kBlock + threadIdx.x;
  if (e >= P.n_elem) return;
  bool bad = false;
  for (int j = 0; j < P.np; ++j) bad |= !isfinite(u[P.u_off + j * P.ld + e]);
  if (bad) ctr[2] = 1;
}

// ---------------------------------------------------------------- launch ---
template <int NP, int RK, int PHYS>
static void fused_go(const StepArgs& a, int gi, const double* uin, double* uout, int32_t off, hipStream_t st) {
  const dim3 g(a.grid[gi]), b(kBlock);
  switch (a.lane_elems) {
    case 1:
      hipLaunchKernelGGL((k_fused_step<NP, RK, PHYS, 1>), g, b, 0, st, a.probs, a.work, a.ctr, a.ring, a.atsum, a.atk,
                         a.group[gi], a.group[gi + 1], uin, uout, off);
      break;
    case 4:
      hipLaunchKernelGGL((k_fused_step<NP, RK, PHYS, 4>), g, b, 0, st, a.probs, a.work, a.ctr, a.ring, a.atsum, a.atk,
                         a.group[gi], a.group[gi + 1], uin, uout, off);
      break;
    default:
      hipLaunchKernelGGL((k_fused_step<NP, RK, PHYS, 2>), g, b, 0, st, a.probs, a.work, a.ctr, a.ring, a.atsum, a.atk,
                         a.group[gi], a.group[gi + 1], uin, uout, off);
      break;
  }
}

template <int RK, int PHYS>
static void fused_np(const StepArgs& a, const double* uin, double* uout, int32_t off, hipStream_t st) {
  // degree ranges np = 5, 4, 3, 2
  if (a.group[1] > a.group[0]) fused_go<5, RK, PHYS>(a, 0, uin, uout, off, st);
  if (a.group[2] > a.group[1]) fused_go<4, RK, PHYS>(a, 1, uin, uout, off, st);
  if (a.group[3] > a.group[2]) fused_go<3, RK, PHYS>(a, 2, uin, uout, off, st);
  if (a.group[4] > a.group[3]) fused_go<2, RK, PHYS>(a, 3, uin, uout, off, st);
}

template <int RK>
static void fused_phys(int phys, const StepArgs& a, const double* uin, double* uout, int32_t off, hipStream_t st) {
  switch (phys) {
    case PHYS_ADV_UPWIND: fused_np<RK, PHYS_ADV_UPWIND>(a, uin, uout, off, st); break;
    case PHYS_ADV_UPWIND_POS: fused_np<RK, PHYS_ADV_UPWIND_POS>(a, uin, uout, off, st); break;
    case PHYS_ADV_CENTRAL: fused_np<RK, PHYS_ADV_CENTRAL>(a, uin, uout, off, st); break;
    default: fused_np<RK, PHYS_BURGERS_LLF>(a, uin, uout, off, st); break;
  }
}

hipError_t launch_fused_step(int rk, int phys, const StepArgs& a, const double* uin, double* uout, int32_t step_offset,
                             hipStream_t stream) {
  switch (rk) {
    case RK_HEUN: fused_phys<RK_HEUN>(phys, a, uin, uout, step_offset, stream); break;
    case RK_SSP3: fused_phys<RK_SSP3>(phys, a, uin, uout, step_offset, stream); break;
    default: fused_phys<RK_RK4>(phys, a, uin, uout, step_offset, stream); break;
  }
  return hipGetLastError();
}

template <int RK, int PHYS, int SI>
static void stage_go(const StepArgs& a, const double* yin, double* yout, double* U, double* A, int32_t off,
                     hipStream_t st) {
  hipLaunchKernelGGL((k_stage<RK, PHYS, SI>), dim3(a.n_work), dim3(kBlock), 0, st, a.probs, a.work, yin, yout, U, A,
                     a.ring, a.ctr, off);
}

template <int RK, int PHYS>
static void stage_si(int si, const StepArgs& a, const double* yin, double* yout, double* U, double* A, int32_t off,
                     hipStream_t st) {
  switch (si) {
    case 0: stage_go<RK, PHYS, 0>(a, yin, yout, U, A, off, st); break;
    case 1: stage_go<RK, PHYS, 1>(a, yin, yout, U, A, off, st); break;
    case 2: if constexpr (rk_stages(RK) > 2) stage_go<RK, PHYS, 2>(a, yin, yout, U, A, off, st); break;
    default: if constexpr (rk_stages(RK) > 3) stage_go<RK, PHYS, 3>(a, yin, yout, U, A, off, st); break;
  }
}

template <int RK>
static void stage_phys(int phys, int si, const StepArgs& a, const double* yin, double* yout, double* U, double* A,
                       int32_t off, hipStream_t st) {
  switch (phys) {
    case PHYS_ADV_UPWIND: stage_si<RK, PHYS_ADV_UPWIND>(si, a, yin, yout, U, A, off, st); break;
    case PHYS_ADV_CENTRAL: stage_si<RK, PHYS_ADV_CENTRAL>(si, a, yin, yout, U, A, off, st); break;
    default: stage_si<RK, PHYS_BURGERS_LLF>(si, a, yin, yout, U, A, off, st); break;
  }
}

hipError_t launch_stage(int rk, int phys, int stage, const StepArgs& a, const double* yin, double* yout, double* U,
                        double* A, int32_t step_offset, hipStream_t stream) {
  switch (rk) {
    case RK_HEUN: stage_phys<RK_HEUN>(phys, stage, a, yin, yout, U, A, step_offset, stream); break;
    case RK_SSP3: stage_phys<RK_SSP3>(phys, stage, a, yin, yout, U, A, step_offset, stream); break;
    default: stage_phys<RK_RK4>(phys, stage, a, yin, yout, U, A, step_offset, stream); break;
  }
  return hipGetLastError();
}

template <int RK, int PHYS, int SI>
static void adj_go(const StepArgs& a, const AdjPtrs& p, int32_t n, hipStream_t st) {
  hipLaunchKernelGGL((k_adj_stage<RK, PHYS, SI>), dim3(a.n_work), dim3(kBlock), 0, st, a.probs, a.work, p, n);
}

template <int RK, int PHYS>
static void adj_si(int si, const StepArgs& a, const AdjPtrs& p, int32_t n, hipStream_t st) {
  switch (si) {
    case 0: adj_go<RK, PHYS, 0>(a, p, n, st); break;
    case 1: adj_go<RK, PHYS, 1>(a, p, n, st); break;
    case 2: if constexpr (rk_stages(RK) > 2) adj_go<RK, PHYS, 2>(a, p, n, st); break;
    default: if constexpr (rk_stages(RK) > 3) adj_go<RK, PHYS, 3>(a, p, n, st); break;
  }
}

template <int RK>
static void adj_phys(int phys, int si, const StepArgs& a, const AdjPtrs& p, int32_t n, hipStream_t st) {
  switch (phys) {
    case PHYS_ADV_UPWIND: adj_si<RK, PHYS_ADV_UPWIND>(si, a, p, n, st); break;
    case PHYS_ADV_CENTRAL: adj_si<RK, PHYS_ADV_CENTRAL>(si, a, p, n, st); break;
    default: adj_si<RK, PHYS_BURGERS_LLF>(si, a, p, n, st); break;
  }
}

hipError_t launch_adj_stage(int rk, int phys, int stage, const StepArgs& a, const double* Y, const double* lam,
                            double* lamu, double* Q, int64_t qstride, const double* ring, double* adjring,
                            double* cpart, int32_t n, hipStream_t stream) {
  const AdjPtrs p{Y, lam, lamu, Q, qstride, ring, adjring, cpart};
  switch (rk) {
    case RK_HEUN: adj_phys<RK_HEUN>(phys, stage, a, p, n, stream); break;
    case RK_SSP3: adj_phys<RK_SSP3>(phys, stage, a, p, n, stream); break;
    default: adj_phys<RK_RK4>(phys, stage, a, p, n, stream); break;
  }
  return hipGetLastError();
}

template <int RK, int PHYS, bool FWD>
static void adj_fused_go(const AdjArgs& a, const double* u, const double* lam, double* lamo, const double* ring,
                         double* adjring, double* cpart, int32_t n, hipStream_t st) {
  for (int gi = 0; gi < 4; ++gi) {
    const int32_t wb = a.group[gi], we = a.group[gi + 1];
    if (we <= wb) continue;
    const dim3 grid(a.grid[gi]), block(kBlock);
    switch (gi) {
      case 0: hipLaunchKernelGGL((k_adj_fused<5, RK, PHYS, FWD>), grid, block, 0, st, a.probs, a.work, wb, we, u,
                                 lam, lamo, ring, adjring, cpart, n); break;
      case 1: hipLaunchKernelGGL((k_adj_fused<4, RK, PHYS, FWD>), grid, block, 0, st, a.probs, a.work, wb, we, u,
                                 lam, lamo, ring, adjring, cpart, n); break;
      case 2: hipLaunchKernelGGL((k_adj_fused<3, RK, PHYS, FWD>), grid, block, 0, st, a.probs, a.work, wb, we, u,
                                 lam, lamo, ring, adjring, cpart, n); break;
      default: hipLaunchKernelGGL((k_adj_fused<2, RK, PHYS, FWD>), grid, block, 0, st, a.probs, a.work, wb, we, u,
                                  lam, lamo, ring, adjring, cpart, n); break;
    }
  }
}

// Linear advection needs the forward stages only for dJ/da (u == nullptr:
// skipped); Burgers always needs them for its Jacobian.
template <int RK>
static void adj_fused_rk(int phys, const AdjArgs& a, const double* u, const double* lam, double* lamo,
                         const double* ring, double* adjring, double* cpart, int32_t n, hipStream_t st) {
  const bool fwd = u != nullptr;
  switch (phys) {
    case PHYS_ADV_CENTRAL:
      if (fwd) adj_fused_go<RK, PHYS_ADV_CENTRAL, true>(a, u, lam, lamo, ring, adjring, cpart, n, st);
      else adj_fused_go<RK, PHYS_ADV_CENTRAL, false>(a, u, lam, lamo, ring, adjring, cpart, n, st);
      break;
    case PHYS_BURGERS_LLF: adj_fused_go<RK, PHYS_BURGERS_LLF, true>(a, u, lam, lamo, ring, adjring, cpart, n, st); break;
    default:
      if (fwd) adj_fused_go<RK, PHYS_ADV_UPWIND, true>(a, u, lam, lamo, ring, adjring, cpart, n, st);
      else adj_fused_go<RK, PHYS_ADV_UPWIND, false>(a, u, lam, lamo, ring, adjring, cpart, n, st);
      break;
  }
}

hipError_t launch_adj_fused(int rk, int phys, const AdjArgs& a, const double* u, const double* lam, double* lamo,
                            const double* ring, double* adjring, double* cpart, int32_t n, hipStream_t stream) {
  switch (rk) {
    case RK_HEUN: adj_fused_rk<RK_HEUN>(phys, a, u, lam, lamo, ring, adjring, cpart, n, stream); break;
    case RK_SSP3: adj_fused_rk<RK_SSP3>(phys, a, u, lam, lamo, ring, adjring, cpart, n, stream); break;
    default: adj_fused_rk<RK_RK4>(phys, a, u, lam, lamo, ring, adjring, cpart, n, stream); break;
  }
  return hipGetLastError();
}

__global__ void k_set_counter(int64_t* __restrict__ ctr, int64_t v) {
  if (threadIdx.x == 0 && blockIdx.x == 0) ctr[0] = v;
}

hipError_t launch_set_counter(int64_t* ctr, int64_t value, hipStream_t stream) {
  hipLaunchKernelGGL(k_set_counter, dim3(1), dim3(64), 0, stream, ctr, value);
  return hipGetLastError();
}

hipError_t launch_advance(int64_t* ctr, int64_t n_steps, hipStream_t stream) {
  hipLaunchKernelGGL(k_advance, dim3(1), dim3(64), 0, stream, ctr, n_steps);
  return hipGetLastError();
}

hipError_t launch_stats(const StepArgs& a, const double* u, const double* ref, double* partials,
                        const int32_t* first_item, int32_t n_probs, double* out, hipStream_t stream) {
  hipLaunchKernelGGL(k_stats_partial, dim3(a.n_work), dim3(kBlock), 0, stream, a.probs, a.work, u, ref, partials);
  hipLaunchKernelGGL(k_stats_final, dim3(n_probs), dim3(kBlock), 0, stream, a.probs, first_item, partials, out);
  return hipGetLastError();
}

hipError_t launch_check_finite(const StepArgs& a, const double* u, hipStream_t stream) {
  hipLaunchKernelGGL(k_check_finite, dim3(a.n_work), dim3(kBlock), 0, stream, a.probs, a.work, u, a.ctr);
  return hipGetLastError();
}

}  // namespace adg
