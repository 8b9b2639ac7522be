// Device helpers shared by the HIP kernels (gfx950, FP64) of the asynchronous
// DG stepper with AT fluxes: physics, the PE-face ring, the element operator,
// the RK updates, lane shifts and the Butcher tables of the adjoint.
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
// Neighbour traces come through DPP lane shifts (fused kernels) or through the cache
// from the neighbouring lanes' own loads (stage kernel).  No MFMA: the
// per-element operators are at most 5x5.
#pragma once

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
struct Physics<PHYS_BURGERS_LDG>;  // viscous Burgers: the inviscid part is Physics<PHYS_BURGERS_LLF>

template <>
struct Physics<PHYS_BURGERS_LLF> {
  __device__ static double f(double u, double) { return 0.5 * u * u; }
  __device__ static double fhat(double um, double up, double) {
#pragma clang fp contract(off)
    const double lam = fmax(fabs(um), fabs(up));
    const double avg = 0.5 * (fma(0.5 * um, um, (0.5 * up) * up));
    return fma(-0.5 * lam, up - um, avg);
  }
};

// ------------------------------------------------------- PE-face AT flux ---
// Slot of level n - back (0 <= back < depth) given slot_n = n mod depth.
__device__ __forceinline__ int ring_slot(int slot_n, int back, int depth) {
  const int s = slot_n - back;
  return s < 0 ? s + depth : s;
}

// Clamped delay of boundary b at (step n, stage s): the hash of
// draw_delay with the threshold count unrolled over kMaxL - 1 (the threshold
// loads issue together instead of one per loop trip).
__device__ __forceinline__ int pe_delay(const DevProblem& P, int64_t n, int s, uint32_t b) {
  int k = 0;
  if (P.caa) {
    k = caa_delay(n);
  } else {
    const uint64_t u = splitmix64(delay_prefix(P.seed, n, P.per_stage ? s : 0) ^ (uint64_t)b) >> 11;
#pragma unroll
    for (int i = 0; i < kMaxL - 1; ++i) k += (i < P.n_delays - 1 && u >= P.thr[i]) ? 1 : 0;
  }
  return clamp_delay(k, n, P.q);
}

// sum_{j<q} c_j(k) F^{n-k-j} over the ring of (boundary, stage); k >= 1, so
// every level is a past one.
__device__ __forceinline__ double at_past_sum(const DevProblem& P, const double* __restrict__ r, int k,
                                              int slot_n) {
  double acc = 0.0;  // oldest level first, as in every other path
  for (int j = P.q - 1; j >= 0; --j) acc = fma(P.atc[k][j], r[ring_slot(slot_n, k + j, P.depth)], acc);
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

// 2N-storage low-storage schemes of the family the paper integrates with
// (Sec. 6.1): dU_s = A_s dU_{s-1} + dt L(U_{s-1}), U_s = U_{s-1} + B_s dU_s.
// Williamson's three-stage third-order scheme (1980) and Carpenter & Kennedy's
// five-stage fourth-order scheme (1994), their published coefficients; each
// ratio of integers below 2^53 is rounded once, by the compiler's division.
__host__ __device__ constexpr double ls_a(int rk, int s) {
  if (rk == RK_LS3) return s == 1 ? -5.0 / 9.0 : (s == 2 ? -153.0 / 128.0 : 0.0);
  return s == 1 ? -567301805773.0 / 1357537059087.0
       : s == 2 ? -2404267990393.0 / 2016746695238.0
       : s == 3 ? -3550918686646.0 / 2091501179385.0
       : s == 4 ? -1275806237668.0 / 842570457699.0 : 0.0;
}
__host__ __device__ constexpr double ls_b(int rk, int s) {
  if (rk == RK_LS3) return s == 0 ? 1.0 / 3.0 : (s == 1 ? 15.0 / 16.0 : 8.0 / 15.0);
  return s == 0 ? 1432997174477.0 / 9575080441755.0
       : s == 1 ? 5161836677717.0 / 13612068292357.0
       : s == 2 ? 1720146321549.0 / 2090206949498.0
       : s == 3 ? 3134564353537.0 / 4481467310338.0 : 2277821191437.0 / 14882151754819.0;
}
__host__ __device__ constexpr bool low_storage(int rk) { return rk == RK_LS3 || rk == RK_LS4; }

// RK update after the stage-s operator value k (oracle's algebraic forms).
// Every multiply-add is an explicit FMA and nothing else is contracted, so
// the rounding does not depend on how the compiler schedules the caller
// (kernels of different launch shapes then agree bitwise).
// u0: u^n; y: stage input (in) -> next stage input or u^{n+1} (out);
// ks: RK4 running sum k1 + 2k2 + 2k3, Heun k1 = dt L(u^n).
template <int NP, int RK>
__device__ __forceinline__ void rk_update(int s, double dt, const double (&u0)[NP], double (&y)[NP],
                                          double (&ks)[NP], const double (&k)[NP]) {
#pragma clang fp contract(off)
  if constexpr (RK == RK_RK4) {
    if (s == 0) {
#pragma unroll
      for (int j = 0; j < NP; ++j) { ks[j] = k[j]; y[j] = fma(0.5 * dt, k[j], u0[j]); }
    } else if (s == 1) {
#pragma unroll
      for (int j = 0; j < NP; ++j) { ks[j] = fma(2.0, k[j], ks[j]); y[j] = fma(0.5 * dt, k[j], u0[j]); }
    } else if (s == 2) {
#pragma unroll
      for (int j = 0; j < NP; ++j) { ks[j] = fma(2.0, k[j], ks[j]); y[j] = fma(dt, k[j], u0[j]); }
    } else {
#pragma unroll
      for (int j = 0; j < NP; ++j) y[j] = fma(dt / 6.0, ks[j] + k[j], u0[j]);
    }
  } else if constexpr (RK == RK_SSP3) {
    if (s == 0) {
#pragma unroll
      for (int j = 0; j < NP; ++j) y[j] = fma(dt, k[j], u0[j]);
    } else if (s == 1) {
#pragma unroll
      for (int j = 0; j < NP; ++j) y[j] = fma(0.25, fma(dt, k[j], y[j]), 0.75 * u0[j]);
    } else {
#pragma unroll
      for (int j = 0; j < NP; ++j) y[j] = fma(2.0 / 3.0, fma(dt, k[j], y[j]), u0[j] / 3.0);
    }
  } else if constexpr (low_storage(RK)) {
    // 2N-storage form, ks holding dU: dU = A_s dU + dt k, y = y + B_s dU
    const double Bs = ls_b(RK, s);
    if (s == 0) {
#pragma unroll
      for (int j = 0; j < NP; ++j) { ks[j] = dt * k[j]; y[j] = fma(Bs, ks[j], y[j]); }
    } else {
      const double As = ls_a(RK, s);
#pragma unroll
      for (int j = 0; j < NP; ++j) { ks[j] = fma(As, ks[j], dt * k[j]); y[j] = fma(Bs, ks[j], y[j]); }
    }
  } else {  // Heun
    if (s == 0) {
#pragma unroll
      for (int j = 0; j < NP; ++j) { ks[j] = dt * k[j]; y[j] = u0[j] + ks[j]; }
    } else {
#pragma unroll
      for (int j = 0; j < NP; ++j) y[j] = fma(0.5, fma(dt, k[j], ks[j]), u0[j]);
    }
  }
}

// Raw buffer resource over the planes of one problem (gfx9 descriptor: base
// address, no stride, byte range 2^31 - 1, dword 3 = 0x00020000 for untyped
// loads and stores); accesses pass the lane's byte offset and the plane's.
typedef unsigned int BufWord4 __attribute__((ext_vector_type(4)));
typedef unsigned int BufWord2 __attribute__((ext_vector_type(2)));
__device__ __forceinline__ __amdgpu_buffer_rsrc_t plane_rsrc(const double* p) {
  return __builtin_amdgcn_make_buffer_rsrc(const_cast<double*>(p), 0, 0x7fffffff, 0x00020000);
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

// Workgroups are dispatched to the 8 XCDs round robin (workgroup i to XCD
// i mod 8), and each XCD has its own L2.  Renumbering so that XCD x runs a
// contiguous range of tiles makes the halo elements shared by neighbouring
// workgroups hit in the same L2 instead of being fetched twice from HBM.
// A bijection of [0, nb) whatever the dispatch order.
constexpr int kXcds = 8;
__device__ __forceinline__ int xcd_block(int i, int nb) {
  const int q = nb / kXcds, r = nb % kXcds;
  const int x = i % kXcds, k = i / kXcds;
  return x < r ? x * (q + 1) + k : r * (q + 1) + (x - r) * q + k;
}

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

// Per-lane PE-face values.  at[kk][s][lane]: the AT sum of step n + kk
// (read by the lane itself), then the raw level-(n + kk) flux of an owner
// lane (read at the end by the lanes that form the next records).  With
// R <= PE size a lane's R left faces hold at most one PE face.  part / kdj:
// per record job (a lane of an owner wave), the sum over the levels before
// the launch and the delay, formed at the start of the launch.
template <int K, int S>
struct WaveSmemK {
  double at[K][kWavesPerBlock][S][kWave];
  double part[kWavesPerBlock][kWave];
  int32_t kdj[kWavesPerBlock][kWave];
};

template <int NP, int PHYS>
__device__ __forceinline__ void folded_rhs(const DevProblem& P, const double (&y)[NP], double fl, double fr,
                                           double (&k)[NP]) {
#pragma clang fp contract(off)
  double g[NP];
#pragma unroll
  for (int j = 0; j < NP; ++j) g[j] = PHYS == PHYS_BURGERS_LLF ? y[j] * y[j] : y[j];
#pragma unroll
  for (int i = 0; i < NP; ++i) {
    double v = fma(-P.Kr[i], fr, P.Kl[i] * fl);
#pragma unroll
    for (int j = 0; j < NP; ++j) v = fma(P.Kd[i * kMaxNp + j], g[j], v);
    k[i] = v;
  }
}

struct FusedPtrs {
  double* __restrict__ ring;
  double* __restrict__ atsum;
  RecWord* __restrict__ atk;
};

// Lane of the i-th set bit (from 0) of a wave-uniform mask, 0 if there is none.
__device__ __forceinline__ int nth_set_lane(uint64_t mask, int i) {
  int lane = 0;
  for (int c = 0; mask != 0; ++c) {
    const int bit = __builtin_ctzll(mask);
    mask &= mask - 1;
    if (c == i) lane = bit;
  }
  return lane;
}

// Record slot of step m (steps below 2^31).
__device__ __forceinline__ int64_t rec_slot(int64_t m) { return (int64_t)((uint32_t)m % (uint32_t)kRecSlots); }

// Part of the AT sum of step m = n + ahead (delay kd >= 1) over the levels
// m - kd - j that precede step n, j = q-1 down to 0, oldest first, one
// explicit FMA per level; rb is the ring of one (boundary, stage), slot_n =
// n mod depth.  The loads are unrolled over kMaxQ and issue together.
// Its two halves: the loads (issued together, so that a caller can issue
// other loads before it waits for these) and the sum.
struct AtLevels {
  double c[kMaxQ], v[kMaxQ];
  bool use[kMaxQ];
};

__device__ __forceinline__ void at_old_levels_load(const DevProblem& P, const double* __restrict__ rb, int ahead,
                                                   int kd, int slot_n, int depth, AtLevels& L) {
#pragma unroll
  for (int j = 0; j < kMaxQ; ++j) {
    const int back = kd + j - ahead;  // level n - back
    L.use[j] = kd > 0 && j < P.q && back >= 1;
    L.c[j] = 0.0;
    L.v[j] = 0.0;
    if (L.use[j]) {
      L.c[j] = P.atc[kd][j];
      L.v[j] = rb[ring_slot(slot_n, back, depth)];
    }
  }
}

__device__ __forceinline__ double at_old_levels_sum(const AtLevels& L) {
#pragma clang fp contract(off)
  double acc = 0.0;
#pragma unroll
  for (int j = kMaxQ - 1; j >= 0; --j)
    if (L.use[j]) acc = fma(L.c[j], L.v[j], acc);
  return acc;
}

__device__ __forceinline__ double at_old_levels(const DevProblem& P, const double* __restrict__ rb, int ahead,
                                                int kd, int slot_n, int depth) {
  AtLevels L;
  at_old_levels_load(P, rb, ahead, kd, slot_n, depth, L);
  return at_old_levels_sum(L);
}


// --------------------------------------------------------------- adjoint ---
// Butcher form of a 2N scheme: U_s = U + dt sum_{j<=s} beta_{s,j} K_j with
// beta_{s,j} = sum_{l=j..s} B_l prod_{m=j+1..l} A_m (K_j the operator at
// U_{j-1}); stage s + 1 reads U_s, so a_{s+1,j} = beta_{s,j}, b_j =
// beta_{S-1,j}.  Evaluated in double at compile time.
__host__ __device__ constexpr double ls_beta(int rk, int s, int j) {
  double acc = 0.0, prod = 1.0;
  for (int l = j; l <= s; ++l) {
    if (l > j) prod *= ls_a(rk, l);
    acc += ls_b(rk, l) * prod;
  }
  return acc;
}

// Butcher form of the integrators (the same maps as the forward algebraic
// forms): Y_i = U + dt sum_{j<i} a_ij K_j, U' = U + dt sum_i b_i K_i.
template <int RK>
__device__ constexpr double bt_a(int i, int j) {
  if constexpr (RK == RK_LS3)  // Williamson's scheme in Butcher form: a21 = 1/3, a31 = -3/16, a32 = 15/16
    return i == 1 ? (j == 0 ? 1.0 / 3.0 : 0.0) : (i == 2 && j < 2 ? (j == 0 ? -3.0 / 16.0 : 15.0 / 16.0) : 0.0);
  if constexpr (RK == RK_LS4) return j < i ? ls_beta(RK, i - 1, j) : 0.0;
  if constexpr (RK == RK_RK4) return (j == i - 1) ? (i == 3 ? 1.0 : 0.5) : 0.0;
  else if constexpr (RK == RK_SSP3) return i == 1 ? (j == 0 ? 1.0 : 0.0) : (i == 2 && j < 2 ? 0.25 : 0.0);
  else return (i == 1 && j == 0) ? 1.0 : 0.0;
}
template <int RK>
__device__ constexpr double bt_b(int i) {
  if constexpr (RK == RK_LS3) return i == 0 ? 1.0 / 6.0 : (i == 1 ? 3.0 / 10.0 : 8.0 / 15.0);
  if constexpr (RK == RK_LS4) return ls_beta(RK, rk_stages(RK) - 1, i);
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

}  // namespace adg
