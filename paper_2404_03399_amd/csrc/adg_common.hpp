// Shared host/device definitions of the ADG library (not part of the ABI).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace adg {

constexpr int kMaxNp = 5;     // degree <= 4
constexpr int kMaxL = 8;      // delays 0..7
constexpr int kMaxQ = 5;      // AT levels
constexpr int kBlock = 256;   // threads per workgroup (4 wave64)
constexpr int kRecSlots = 4;  // fused kernel PE-face record slots, indexed by step mod 4

// PHYS_ADV_UPWIND_POS: upwind advection with a > 0 in the fused kernel, which
// folds the right-face flux a u_p into the volume operator.
enum Phys : int {
  PHYS_ADV_UPWIND = 0, PHYS_ADV_CENTRAL = 1, PHYS_BURGERS_LLF = 2, PHYS_ADV_UPWIND_POS = 3, PHYS_BURGERS_LDG = 4
};
enum Rk : int { RK_HEUN = 0, RK_SSP3 = 1, RK_RK4 = 2, RK_LS3 = 3, RK_LS4 = 4 };
enum Scheme : int { SCH_DG = 0, SCH_ADG = 1, SCH_AT = 2 };

__host__ __device__ constexpr int rk_stages(int rk) {
  return rk == RK_HEUN ? 2 : (rk == RK_RK4 ? 4 : (rk == RK_LS4 ? 5 : 3));
}
constexpr int kMaxStages = 5;

// Packed delays of one PE face and step in the fused kernel's records: byte s
// holds the clamped delay of stage s (delays < kMaxL <= 255), so that the
// record jobs of different stages write different bytes of one word.
using RecWord = uint64_t;
static_assert(kMaxStages <= (int)sizeof(RecWord), "one byte per stage");

// Division by a run-time invariant 0 < d < 2^31 for dividends n < 2^31 by
// multiplication (Granlund & Montgomery, PLDI 1994): with l = ceil(log2 d),
// m = floor(2^(31+l) / d) + 1 and s = 31 + l, q = (n * m) >> s is exact
// because the rounding excess n (m - 2^s/d) / 2^s < 2^-l <= 1/d.
struct FastDiv {
  uint32_t d;
  uint32_t m;
  uint32_t s;
  uint32_t pad;
};

__host__ __device__ inline uint32_t fast_div(uint32_t n, const FastDiv& f) {
  return (uint32_t)(((uint64_t)n * (uint64_t)f.m) >> f.s);
}

inline FastDiv make_fast_div(uint32_t d) {
  uint32_t l = 0;
  while ((1ull << l) < d) ++l;
  FastDiv f;
  f.d = d;
  f.m = (uint32_t)(((1ull << (31 + l)) / d) + 1ull);
  f.s = 31 + l;
  f.pad = 0;
  return f;
}

// Per-problem descriptor, resident in the device workspace and read with
// uniform (scalar) loads by every workgroup of that problem.
struct DevProblem {
  int64_t n_elem;        // N_E
  int64_t pe_size;       // elements per PE
  int64_t n_pe;          // P (1: no PE faces)
  int64_t ld;            // plane stride of the state
  int64_t u_off;         // offset of the problem in the state vector
  int64_t ring_off;      // offset of the problem's delay ring (doubles)
  int64_t ring2_off;     // local DG: offset of the u-hat ring (same shape as the flux ring)
  int64_t at_off;        // offset of the problem's AT sums ([kRecSlots][P][S] doubles)
  int64_t atk_off;       // offset of the problem's delays ([kRecSlots][P] RecWords, byte s = stage s)
  int32_t np;            // degree + 1
  int32_t q;             // AT levels (1 for ADG)
  int32_t n_delays;      // L
  int32_t depth;         // ring slots per (boundary, stage): L + q, or the recorded steps + L + q
  int32_t per_stage;     // delay key includes the stage
  int32_t scheme;        // Scheme
  int32_t async_faces;   // 1 if PE faces use delayed data (scheme != DG and P > 1)
  int32_t caa;           // delays follow the communication-avoiding cycle
  FastDiv pe_div;        // division by pe_size
  uint64_t seed;
  uint64_t thr[kMaxL - 1];
  double two_over_dx;
  double speed;
  double dt;
  double half_dx;
  double nu;             // viscosity (local DG)
  double D[kMaxNp * kMaxNp];   // M^-1 S, row major
  double lift_l[kMaxNp];       // M^-1 phi(-1)
  double lift_r[kMaxNp];       // M^-1 phi(+1)
  double wq[kMaxNp];           // M 1 (quadrature weights)
  // Element operator with the metric (2/dx) and the flux constant folded in:
  //   (2/dx) (D f(y) + l_l fl - l_r fr) = Kd g(y) + Kl fl - Kr fr,
  // g(y) = y, Kd = (2/dx) a D for advection; g(y) = y^2, Kd = (2/dx) D / 2 for
  // Burgers; Kl = (2/dx) l_l, Kr = (2/dx) l_r.
  double Kd[kMaxNp * kMaxNp];
  double Kl[kMaxNp];
  double Kr[kMaxNp];
  // Kd with the interior upwind right-face term folded in (a > 0):
  // Kdu[i][p] = Kd[i][p] - Kr[i] a, so Kd y - Kr (a y_p) = Kdu y.
  double Kdu[kMaxNp * kMaxNp];
  FastDiv depth_div;     // division by the ring depth (step indices < 2^31)
  double atc[kMaxL][kMaxQ];    // c_j(k), j < q, k < L
};

struct WorkItem {
  int32_t prob;
  int32_t tile;
};

// SplitMix64 output function for state x (Steele, Lea & Flood 2014; the
// variant-13 finaliser of the public-domain reference generator).
__host__ __device__ inline uint64_t splitmix64(uint64_t x) {
  uint64_t z = x + 0x9E3779B97F4A7C15ull;
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}

// The delay hash chains SplitMix64 over (seed, step, stage key, boundary):
// h = mix(mix(mix(mix(seed) ^ step) ^ key) ^ boundary).  The first three
// links do not depend on the boundary.
__host__ __device__ inline uint64_t delay_prefix(uint64_t seed, int64_t step, int32_t key) {
  uint64_t h = splitmix64(seed);
  h = splitmix64(h ^ (uint64_t)step);
  return splitmix64(h ^ (uint64_t)(int64_t)key);
}

// Delay before clamping: number of thresholds at or below the 53-bit
// uniform u = h >> 11.
__host__ __device__ inline int delay_from_prefix(uint64_t prefix, int64_t boundary, const uint64_t* thr,
                                                 int n_delays) {
  const uint64_t u = splitmix64(prefix ^ (uint64_t)boundary) >> 11;
  int k = 0;
  for (int i = 0; i < n_delays - 1; ++i) k += (u >= thr[i]) ? 1 : 0;
  return k;
}

__host__ __device__ inline int draw_delay(uint64_t seed, int64_t step, int32_t key, int64_t boundary,
                                          const uint64_t* thr, int n_delays) {
  return delay_from_prefix(delay_prefix(seed, step, key), boundary, thr, n_delays);
}

// Communication-avoiding schedule (Sec. 7): of every five steps the first two
// communicate with synchronisation and the next three do not, so the PE-face
// data are 0, 1 and 2 levels old: delays (0, 0, 0, 1, 2) at every face.
__host__ __device__ inline int caa_delay(int64_t step) {
  const int c = (int)(step % 5);
  return c < 3 ? 0 : c - 2;
}

// Usable delay: every level n-k-j, j < q, must exist.
__host__ __device__ inline int clamp_delay(int k, int64_t step, int q) {
  int64_t lim = step - q + 1;
  if (lim < 0) lim = 0;
  return (int64_t)k < lim ? k : (int)lim;
}

}  // namespace adg
