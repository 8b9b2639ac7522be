// Per-stage kernels (one launch per RK stage, RK registers in HBM), the
// statistics and counter kernels, and the dispatch of the fused step to its
// per-integrator translation units.
#include <algorithm>

#include "adg_device.hpp"

namespace adg {

// The absolute step index of a launch is ctr[0] + step_offset: launches of
// one batch (or one captured graph) carry offsets 0, 1, 2, ... and a single
// k_advance at the end of the batch adds the batch length to ctr[0].  No
// workgroup ever writes the counter while others read it.
__global__ void k_advance(int64_t* __restrict__ ctr, int64_t n_steps) {
  if (threadIdx.x == 0 && blockIdx.x == 0) ctr[0] = ctr[0] + n_steps;
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
                                           double* __restrict__ A, double* __restrict__ ring, int64_t n,
                                           const double* __restrict__ qb) {
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
  constexpr bool ldg = PHYS == PHYS_BURGERS_LDG;
  constexpr int PF = ldg ? PHYS_BURGERS_LLF : PHYS;  // the inviscid face flux
  double qv[NP];
  double fl, fr;
  if constexpr (ldg) {
    // total flux G = fhat_LLF(u-, u+) - nu q+ (q-hat from the right element)
#pragma unroll
    for (int j = 0; j < NP; ++j) qv[j] = qb[off + j * ld + e];
    fl = Physics<PF>::fhat(um, y[0], a) - P.nu * qv[0];
    fr = Physics<PF>::fhat(y[NP - 1], upr, a) - P.nu * qb[off + e1];
  } else {
    fl = Physics<PF>::fhat(um, y[0], a);
    fr = Physics<PF>::fhat(y[NP - 1], upr, a);
  }
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
  if constexpr (ldg) {
    // (2/dx)(D g + l_l G_left - l_r G_right), g = u^2/2 - nu q (Kd = (2/dx) D)
    double g[NP];
#pragma unroll
    for (int j = 0; j < NP; ++j) g[j] = 0.5 * y[j] * y[j] - P.nu * qv[j];
#pragma unroll
    for (int i = 0; i < NP; ++i) {
      double v = P.Kl[i] * fl - P.Kr[i] * fr;
#pragma unroll
      for (int j = 0; j < NP; ++j) v += P.Kd[i * kMaxNp + j] * g[j];
      k[i] = v;
    }
  } else {
    element_rhs<NP, PF>(Dm, ll, lr, P.two_over_dx, a, y, fl, fr, k);
  }

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
  } else if constexpr (low_storage(RK)) {
    // 2N-storage scheme, A = dU: dU = A_s dU + dt k, next = y + B_s dU
    constexpr double Acoef = ls_a(RK, SI);
    constexpr double Bcoef = ls_b(RK, SI);
#pragma unroll
    for (int j = 0; j < NP; ++j) {
      const int64_t i = j * ld + e;
      const double du = SI == 0 ? dt * k[j] : fma(Acoef, Ao[i], dt * k[j]);
      if constexpr (SI < S - 1) {
        Ao[i] = du;
        Yo[i] = fma(Bcoef, du, y[j]);
      } else {
        Uo[i] = fma(Bcoef, du, y[j]);
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
                                                  const int64_t* __restrict__ ctr, int32_t step_offset,
                                                  const double* __restrict__ qb) {
  const WorkItem wi = work[blockIdx.x];
  const DevProblem& P = probs[wi.prob];
  const int64_t n = ctr[0] + step_offset;
  switch (P.np) {
    case 2: stage_elem<2, RK, PHYS, SI>(P, wi.tile, yin, yout, U, A, ring, n, qb); break;
    case 3: stage_elem<3, RK, PHYS, SI>(P, wi.tile, yin, yout, U, A, ring, n, qb); break;
    case 4: stage_elem<4, RK, PHYS, SI>(P, wi.tile, yin, yout, U, A, ring, n, qb); break;
    default: stage_elem<5, RK, PHYS, SI>(P, wi.tile, yin, yout, U, A, ring, n, qb); break;
  }
}

// Local DG, first pass: q = (2/dx)(-D u + l_r u-hat_right - l_l u-hat_left)
// with u-hat from the left element (alternating flux).  At a PE face the
// element right of it writes the raw level-n u-hat to the u-hat ring and
// both neighbours take the AT combination of past levels when delayed.
template <int NP, int RK, int SI>
__device__ __forceinline__ void ldg_q_elem(const DevProblem& P, int tile, const double* __restrict__ yin,
                                           double* __restrict__ qout, double* __restrict__ ring, int64_t n) {
  constexpr int S = rk_stages(RK);
  const int N = (int)P.n_elem;
  const int e = tile * kBlock + (int)threadIdx.x;
  if (e >= N) return;
  const int64_t ld = P.ld, off = P.u_off;
  const int em = e == 0 ? N - 1 : e - 1;
  const int e1 = e + 1 == N ? 0 : e + 1;
  double y[NP];
#pragma unroll
  for (int j = 0; j < NP; ++j) y[j] = yin[off + j * ld + e];
  double hl = yin[off + (NP - 1) * ld + em];
  double hr = y[NP - 1];
  if (P.async_faces) {
    const uint32_t pes = P.pe_div.d;
    const int slot_n = (int)(n % (int64_t)P.depth);
    const uint32_t bl = fast_div((uint32_t)e, P.pe_div);
    if ((uint32_t)e == bl * pes) {
      const int64_t rb = P.ring2_off + ((int64_t)bl * S + SI) * P.depth;
      const int kd = pe_delay(P, n, SI, bl);
      ring[rb + slot_n] = hl;
      if (kd > 0) hl = at_past_sum(P, ring + rb, kd, slot_n);
    }
    const uint32_t br = fast_div((uint32_t)e1, P.pe_div);
    if ((uint32_t)e1 == br * pes) {
      const int kd = pe_delay(P, n, SI, br);
      if (kd > 0) hr = at_past_sum(P, ring + P.ring2_off + ((int64_t)br * S + SI) * P.depth, kd, slot_n);
    }
  }
#pragma unroll
  for (int i = 0; i < NP; ++i) {
    double v = P.Kr[i] * hr - P.Kl[i] * hl;
#pragma unroll
    for (int j = 0; j < NP; ++j) v -= P.Kd[i * kMaxNp + j] * y[j];
    qout[off + i * ld + e] = v;
  }
}

template <int RK, int SI>
__global__ __launch_bounds__(kBlock) void k_ldg_q(const DevProblem* __restrict__ probs,
                                                  const WorkItem* __restrict__ work, const double* __restrict__ yin,
                                                  double* __restrict__ qout, double* __restrict__ ring,
                                                  const int64_t* __restrict__ ctr, int32_t step_offset) {
  const WorkItem wi = work[blockIdx.x];
  const DevProblem& P = probs[wi.prob];
  const int64_t n = ctr[0] + step_offset;
  switch (P.np) {
    case 2: ldg_q_elem<2, RK, SI>(P, wi.tile, yin, qout, ring, n); break;
    case 3: ldg_q_elem<3, RK, SI>(P, wi.tile, yin, qout, ring, n); break;
    case 4: ldg_q_elem<4, RK, SI>(P, wi.tile, yin, qout, ring, n); break;
    default: ldg_q_elem<5, RK, SI>(P, wi.tile, yin, qout, ring, n); break;
  }
}

// ----------------------------------------------------------- statistics ---
// Maximum that propagates NaN (fmax drops it): a blown-up realization must
// report a non-finite max error, as a plain maximum over its values would.
__device__ __forceinline__ double max_nan(double a, double b) {
  return a != a ? a : (b != b ? b : fmax(a, b));
}

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
      mabs = max_nan(mabs, d);
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
      red[1][threadIdx.x] = max_nan(red[1][threadIdx.x], red[1][threadIdx.x + w]);
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
    s1 = max_nan(s1, part[3 * i + 1]);
    s2 += part[3 * i + 2];
  }
  red[0][threadIdx.x] = s0;
  red[1][threadIdx.x] = s1;
  red[2][threadIdx.x] = s2;
  __syncthreads();
  for (int w = kBlock / 2; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) {
      red[0][threadIdx.x] += red[0][threadIdx.x + w];
      red[1][threadIdx.x] = max_nan(red[1][threadIdx.x], red[1][threadIdx.x + w]);
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
template <int RK, int PHYS, int SI>
static void stage_go(const StepArgs& a, const double* yin, double* yout, double* U, double* A, int32_t off,
                     hipStream_t st) {
  hipLaunchKernelGGL((k_stage<RK, PHYS, SI>), dim3(a.n_work), dim3(kBlock), 0, st, a.probs, a.work, yin, yout, U, A,
                     a.ring, a.ctr, off, a.qbuf);
}

template <int RK>
static void ldg_q_si(int si, const StepArgs& a, const double* yin, int32_t off, hipStream_t st) {
  const dim3 g(a.n_work), b(kBlock);
  switch (si) {
    case 0: hipLaunchKernelGGL((k_ldg_q<RK, 0>), g, b, 0, st, a.probs, a.work, yin, a.qbuf, a.ring, a.ctr, off); break;
    case 1: hipLaunchKernelGGL((k_ldg_q<RK, 1>), g, b, 0, st, a.probs, a.work, yin, a.qbuf, a.ring, a.ctr, off); break;
    case 2:
      if constexpr (rk_stages(RK) > 2)
        hipLaunchKernelGGL((k_ldg_q<RK, 2>), g, b, 0, st, a.probs, a.work, yin, a.qbuf, a.ring, a.ctr, off);
      break;
    case 3:
      if constexpr (rk_stages(RK) > 3)
        hipLaunchKernelGGL((k_ldg_q<RK, 3>), g, b, 0, st, a.probs, a.work, yin, a.qbuf, a.ring, a.ctr, off);
      break;
    default:
      if constexpr (rk_stages(RK) > 4)
        hipLaunchKernelGGL((k_ldg_q<RK, 4>), g, b, 0, st, a.probs, a.work, yin, a.qbuf, a.ring, a.ctr, off);
      break;
  }
}

hipError_t launch_ldg_q(int rk, int stage, const StepArgs& a, const double* yin, int32_t step_offset,
                        hipStream_t stream) {
  switch (rk) {
    case RK_HEUN: ldg_q_si<RK_HEUN>(stage, a, yin, step_offset, stream); break;
    case RK_SSP3: ldg_q_si<RK_SSP3>(stage, a, yin, step_offset, stream); break;
    case RK_LS3: ldg_q_si<RK_LS3>(stage, a, yin, step_offset, stream); break;
    case RK_LS4: ldg_q_si<RK_LS4>(stage, a, yin, step_offset, stream); break;
    default: ldg_q_si<RK_RK4>(stage, a, yin, step_offset, stream); break;
  }
  return hipGetLastError();
}

template <int RK, int PHYS>
static void stage_si(int si, const StepArgs& a, const double* yin, double* yout, double* U, double* A, int32_t off,
                     hipStream_t st) {
  switch (si) {
    case 0: stage_go<RK, PHYS, 0>(a, yin, yout, U, A, off, st); break;
    case 1: stage_go<RK, PHYS, 1>(a, yin, yout, U, A, off, st); break;
    case 2: if constexpr (rk_stages(RK) > 2) stage_go<RK, PHYS, 2>(a, yin, yout, U, A, off, st); break;
    case 3: if constexpr (rk_stages(RK) > 3) stage_go<RK, PHYS, 3>(a, yin, yout, U, A, off, st); break;
    default: if constexpr (rk_stages(RK) > 4) stage_go<RK, PHYS, 4>(a, yin, yout, U, A, off, st); break;
  }
}

template <int RK>
static void stage_phys(int phys, int si, const StepArgs& a, const double* yin, double* yout, double* U, double* A,
                       int32_t off, hipStream_t st) {
  switch (phys) {
    case PHYS_ADV_UPWIND: stage_si<RK, PHYS_ADV_UPWIND>(si, a, yin, yout, U, A, off, st); break;
    case PHYS_ADV_CENTRAL: stage_si<RK, PHYS_ADV_CENTRAL>(si, a, yin, yout, U, A, off, st); break;
    case PHYS_BURGERS_LDG: stage_si<RK, PHYS_BURGERS_LDG>(si, a, yin, yout, U, A, off, st); break;
    default: stage_si<RK, PHYS_BURGERS_LLF>(si, a, yin, yout, U, A, off, st); break;
  }
}

hipError_t launch_fused_step(int rk, int phys, const StepArgs& a, const double* uin, double* uout, int32_t step_offset,
                             hipStream_t stream) {
  switch (rk) {
    case RK_HEUN: return launch_fused_rk<RK_HEUN>(phys, a, uin, uout, step_offset, stream);
    case RK_SSP3: return launch_fused_rk<RK_SSP3>(phys, a, uin, uout, step_offset, stream);
    case RK_LS3: return launch_fused_rk<RK_LS3>(phys, a, uin, uout, step_offset, stream);
    case RK_LS4: return launch_fused_rk<RK_LS4>(phys, a, uin, uout, step_offset, stream);
    default: return launch_fused_rk<RK_RK4>(phys, a, uin, uout, step_offset, stream);
  }
}

hipError_t launch_stage(int rk, int phys, int stage, const StepArgs& a, const double* yin, double* yout, double* U,
                        double* A, int32_t step_offset, hipStream_t stream) {
  switch (rk) {
    case RK_HEUN: stage_phys<RK_HEUN>(phys, stage, a, yin, yout, U, A, step_offset, stream); break;
    case RK_SSP3: stage_phys<RK_SSP3>(phys, stage, a, yin, yout, U, A, step_offset, stream); break;
    case RK_LS3: stage_phys<RK_LS3>(phys, stage, a, yin, yout, U, A, step_offset, stream); break;
    case RK_LS4: stage_phys<RK_LS4>(phys, stage, a, yin, yout, U, A, step_offset, stream); break;
    default: stage_phys<RK_RK4>(phys, stage, a, yin, yout, U, A, step_offset, stream); break;
  }
  return hipGetLastError();
}

// Zero fill of n 8-byte words (grid-stride): the library clears counters,
// rings and accumulators with a kernel rather than a memset node, so that
// a caller's graph capture of its calls records only kernels.
__global__ __launch_bounds__(kBlock) void k_zero(uint64_t* __restrict__ p, int64_t n) {
  const int64_t stride = (int64_t)gridDim.x * kBlock;
  for (int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x; i < n; i += stride) p[i] = 0;
}

hipError_t launch_zero(void* p, int64_t bytes, hipStream_t stream) {
  if (bytes <= 0) return hipSuccess;
  if (((uintptr_t)p & 7u) != 0 || (bytes & 7) != 0) return hipErrorInvalidValue;
  const int64_t n = bytes / 8;
  const int64_t blocks = std::min<int64_t>((n + kBlock - 1) / kBlock, 2048);
  hipLaunchKernelGGL(k_zero, dim3((unsigned)blocks), dim3(kBlock), 0, stream, (uint64_t*)p, n);
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
