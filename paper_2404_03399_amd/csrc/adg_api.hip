// C ABI of the ADG library: validation, reference operators, AT table,
// workspace layout, launch sequencing and hipGraph replay.
#include <algorithm>
#include <cmath>
#include <cstring>
#include <mutex>
#include <string>
#include <vector>

#include "adg.h"
#include "adg_launch.hpp"

using namespace adg;

namespace {

thread_local std::string g_err;

int fail(int code, const std::string& msg) {
  g_err = msg;
  return code;
}

// State vectors are read and written as 16-byte pairs of nodal values.
bool state_aligned(const void* p) { return ((uintptr_t)p & 15u) == 0; }

#define ADG_HIP(expr)                                                                         \
  do {                                                                                        \
    hipError_t e_ = (expr);                                                                   \
    if (e_ != hipSuccess) return fail(ADG_E_HIP, std::string(#expr) + ": " + hipGetErrorString(e_)); \
  } while (0)

constexpr int64_t kAlign = 256;
int64_t align_up(int64_t x, int64_t a) { return (x + a - 1) / a * a; }

// ------------------------------------------------ reference element (host) --
// Legendre P_p and P_p' at x by the three-term recurrence.
void legendre(int p, long double x, long double* P, long double* dP) {
  long double p0 = 1.0L, p1 = x;
  if (p == 0) { *P = 1.0L; *dP = 0.0L; return; }
  for (int k = 1; k < p; ++k) {
    const long double p2 = ((2 * k + 1) * x * p1 - k * p0) / (k + 1);
    p0 = p1;
    p1 = p2;
  }
  *P = p1;
  *dP = p * (x * p1 - p0) / (x * x - 1.0L);  // valid for |x| < 1
}

// Gauss-Lobatto-Legendre nodes: -1, roots of P_p' (Newton from the
// Chebyshev-Lobatto points), +1.
void gll(int p, long double* x) {
  x[0] = -1.0L;
  x[p] = 1.0L;
  for (int i = 1; i < p; ++i) {
    long double z = -std::cos(3.14159265358979323846264338327950288L * i / p);
    for (int it = 0; it < 100; ++it) {
      long double P, dP;
      legendre(p, z, &P, &dP);
      // (1 - z^2) P'' = 2 z P' - p (p + 1) P
      const long double d2P = (2.0L * z * dP - p * (p + 1) * P) / (1.0L - z * z);
      const long double step = dP / d2P;
      z -= step;
      if (std::fabs(step) < 1e-30L) break;
    }
    x[i] = z;
  }
  std::sort(x, x + p + 1);
}

// Monomial coefficients c[j][m] of the Lagrange cardinal polynomials.
void lagrange_monomials(int p, const long double* x, long double c[kMaxNp][kMaxNp]) {
  for (int j = 0; j <= p; ++j) {
    long double poly[kMaxNp] = {1.0L};
    int deg = 0;
    for (int m = 0; m <= p; ++m) {
      if (m == j) continue;
      const long double inv = 1.0L / (x[j] - x[m]);
      long double nxt[kMaxNp] = {0};
      for (int d = 0; d <= deg; ++d) {
        nxt[d + 1] += poly[d] * inv;
        nxt[d] -= poly[d] * x[m] * inv;
      }
      ++deg;
      std::memcpy(poly, nxt, sizeof(poly));
    }
    for (int m = 0; m <= p; ++m) c[j][m] = poly[m];
  }
}

long double mono_int(int k) { return (k % 2) ? 0.0L : 2.0L / (k + 1); }  // int_{-1}^{1} xi^k

// Solve A X = B (n x n, m right-hand sides) by Gaussian elimination with
// partial pivoting, in place (B becomes X).
void solve(int n, int m, long double A[kMaxNp][kMaxNp], long double B[kMaxNp][kMaxNp + 2]) {
  for (int c = 0; c < n; ++c) {
    int piv = c;
    for (int r = c + 1; r < n; ++r)
      if (std::fabs(A[r][c]) > std::fabs(A[piv][c])) piv = r;
    for (int k = 0; k < n; ++k) std::swap(A[c][k], A[piv][k]);
    for (int k = 0; k < m; ++k) std::swap(B[c][k], B[piv][k]);
    for (int r = 0; r < n; ++r) {
      if (r == c) continue;
      const long double f = A[r][c] / A[c][c];
      for (int k = 0; k < n; ++k) A[r][k] -= f * A[c][k];
      for (int k = 0; k < m; ++k) B[r][k] -= f * B[c][k];
    }
  }
  for (int r = 0; r < n; ++r)
    for (int k = 0; k < m; ++k) B[r][k] /= A[r][r];
}

// D = M^-1 S, lift_l = M^-1 e_0, lift_r = M^-1 e_p, w = M 1; M and S integrated
// exactly on monomials: M_ij = int phi_i phi_j, S_ij = int phi_j phi_i'.
void element_operators(int p, DevProblem* dp) {
  const int np = p + 1;
  long double x[kMaxNp], c[kMaxNp][kMaxNp];
  gll(p, x);
  lagrange_monomials(p, x, c);
  long double M[kMaxNp][kMaxNp] = {}, RHS[kMaxNp][kMaxNp + 2] = {};
  for (int i = 0; i < np; ++i)
    for (int j = 0; j < np; ++j) {
      long double m = 0.0L, s = 0.0L;
      for (int a = 0; a < np; ++a)
        for (int b = 0; b < np; ++b) {
          m += c[i][a] * c[j][b] * mono_int(a + b);
          if (b >= 1) s += c[j][a] * (b * c[i][b]) * mono_int(a + b - 1);
        }
      M[i][j] = m;
      RHS[i][j] = s;
    }
  long double w[kMaxNp] = {};
  for (int i = 0; i < np; ++i)
    for (int j = 0; j < np; ++j) w[i] += M[i][j];
  RHS[0][np] = 1.0L;       // e_0
  RHS[p][np + 1] = 1.0L;   // e_p
  solve(np, np + 2, M, RHS);
  for (int i = 0; i < kMaxNp * kMaxNp; ++i) dp->D[i] = 0.0;
  for (int i = 0; i < np; ++i) {
    for (int j = 0; j < np; ++j) dp->D[i * kMaxNp + j] = (double)RHS[i][j];
    dp->lift_l[i] = (double)RHS[i][np];
    dp->lift_r[i] = (double)RHS[i][np + 1];
    dp->wq[i] = (double)w[i];
  }
}

// AT coefficients in closed form: the moment conditions of the AT flux make
// c_j(k) the Lagrange weights extrapolating levels -(k+j) to 0:
// c_j(k) = prod_{m != j} (k + m) / (m - j)  (integers).
double at_coefficient(int q, int k, int j) {
  long long num = 1, den = 1;
  for (int m = 0; m < q; ++m) {
    if (m == j) continue;
    num *= (long long)(k + m);
    den *= (long long)(m - j);
  }
  return (double)(num / den);
}

int phys_of(const adg_problem& p) {
  if (p.equation == ADG_EQ_BURGERS) return PHYS_BURGERS_LLF;
  if (p.equation == ADG_EQ_VISCOUS_BURGERS) return PHYS_BURGERS_LDG;
  return p.flux == ADG_FLUX_CENTRAL ? PHYS_ADV_CENTRAL : PHYS_ADV_UPWIND;
}

int q_of(const adg_problem& p) {
  if (p.scheme != ADG_SCHEME_ADG_AT) return 1;
  return p.at_levels ? (int)p.at_levels : (int)p.degree + 1;
}

int64_t ld_of(const adg_problem& p) { return align_up(p.n_elem, 64); }

bool async_of(const adg_problem& p) { return p.scheme != ADG_SCHEME_DG && p.n_elem / p.pe_size > 1; }

int validate_one(const adg_problem& p, int idx) {
  const std::string at = "problem " + std::to_string(idx) + ": ";
  if (p.abi_version != ADG_ABI_VERSION) return fail(ADG_E_ABI, at + "abi_version mismatch");
  if (p.equation > ADG_EQ_VISCOUS_BURGERS) return fail(ADG_E_INVALID, at + "unknown equation");
  if (p.equation == ADG_EQ_VISCOUS_BURGERS && (p.flux != ADG_FLUX_LLF || !(p.viscosity >= 0.0) ||
                                               !std::isfinite(p.viscosity)))
    return fail(ADG_E_INVALID, at + "viscous Burgers needs the llf flux and a finite viscosity >= 0");
  if (p.equation != ADG_EQ_VISCOUS_BURGERS && p.viscosity != 0.0)
    return fail(ADG_E_INVALID, at + "viscosity is only for viscous Burgers");
  if (p.scheme > ADG_SCHEME_ADG_AT) return fail(ADG_E_INVALID, at + "unknown scheme");
  if (p.flux > ADG_FLUX_LLF) return fail(ADG_E_INVALID, at + "unknown flux");
  if (p.rk > ADG_LSRK4) return fail(ADG_E_INVALID, at + "unknown rk");
  if (p.degree < 1 || p.degree > 4) return fail(ADG_E_INVALID, at + "degree must be in 1..4");
  if (p.equation == ADG_EQ_ADVECTION && p.flux == ADG_FLUX_LLF)
    return fail(ADG_E_INVALID, at + "llf flux is for Burgers");
  if (p.equation == ADG_EQ_BURGERS && p.flux != ADG_FLUX_LLF)
    return fail(ADG_E_INVALID, at + "Burgers needs the llf flux");
  if (p.at_levels != 0 && p.scheme != ADG_SCHEME_ADG_AT)
    return fail(ADG_E_INVALID, at + "at_levels is only for ADG-AT");
  if (p.at_levels > (uint32_t)kMaxQ) return fail(ADG_E_INVALID, at + "at_levels must be <= 5");
  if (p.scheme == ADG_SCHEME_ADG_AT && p.at_levels == 0 && p.degree + 1 > (uint32_t)kMaxQ)
    return fail(ADG_E_INVALID, at + "q = degree + 1 exceeds 5");
  if (p.n_delays < 1 || p.n_delays > (uint32_t)kMaxL) return fail(ADG_E_INVALID, at + "n_delays must be in 1..8");
  if (p.delay_granularity > ADG_DELAY_CAA) return fail(ADG_E_INVALID, at + "bad delay_granularity");
  if (p.delay_granularity == ADG_DELAY_CAA && p.n_delays != 3)
    return fail(ADG_E_INVALID, at + "the communication-avoiding cycle needs n_delays = 3");
  if (p.reserved != 0) return fail(ADG_E_INVALID, at + "reserved must be 0");
  if (p.n_elem < 2 || p.n_elem > (int64_t)1 << 30) return fail(ADG_E_INVALID, at + "n_elem must be in 2..2^30");
  if (p.pe_size < 1 || p.n_elem % p.pe_size != 0) return fail(ADG_E_INVALID, at + "pe_size must divide n_elem");
  for (uint32_t i = 0; i + 1 < p.n_delays; ++i) {
    if (p.delay_threshold[i] > (1ull << 53)) return fail(ADG_E_INVALID, at + "threshold > 2^53");
    if (i > 0 && p.delay_threshold[i] < p.delay_threshold[i - 1])
      return fail(ADG_E_INVALID, at + "thresholds must be non-decreasing");
  }
  if (!(p.length > 0.0) || !std::isfinite(p.length)) return fail(ADG_E_INVALID, at + "length must be > 0");
  if (!(p.dt > 0.0) || !std::isfinite(p.dt)) return fail(ADG_E_INVALID, at + "dt must be > 0");
  if (!std::isfinite(p.x_left)) return fail(ADG_E_INVALID, at + "x_left must be finite");
  if (p.equation == ADG_EQ_ADVECTION && (!(p.speed != 0.0) || !std::isfinite(p.speed)))
    return fail(ADG_E_INVALID, at + "speed must be finite and non-zero");
  return ADG_OK;
}

int validate(const adg_problem* probs, int32_t n) {
  if (!probs || n < 1) return fail(ADG_E_INVALID, "need at least one problem");
  for (int32_t i = 0; i < n; ++i) {
    const int rc = validate_one(probs[i], i);
    if (rc) return rc;
  }
  for (int32_t i = 1; i < n; ++i) {
    const adg_problem &a = probs[0], &b = probs[i];
    if (a.equation != b.equation || a.flux != b.flux || a.rk != b.rk || a.scheme != b.scheme)
      return fail(ADG_E_INVALID, "all problems of a context must share equation, flux, rk and scheme");
  }
  return ADG_OK;
}

struct Layout {
  int64_t probs, work_f, work_f2, work_s, first_s, ctr, ring, atsum, atk, state2, y0, y1, acc, qbuf, part, stats_out;
  int64_t groups, gstats;  // ensemble statistics: group CSR (2n+1 int32) and 4 doubles per group
  // adjoint recording (-1 if not recording); ckrec holds the fused kernel's
  // PE-face records (AT sums, delays) at every checkpoint plus one spare slot
  int64_t ckpt, useg, ybuf, lam, q, adjring, cpart, ckrec, work_a, work_a2;
  int64_t total;
  int32_t n_work_f, n_work_f2, n_work_s, n_work_a, n_work_a2;
  int64_t rec_atsum_bytes, rec_atk_bytes, rec_bytes;
  int64_t total_doubles;
  int64_t ring_doubles;
  int64_t at_entries;  // boundaries x kRecSlots (x S for the sums)
  int64_t n_rec, ckpt_every, n_ckpt;
};

// Ring slots per (boundary, stage): the AT window L + q - 1 plus one, or,
// when an adjoint recording horizon is given, the whole run (every level is
// kept).  A two-step launch writes levels n and n + 1 while waves that start
// later still read levels down to n + 2 - L - q (the local DG kernel's halo
// waves read the ring at their start); with L + q slots level n + 1 never
// shares a slot with a level the launch reads.
int64_t depth_of(const adg_problem& p, int64_t n_rec) {
  return n_rec > 0 ? n_rec + p.n_delays + q_of(p) : (int64_t)p.n_delays + q_of(p);
}

// Elements per lane of the fused kernel (0 if the request is invalid).
int lane_elems_of(const adg_problem* probs, int32_t n, const adg_options* opt) {
  int64_t min_pes = (int64_t)1 << 62;
  for (int32_t i = 0; i < n; ++i)
    if (async_of(probs[i])) min_pes = std::min(min_pes, probs[i].pe_size);
  const int req = opt ? opt->lane_elems : 0;
  if (req == 0) return min_pes < 2 ? 1 : 2;
  if (req != 1 && req != 2 && req != 4) return 0;
  return req <= min_pes ? req : 0;
}

// Time steps per fused launch (0 if the request is invalid).
int fused_steps_of(const adg_options* opt) {
  const int req = opt ? (int)opt->fused_steps : 0;
  if (req == 0) return 2;
  return (req == 1 || req == 2) ? req : 0;
}

// Kernel family: AUTO picks the fused kernel.
int kernel_of(const adg_problem*, const adg_options* opt) {
  if (!opt || opt->kernel == ADG_KERNEL_AUTO) return ADG_KERNEL_FUSED;
  return opt->kernel;
}

bool is_ldg(const adg_problem* probs) { return probs[0].equation == ADG_EQ_VISCOUS_BURGERS; }

// PE-face split of the fused kernel (fused_mode): tile waves with every
// PE-face path compiled out and window waves centred on the PE faces, in one
// launch.  Every asynchronous problem's PE size must hold one window of the
// longest launch (one face per window).  By default the split is used only
// where a wave holds at least two windows and every PE size holds four: the
// windows' extra work then stays below what the lighter tile waves save
// (measured on 2^20 and 2^24 elements: 10-11 % faster per step at PE size
// 256 with RK4 and two steps per launch, 7 % slower at PE size 64, and
// slower for the five-stage scheme, whose 40-element window fills a wave).
bool pe_split_of(const adg_problem* probs, int32_t n, const adg_options* opt) {
  const uint32_t f = opt ? opt->flags : 0u;
  if ((f & (ADG_OPT_PE_SPLIT_OFF | ADG_OPT_ONE_LAUNCH)) || kernel_of(probs, opt) != ADG_KERNEL_FUSED || is_ldg(probs))
    return false;
  const int K = fused_steps_of(opt) == 1 ? 1 : 2;
  const bool force = (f & ADG_OPT_PE_SPLIT_ON) != 0;
  if (!force && fused_windows_per_wave((int)probs[0].rk, K) < 2) return false;
  const int64_t need = (int64_t)fused_window((int)probs[0].rk, K) * (force ? 1 : 4);
  bool any = false;
  for (int32_t i = 0; i < n; ++i) {
    if (!async_of(probs[i])) continue;
    any = true;
    if (probs[i].pe_size < need) return false;
  }
  return any;
}
// linear advection can reverse two steps per launch (no forward stages needed)
bool adj_two_steps(const adg_problem* probs) { return probs[0].equation == ADG_EQ_ADVECTION; }
// elements per lane of the two-step reverse: the forward's, at most 2 (its
// reverse stages keep R sets of Butcher accumulators in registers)
int adj_lane_elems(int lane_elems) { return lane_elems >= 2 ? 2 : 1; }

Layout make_layout(const adg_problem* probs, int32_t n, const adg_options* opt, int64_t n_rec) {
  Layout L{};
  const int S = rk_stages((int)probs[0].rk);
  const int R = std::max(1, lane_elems_of(probs, n, opt));
  const int T = fused_tile((int)probs[0].rk, R, 1);
  const int T2 = fused_tile((int)probs[0].rk, R, 2);
  const int T1 = adj_tile_elems((int)probs[0].rk, probs[0].equation == ADG_EQ_BURGERS);
  const int TA2 = adj_tile_elems2((int)probs[0].rk, adj_lane_elems(R));
  int64_t nwf = 0, nwf2 = 0, nws = 0, nwa = 0, nwa2 = 0, tot = 0, ring = 0, at = 0, nww[2] = {0, 0};
  const bool split = pe_split_of(probs, n, opt);
  for (int32_t i = 0; i < n; ++i) {
    const adg_problem& p = probs[i];
    nwf += (p.n_elem + T - 1) / T;
    nwf2 += (p.n_elem + T2 - 1) / T2;
    nwa += (p.n_elem + T1 - 1) / T1;
    nwa2 += (p.n_elem + TA2 - 1) / TA2;
    nws += (p.n_elem + kBlock - 1) / kBlock;
    tot += ld_of(p) * (p.degree + 1);
    if (split && async_of(p))  // window items of the PE-face split, in the same lists
      for (int K = 1; K <= 2; ++K) {
        const int64_t fw = fused_windows_per_wave((int)p.rk, K);
        nww[K - 1] += (p.n_elem / p.pe_size + fw - 1) / fw;
      }
    if (async_of(p)) {
      // local DG keeps a second ring of the same shape for u-hat
      ring += (is_ldg(probs) ? 2 : 1) * (p.n_elem / p.pe_size) * S * depth_of(p, n_rec);
      at += kRecSlots * (p.n_elem / p.pe_size);
    }
  }
  L.at_entries = at;
  L.n_work_f = (int32_t)(nwf + nww[0]);
  L.n_work_f2 = (int32_t)(nwf2 + nww[1]);
  L.n_work_s = (int32_t)nws;
  L.n_work_a = n_rec > 0 ? (int32_t)nwa : 0;
  L.n_work_a2 = n_rec > 0 && adj_two_steps(probs) ? (int32_t)nwa2 : 0;
  L.total_doubles = tot;
  L.ring_doubles = ring;
  const int kern = kernel_of(probs, opt);
  int64_t off = 0;
  auto take = [&](int64_t bytes) { const int64_t o = off; off = align_up(off + bytes, kAlign); return o; };
  L.probs = take((int64_t)sizeof(DevProblem) * n);
  L.work_f = take((int64_t)sizeof(WorkItem) * L.n_work_f);
  L.work_f2 = take((int64_t)sizeof(WorkItem) * L.n_work_f2);
  L.work_s = take((int64_t)sizeof(WorkItem) * nws);
  L.first_s = take((int64_t)sizeof(int32_t) * (n + 1));
  L.ctr = take(8 * sizeof(int64_t));
  L.ring = take(8 * std::max<int64_t>(ring, 1));
  L.atsum = take(8 * S * std::max<int64_t>(at, 1));
  L.atk = take((int64_t)sizeof(RecWord) * std::max<int64_t>(at, 1));
  const bool rec = n_rec > 0;
  L.state2 = kern == ADG_KERNEL_FUSED ? take(8 * tot) : -1;
  L.y0 = kern == ADG_KERNEL_STAGE ? take(8 * tot) : -1;
  L.y1 = kern == ADG_KERNEL_STAGE ? take(8 * tot) : -1;
  L.acc = kern == ADG_KERNEL_STAGE ? take(8 * tot) : -1;
  L.qbuf = (is_ldg(probs) && kern == ADG_KERNEL_STAGE) ? take(8 * tot) : -1;  // the fused kernel keeps q on chip
  L.part = take(3 * 8 * nws);
  L.stats_out = take(3 * 8 * (int64_t)n);
  L.groups = take(4 * (2 * (int64_t)n + 1));
  L.gstats = take(4 * 8 * (int64_t)n);
  L.n_rec = n_rec;
  L.ckpt_every = (opt && opt->ckpt_every > 0) ? opt->ckpt_every : 64;
  L.n_ckpt = rec ? (n_rec + L.ckpt_every - 1) / L.ckpt_every : 0;
  L.ckpt = L.useg = L.ybuf = L.lam = L.q = L.adjring = L.cpart = L.ckrec = L.work_a = L.work_a2 = -1;
  L.rec_atsum_bytes = 8 * S * std::max<int64_t>(at, 1);
  L.rec_atk_bytes = (int64_t)sizeof(RecWord) * std::max<int64_t>(at, 1);
  L.rec_bytes = align_up(L.rec_atsum_bytes, kAlign) + align_up(L.rec_atk_bytes, kAlign);
  if (rec) {
    // stage kernels recompute a segment into seg slots; the fused adjoint
    // reads the segment's first state from its checkpoint and needs seg - 1
    const int64_t seg = std::min<int64_t>(L.ckpt_every, n_rec);
    L.ckpt = take(8 * tot * L.n_ckpt);
    L.useg = take(8 * tot * (kern == ADG_KERNEL_STAGE ? seg : std::max<int64_t>(seg - 1, 1)));
    L.lam = take(8 * tot * 2);
    L.adjring = take(8 * std::max<int64_t>(ring, 1));
    if (kern == ADG_KERNEL_STAGE) {
      L.ybuf = take(8 * tot * (S - 1));
      L.q = take(8 * tot * (S - 1));
      L.cpart = take(8 * nws);
    } else {
      L.ckrec = take(L.rec_bytes * (L.n_ckpt + 1));
      L.work_a = take((int64_t)sizeof(WorkItem) * nwa);
      if (L.n_work_a2 > 0) L.work_a2 = take((int64_t)sizeof(WorkItem) * nwa2);
      L.cpart = take(8 * nwa);
    }
  }
  L.total = off;
  return L;
}

}  // namespace

struct adg_ctx {
  std::vector<adg_problem> probs;
  std::vector<DevProblem> dev;
  adg_options opt{};
  int kernel = ADG_KERNEL_FUSED;
  int rk = 0, phys = 0, S = 0;
  int fused_phys = 0;  // phys of the fused kernel (its launcher takes the a > 0 upwind form per work range)
  hipStream_t stream = nullptr;
  char* ws = nullptr;
  Layout L{};
  int64_t steps = 0;
  // adjoint recording: steps recorded by the last ADG_RUN_RECORD run (0: none)
  int64_t rec_steps = 0;
  // adg_init_scratch: the device whose static scratch array holds the
  // workspace and the generation of that use (-1: caller's workspace)
  int scratch_dev = -1;
  uint64_t scratch_gen = 0;
  // graph cache
  hipGraphExec_t graph = nullptr;
  const double* graph_u = nullptr;
  int graph_steps = 0;

  int32_t group[2][kFusedRanges + 1] = {};  // fused work lists, 1 and 2 steps per launch
  int32_t grid[2][kFusedRanges] = {};
  int32_t single[2][kFusedRanges] = {};
  int32_t one_launch = 0;  // ADG_OPT_ONE_LAUNCH
  int32_t mode[2][kFusedRanges] = {};       // fused_mode of each range of those lists
  bool split = false;                       // PE-face split in use
  int32_t lane_elems = 2;
  int32_t fused_steps = 2;
  // fused adjoint work list (recording contexts of the fused kernel)
  std::vector<WorkItem> work_a, work_a2;
  int32_t group_a[5] = {0, 0, 0, 0, 0}, group_a2[5] = {0, 0, 0, 0, 0};
  int32_t grid_a[4] = {1, 1, 1, 1}, grid_a2[4] = {1, 1, 1, 1};

  StepArgs base_args(int64_t work_off, int32_t n_work, int K = 1) const {
    StepArgs a{};
    a.probs = (const DevProblem*)(ws + L.probs);
    a.work = (const WorkItem*)(ws + work_off);
    a.n_work = n_work;
    a.ring = (double*)(ws + L.ring);
    a.ctr = (int64_t*)(ws + L.ctr);
    a.atsum = (double*)(ws + L.atsum);
    a.atk = (RecWord*)(ws + L.atk);
    for (int i = 0; i <= kFusedRanges; ++i) a.group[i] = group[K - 1][i];
    for (int i = 0; i < kFusedRanges; ++i) a.grid[i] = grid[K - 1][i];
    for (int i = 0; i < kFusedRanges; ++i) a.single[i] = single[K - 1][i];
    for (int i = 0; i < kFusedRanges; ++i) a.mode[i] = mode[K - 1][i];
    a.lane_elems = lane_elems;
    a.one_launch = one_launch;
    a.steps = K;
    a.qbuf = L.qbuf >= 0 ? (double*)(ws + L.qbuf) : nullptr;
    return a;
  }
  StepArgs fused_args(int K = 1) const {
    return K == 2 ? base_args(L.work_f2, L.n_work_f2, 2) : base_args(L.work_f, L.n_work_f, 1);
  }
  StepArgs stage_args() const { return base_args(L.work_s, L.n_work_s); }

  AdjArgs adj_args(int K = 1) const {
    AdjArgs a{};
    a.probs = (const DevProblem*)(ws + L.probs);
    a.work = (const WorkItem*)(ws + (K == 2 ? L.work_a2 : L.work_a));
    for (int i = 0; i < 5; ++i) a.group[i] = K == 2 ? group_a2[i] : group_a[i];
    for (int i = 0; i < 4; ++i) a.grid[i] = K == 2 ? grid_a2[i] : grid_a[i];
    a.lane_elems = K == 2 ? adj_lane_elems(lane_elems) : 1;
    return a;
  }
  // copy the fused kernel's PE-face records to / from checkpoint slot k
  int save_records(int64_t k, bool restore) {
    if (L.ckrec < 0) return ADG_OK;
    char* rec = ws + L.ckrec + L.rec_bytes * k;
    char* sum = ws + L.atsum;
    char* kk = ws + L.atk;
    char* rk_ = rec + align_up(L.rec_atsum_bytes, kAlign);
    ADG_HIP(hipMemcpyAsync(restore ? sum : rec, restore ? rec : sum, L.rec_atsum_bytes, hipMemcpyDeviceToDevice,
                           stream));
    ADG_HIP(hipMemcpyAsync(restore ? kk : rk_, restore ? rk_ : kk, L.rec_atk_bytes, hipMemcpyDeviceToDevice, stream));
    return ADG_OK;
  }

  double* state2() const { return (double*)(ws + L.state2); }
};

namespace {

// Enqueue K steps (K = 2 only for the fused kernel); for the fused kernel the
// result lands in *cur after a swap with the internal buffer.
// K fused steps uin -> uout (with K = 2 also the state after the first step
// into umid, if not null).
int launch_fused(const adg_ctx* c, int K, const double* uin, double* uout, double* umid, int32_t step_offset,
                 hipStream_t st) {
  StepArgs a = c->fused_args(K);
  a.umid = umid;
  ADG_HIP(launch_fused_step(c->rk, c->fused_phys, a, uin, uout, step_offset, st));
  return ADG_OK;
}

int enqueue_steps(adg_ctx* c, double** cur, double** other, int32_t step_offset, int K, hipStream_t st) {
  if (c->kernel == ADG_KERNEL_FUSED) {
    if (int rc = launch_fused(c, K, *cur, *other, nullptr, step_offset, st)) return rc;
    std::swap(*cur, *other);
    return ADG_OK;
  }
  const StepArgs a = c->stage_args();
  double* U = *cur;
  double* Y0 = (double*)(c->ws + c->L.y0);
  double* Y1 = (double*)(c->ws + c->L.y1);
  double* A = (double*)(c->ws + c->L.acc);
  for (int k = 0; k < K; ++k)
    for (int s = 0; s < c->S; ++s) {
      const double* yin = s == 0 ? U : ((s & 1) ? Y0 : Y1);
      double* yout = (s & 1) ? Y1 : Y0;
      if (c->phys == PHYS_BURGERS_LDG) ADG_HIP(launch_ldg_q(c->rk, s, a, yin, step_offset + k, st));
      ADG_HIP(launch_stage(c->rk, c->phys, s, a, yin, yout, U, A, step_offset + k, st));
    }
  return ADG_OK;
}

// Steps [0, m) of a batch: two per launch where the kernel allows.
int enqueue_batch(adg_ctx* c, double** cur, double** other, int32_t m, hipStream_t st) {
  const int kmax = c->kernel == ADG_KERNEL_FUSED ? c->fused_steps : 1;
  for (int32_t i = 0; i < m;) {
    const int K = (kmax == 2 && i + 1 < m) ? 2 : 1;
    const int rc = enqueue_steps(c, cur, other, i, K, st);
    if (rc) return rc;
    i += K;
  }
  return ADG_OK;
}

int reset_device(adg_ctx* c) {
  ADG_HIP(launch_zero(c->ws + c->L.ctr, 8 * sizeof(int64_t), c->stream));
  ADG_HIP(launch_zero(c->ws + c->L.ring, 8 * std::max<int64_t>(c->L.ring_doubles, 1), c->stream));
  ADG_HIP(launch_zero(c->ws + c->L.atsum, 8 * c->S * std::max<int64_t>(c->L.at_entries, 1), c->stream));
  ADG_HIP(launch_zero(c->ws + c->L.atk, sizeof(RecWord) * std::max<int64_t>(c->L.at_entries, 1), c->stream));
  c->steps = 0;
  c->rec_steps = 0;
  return ADG_OK;
}

void drop_graph(adg_ctx* c) {
  if (c->graph) (void)hipGraphExecDestroy(c->graph);
  c->graph = nullptr;
  c->graph_u = nullptr;
  c->graph_steps = 0;
}

constexpr int kGraphSteps = 16;  // even: the fused ping-pong ends in the caller's buffer

int build_graph(adg_ctx* c, double* d_u) {
  drop_graph(c);
  hipStream_t cap;
  ADG_HIP(hipStreamCreateWithFlags(&cap, hipStreamNonBlocking));
  hipGraph_t g = nullptr;
  int rc = ADG_OK;
  if (hipStreamBeginCapture(cap, hipStreamCaptureModeThreadLocal) != hipSuccess) {
    (void)hipStreamDestroy(cap);
    return fail(ADG_E_HIP, "hipStreamBeginCapture failed");
  }
  double* cur = d_u;
  double* other = c->state2();
  rc = enqueue_batch(c, &cur, &other, kGraphSteps, cap);
  if (rc == ADG_OK && launch_advance((int64_t*)(c->ws + c->L.ctr), kGraphSteps, cap) != hipSuccess)
    rc = fail(ADG_E_HIP, "capture of the step-counter advance failed");
  const hipError_t e1 = hipStreamEndCapture(cap, &g);
  (void)hipStreamDestroy(cap);
  if (rc != ADG_OK) { if (g) (void)hipGraphDestroy(g); return rc; }
  if (e1 != hipSuccess) return fail(ADG_E_HIP, std::string("hipStreamEndCapture: ") + hipGetErrorString(e1));
  hipGraphExec_t ex = nullptr;
  const hipError_t e2 = hipGraphInstantiate(&ex, g, nullptr, nullptr, 0);
  (void)hipGraphDestroy(g);
  if (e2 != hipSuccess) return fail(ADG_E_HIP, std::string("hipGraphInstantiate: ") + hipGetErrorString(e2));
  c->graph = ex;
  c->graph_u = d_u;
  c->graph_steps = kGraphSteps;
  return ADG_OK;
}

}  // namespace

// Workspace of adg_init_scratch, for callers that cannot allocate device
// memory: one array per GPU the library runs on, held until the process ends.
// Host code never uses this name as a device address (on the host it is a
// stand-in); its per-device address comes from hipGetSymbolAddress.
constexpr int64_t kScratchBytes = ADG_SCRATCH_BYTES;
static __device__ __align__(256) unsigned char scratch[kScratchBytes];

namespace {

std::mutex g_scratch_mu;
std::vector<void*> g_scratch_ptr;       // per device: address of `scratch`
std::vector<uint64_t> g_scratch_gen;    // per device: generation of the current use

// Address of the scratch array on the current device (looked up once per
// device) and a new generation number for its next use.
int scratch_acquire(int* dev_out, void** ptr_out, uint64_t* gen_out) {
  int dev = 0;
  ADG_HIP(hipGetDevice(&dev));
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if ((int)g_scratch_ptr.size() <= dev) {
    g_scratch_ptr.resize(dev + 1, nullptr);
    g_scratch_gen.resize(dev + 1, 0);
  }
  if (!g_scratch_ptr[dev]) {
    void* p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !p)
      return fail(ADG_E_HIP, std::string("hipGetSymbolAddress(scratch): ") + hipGetErrorString(e));
    g_scratch_ptr[dev] = p;
  }
  *dev_out = dev;
  *ptr_out = g_scratch_ptr[dev];
  *gen_out = ++g_scratch_gen[dev];
  return ADG_OK;
}

// A context on the scratch array is live until a later adg_init_scratch on
// the same device takes the array over.
int check_live(const adg_ctx* c) {
  if (c->scratch_dev < 0) return ADG_OK;
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (c->scratch_gen != g_scratch_gen[c->scratch_dev])
    return fail(ADG_E_STATE, "the scratch workspace was taken over by a later adg_init_scratch");
  return ADG_OK;
}

}  // namespace

extern "C" {

int adg_abi_version(void) { return ADG_ABI_VERSION; }

const char* adg_last_error(void) { return g_err.c_str(); }

#ifndef ADG_SOURCE_HASH
#error "compile with -DADG_SOURCE_HASH=\"<hash of csrc/ and include/>\" (paper_2404_03399_amd/build.py does)"
#endif
const char* adg_build_id(void) { return ADG_SOURCE_HASH; }

int adg_nodes(int32_t degree, double* xi) {
  if (degree < 1 || degree > 4 || !xi) return fail(ADG_E_INVALID, "adg_nodes: degree must be 1..4");
  long double x[kMaxNp];
  gll(degree, x);
  for (int i = 0; i <= degree; ++i) xi[i] = (double)x[i];
  return ADG_OK;
}

int adg_state_layout(const adg_problem* probs, int32_t n_probs, int64_t* offsets, int64_t* lds,
                     int64_t* total_doubles) {
  int rc = validate(probs, n_probs);
  if (rc) return rc;
  int64_t off = 0;
  for (int32_t i = 0; i < n_probs; ++i) {
    if (offsets) offsets[i] = off;
    if (lds) lds[i] = ld_of(probs[i]);
    off += ld_of(probs[i]) * (probs[i].degree + 1);
  }
  if (total_doubles) *total_doubles = off;
  return ADG_OK;
}

int adg_workspace_size(const adg_problem* probs, int32_t n_probs, const adg_options* opt, int64_t n_steps_record,
                       int64_t* bytes_out) {
  int rc = validate(probs, n_probs);
  if (rc) return rc;
  if (!bytes_out) return fail(ADG_E_INVALID, "bytes_out is null");
  if (n_steps_record < 0 || n_steps_record > (1 << 28)) return fail(ADG_E_INVALID, "n_steps_record out of range");
  if (opt && opt->ckpt_every < 0) return fail(ADG_E_INVALID, "ckpt_every < 0");
  const int k = kernel_of(probs, opt);
  if (k != ADG_KERNEL_FUSED && k != ADG_KERNEL_STAGE) return fail(ADG_E_INVALID, "unknown kernel family");
  if (lane_elems_of(probs, n_probs, opt) == 0)
    return fail(ADG_E_INVALID, "lane_elems must be 1, 2 or 4 and not exceed the PE size");
  if (fused_steps_of(opt) == 0) return fail(ADG_E_INVALID, "fused_steps must be 0, 1 or 2");
  if (opt && (opt->flags & ~(ADG_OPT_PE_SPLIT_OFF | ADG_OPT_PE_SPLIT_ON | ADG_OPT_ONE_LAUNCH)))
    return fail(ADG_E_INVALID, "unknown adg_options.flags bits");
  if (opt && (opt->flags & ADG_OPT_PE_SPLIT_OFF) && (opt->flags & ADG_OPT_PE_SPLIT_ON))
    return fail(ADG_E_INVALID, "ADG_OPT_PE_SPLIT_OFF and ADG_OPT_PE_SPLIT_ON together");
  if (opt && (opt->flags & ADG_OPT_ONE_LAUNCH)) {
    if ((opt->flags & ADG_OPT_PE_SPLIT_ON) || k != ADG_KERNEL_FUSED || lane_elems_of(probs, n_probs, opt) != 2)
      return fail(ADG_E_INVALID, "ADG_OPT_ONE_LAUNCH needs the fused kernel, two elements per lane and no PE-face split");
    if (is_ldg(probs)) return fail(ADG_E_UNSUPPORTED, "ADG_OPT_ONE_LAUNCH: the local DG kernel launches per range");
  }
  if (is_ldg(probs) && n_steps_record > 0)
    return fail(ADG_E_UNSUPPORTED, "no adjoint for viscous Burgers (local DG)");
  *bytes_out = make_layout(probs, n_probs, opt, n_steps_record).total;
  return ADG_OK;
}

int adg_init(adg_ctx** out, const adg_problem* probs, int32_t n_probs, const adg_options* opt, int64_t n_steps_record,
             void* d_workspace, int64_t workspace_bytes, void* hip_stream) {
  if (!out) return fail(ADG_E_INVALID, "out is null");
  *out = nullptr;
  int64_t need = 0;
  int rc = adg_workspace_size(probs, n_probs, opt, n_steps_record, &need);
  if (rc) return rc;
  if (!d_workspace || workspace_bytes < need) return fail(ADG_E_WORKSPACE, "workspace too small: need " + std::to_string(need));
  if (((uintptr_t)d_workspace) % kAlign) return fail(ADG_E_WORKSPACE, "workspace must be 256-byte aligned");

  adg_ctx* c = new adg_ctx();
  c->probs.assign(probs, probs + n_probs);
  if (opt) c->opt = *opt;
  c->kernel = kernel_of(probs, opt);
  c->rk = (int)probs[0].rk;
  c->phys = phys_of(probs[0]);
  c->fused_phys = c->phys;
  c->S = rk_stages(c->rk);
  c->stream = (hipStream_t)hip_stream;
  c->ws = (char*)d_workspace;
  c->L = make_layout(probs, n_probs, opt, n_steps_record);

  // descriptors
  c->dev.resize(n_probs);
  int64_t uoff = 0, roff = 0, aoff = 0;
  for (int32_t i = 0; i < n_probs; ++i) {
    const adg_problem& p = probs[i];
    DevProblem& d = c->dev[i];
    std::memset(&d, 0, sizeof(d));
    d.n_elem = p.n_elem;
    d.pe_size = p.pe_size;
    d.n_pe = p.n_elem / p.pe_size;
    d.ld = ld_of(p);
    d.u_off = uoff;
    uoff += d.ld * (p.degree + 1);
    d.np = (int)p.degree + 1;
    d.q = q_of(p);
    d.n_delays = (int)p.n_delays;
    d.depth = (int32_t)depth_of(p, n_steps_record);
    d.per_stage = p.delay_granularity == ADG_DELAY_PER_STAGE;
    d.caa = p.delay_granularity == ADG_DELAY_CAA;
    d.scheme = (int)p.scheme;
    d.async_faces = async_of(p) ? 1 : 0;
    d.pe_div = make_fast_div((uint32_t)p.pe_size);
    for (int64_t v : {(int64_t)0, p.pe_size - 1, p.pe_size, p.n_elem - 1, p.n_elem, p.n_elem / 2 + 1}) {
      if (v < 0) continue;
      if ((int64_t)fast_div((uint32_t)v, d.pe_div) != v / p.pe_size) {
        delete c;
        return fail(ADG_E_INVALID, "internal: division by pe_size failed self-check");
      }
    }
    d.ring_off = roff;
    d.at_off = aoff * c->S;
    d.atk_off = aoff;
    if (d.async_faces) {
      const int64_t one_ring = d.n_pe * c->S * (int64_t)d.depth;
      d.ring2_off = roff + one_ring;
      roff += (is_ldg(probs) ? 2 : 1) * one_ring;
      aoff += kRecSlots * d.n_pe;
    }
    d.seed = p.seed;
    for (int k = 0; k + 1 < d.n_delays; ++k) d.thr[k] = p.delay_threshold[k];
    const double dx = p.length / (double)p.n_elem;
    d.two_over_dx = 2.0 / dx;
    d.half_dx = 0.5 * dx;
    d.speed = p.equation == ADG_EQ_ADVECTION ? p.speed : 1.0;
    d.nu = p.viscosity;
    d.dt = p.dt;
    element_operators((int)p.degree, &d);
    {
      // Kd folds the flux constant: a (advection), 1/2 (Burgers: g = u^2), 1
      // (local DG: g = u^2/2 - nu q is formed in the kernel)
      const double fac = p.equation == ADG_EQ_ADVECTION ? p.speed
                         : (p.equation == ADG_EQ_BURGERS ? 0.5 : 1.0);
      for (int i = 0; i < kMaxNp * kMaxNp; ++i) d.Kd[i] = d.two_over_dx * fac * d.D[i];
      for (int i = 0; i < kMaxNp; ++i) {
        d.Kl[i] = d.two_over_dx * d.lift_l[i];
        d.Kr[i] = d.two_over_dx * d.lift_r[i];
      }
      for (int i = 0; i < kMaxNp * kMaxNp; ++i) d.Kdu[i] = d.Kd[i];
      const int pn = (int)p.degree;
      for (int i = 0; i <= pn; ++i) d.Kdu[i * kMaxNp + pn] -= d.Kr[i] * p.speed;
    }
    d.depth_div = make_fast_div((uint32_t)d.depth);
    for (int k = 0; k < d.n_delays; ++k)
      for (int j = 0; j < d.q; ++j) d.atc[k][j] = at_coefficient(d.q, k, j);
  }
  if (roff != c->L.ring_doubles || aoff != c->L.at_entries) {
    delete c;
    return fail(ADG_E_INVALID, "internal: ring or record layout does not match the workspace layout");
  }
  // work lists: heaviest (highest degree) problems first
  std::vector<int32_t> order(n_probs);
  for (int32_t i = 0; i < n_probs; ++i) order[i] = i;
  std::stable_sort(order.begin(), order.end(), [&](int32_t a, int32_t b) { return probs[a].degree > probs[b].degree; });
  c->lane_elems = lane_elems_of(probs, n_probs, opt);
  c->fused_steps = fused_steps_of(opt);
  std::vector<WorkItem> wfk[2], ws_;
  std::vector<int32_t> first(n_probs + 1, 0);
  // PE-face split: in each range the window items of its asynchronous
  // problems (fused_windows_per_wave faces per item, tile index -(group + 1))
  // are interleaved with the tiles of every problem in order of their first
  // element; ranges without asynchronous problems take the kernel with the
  // PE-face paths compiled out
  c->split = pe_split_of(probs, n_probs, opt);
  c->one_launch = (opt && (opt->flags & ADG_OPT_ONE_LAUNCH)) ? 1 : 0;
  for (int K = 1; K <= 2; ++K) {
    const int T = fused_tile(c->rk, c->lane_elems, K);
    const int fw = fused_windows_per_wave(c->rk, K);
    std::vector<WorkItem>& wf = wfk[K - 1];
    wf.reserve(K == 1 ? c->L.n_work_f : c->L.n_work_f2);
    // ranges per degree, np = 5, 4, 3, 2 (order is sorted by degree,
    // descending), each split into the a > 0 upwind form and the rest
    for (int gi = 0; gi < kFusedRanges; ++gi) {
      const int np = 5 - gi / 2;
      const bool pos_range = (gi & 1) == 0;
      auto in_range = [&](int32_t i) {
        const bool pos = c->phys == PHYS_ADV_UPWIND && probs[i].speed > 0.0;
        return (int)probs[i].degree + 1 == np && pos == pos_range;
      };
      c->group[K - 1][gi] = (int32_t)wf.size();
      bool range_async = false;
      for (int32_t i : order)
        if (in_range(i) && async_of(probs[i])) range_async = true;
      for (int32_t i : order) {
        if (!in_range(i)) continue;
        const int64_t nt = (probs[i].n_elem + T - 1) / T;
        const bool win = c->split && async_of(probs[i]);
        const int64_t ng = win ? (probs[i].n_elem / probs[i].pe_size + fw - 1) / fw : 0;
        const int64_t gstride = (int64_t)fw * probs[i].pe_size;  // elements between window groups
        // merge by first element: window group g at g * fw * pe_size, tile t at t * T
        for (int64_t t = 0, g = 0; t < nt || g < ng;) {
          if (g < ng && (t >= nt || g * gstride <= t * T)) {
            wf.push_back(WorkItem{i, (int32_t)(-g - 1)});
            ++g;
          } else {
            wf.push_back(WorkItem{i, (int32_t)t});
            ++t;
          }
        }
      }
      c->mode[K - 1][gi] = !range_async ? FUSED_NOPE : (c->split ? FUSED_SPLIT : FUSED_FULL);
    }
    c->group[K - 1][kFusedRanges] = (int32_t)wf.size();
    if ((int64_t)wf.size() != (K == 1 ? c->L.n_work_f : c->L.n_work_f2)) {
      delete c;
      return fail(ADG_E_INVALID, "internal: fused work list does not match the workspace layout");
    }
    for (int gi = 0; gi < kFusedRanges; ++gi) {
      const int32_t b = c->group[K - 1][gi], e = c->group[K - 1][gi + 1];
      c->grid[K - 1][gi] = fused_grid(e - b);
      // one problem whose tiles are listed in order: the kernel forms its
      // items without loading the list (never under the split)
      bool one = e > b && c->mode[K - 1][gi] != FUSED_SPLIT;
      for (int32_t w = b; w < e && one; ++w) one = wf[w].prob == wf[b].prob && wf[w].tile == w - b;
      c->single[K - 1][gi] = one ? wf[b].prob : -1;
    }
  }
  for (int32_t i = 0; i < n_probs; ++i) {  // stage/stats list in problem order (contiguous per problem)
    first[i] = (int32_t)ws_.size();
    const int64_t nt = (probs[i].n_elem + kBlock - 1) / kBlock;
    for (int64_t t = 0; t < nt; ++t) ws_.push_back(WorkItem{i, (int32_t)t});
  }
  first[n_probs] = (int32_t)ws_.size();
  // fused adjoint: one element per lane, same degree grouping
  auto adj_list = [&](int T1, std::vector<WorkItem>& wl, int32_t* grp, int32_t* grd) {
    for (int np = 5, gi = 0; np >= 2; --np, ++gi) {
      grp[gi] = (int32_t)wl.size();
      for (int32_t i : order) {
        if ((int)probs[i].degree + 1 != np) continue;
        const int64_t nt = (probs[i].n_elem + T1 - 1) / T1;
        for (int64_t t = 0; t < nt; ++t) wl.push_back(WorkItem{i, (int32_t)t});
      }
    }
    grp[4] = (int32_t)wl.size();
    for (int gi = 0; gi < 4; ++gi) grd[gi] = fused_grid(grp[gi + 1] - grp[gi]);
  };
  if (c->L.work_a >= 0)
    adj_list(adj_tile_elems(c->rk, probs[0].equation == ADG_EQ_BURGERS), c->work_a, c->group_a, c->grid_a);
  if (c->L.work_a2 >= 0)
    adj_list(adj_tile_elems2(c->rk, adj_lane_elems(c->lane_elems)), c->work_a2, c->group_a2, c->grid_a2);
  if ((c->L.work_a >= 0 && (int64_t)c->work_a.size() != c->L.n_work_a) ||
      (c->L.work_a2 >= 0 && (int64_t)c->work_a2.size() != c->L.n_work_a2)) {
    delete c;
    return fail(ADG_E_INVALID, "internal: adjoint work list does not match the workspace layout");
  }

  auto up = [&](int64_t off, const void* src, int64_t bytes) -> int {
    ADG_HIP(hipMemcpyAsync(c->ws + off, src, bytes, hipMemcpyHostToDevice, c->stream));
    return ADG_OK;
  };
  if ((rc = up(c->L.probs, c->dev.data(), (int64_t)sizeof(DevProblem) * n_probs)) ||
      (rc = up(c->L.work_f, wfk[0].data(), (int64_t)sizeof(WorkItem) * wfk[0].size())) ||
      (rc = up(c->L.work_f2, wfk[1].data(), (int64_t)sizeof(WorkItem) * wfk[1].size())) ||
      (rc = up(c->L.work_s, ws_.data(), (int64_t)sizeof(WorkItem) * ws_.size())) ||
      (rc = up(c->L.first_s, first.data(), (int64_t)sizeof(int32_t) * first.size())) ||
      (c->L.work_a >= 0 &&
       (rc = up(c->L.work_a, c->work_a.data(), (int64_t)sizeof(WorkItem) * c->work_a.size()))) ||
      (c->L.work_a2 >= 0 &&
       (rc = up(c->L.work_a2, c->work_a2.data(), (int64_t)sizeof(WorkItem) * c->work_a2.size()))) ||
      (rc = reset_device(c))) {
    delete c;
    return rc;
  }
  // host data above must stay valid until the copies ran
  if (hipStreamSynchronize(c->stream) != hipSuccess) {
    delete c;
    return fail(ADG_E_HIP, "stream synchronisation after upload failed");
  }
  *out = c;
  return ADG_OK;
}

int adg_init_scratch(adg_ctx** out, const adg_problem* probs, int32_t n_probs, const adg_options* opt,
                     void* hip_stream) {
  if (!out) return fail(ADG_E_INVALID, "out is null");
  *out = nullptr;
  int64_t need = 0;
  int rc = adg_workspace_size(probs, n_probs, opt, 0, &need);
  if (rc) return rc;
  if (need > kScratchBytes)
    return fail(ADG_E_WORKSPACE, "adg_init_scratch: these problems need " + std::to_string(need) +
                                     " bytes of workspace; the static scratch array holds " +
                                     std::to_string(kScratchBytes));
  int dev = 0;
  void* ws = nullptr;
  uint64_t gen = 0;
  if ((rc = scratch_acquire(&dev, &ws, &gen))) return rc;
  if ((rc = adg_init(out, probs, n_probs, opt, 0, ws, need, hip_stream))) return rc;
  (*out)->scratch_dev = dev;
  (*out)->scratch_gen = gen;
  return ADG_OK;
}

int adg_reset(adg_ctx* c) {
  if (!c) return fail(ADG_E_INVALID, "null context");
  if (int rc = check_live(c)) return rc;
  return reset_device(c);
}

int adg_step_count(const adg_ctx* c, int64_t* steps) {
  if (!c || !steps) return fail(ADG_E_INVALID, "null argument");
  *steps = c->steps;
  return ADG_OK;
}

int adg_run(adg_ctx* c, double* d_u, int64_t n_steps, uint32_t flags) {
  if (!c || !d_u) return fail(ADG_E_INVALID, "null argument");
  if (int rc = check_live(c)) return rc;
  if (!state_aligned(d_u)) return fail(ADG_E_INVALID, "d_u must be 16-byte aligned");
  if (n_steps < 0) return fail(ADG_E_INVALID, "n_steps < 0");
  if (c->steps + n_steps >= ((int64_t)1 << 31)) return fail(ADG_E_INVALID, "step index would exceed 2^31 - 1");
  if (flags & ~(ADG_RUN_GRAPH | ADG_RUN_RECORD | ADG_RUN_CHECK_FINITE)) return fail(ADG_E_INVALID, "unknown flags");
  if (flags & ADG_RUN_RECORD) {
    if (c->L.n_rec <= 0) return fail(ADG_E_STATE, "context was created without a recording horizon");
    if (c->steps != 0) return fail(ADG_E_STATE, "ADG_RUN_RECORD must start at step 0 (call adg_reset)");
    if (n_steps > c->L.n_rec) return fail(ADG_E_INVALID, "n_steps exceeds the recording horizon");
    const int64_t C = c->L.ckpt_every, tot = c->L.total_doubles;
    int64_t done = 0;
    int rc;
    if (C == 1 && c->kernel == ADG_KERNEL_FUSED) {
      // every state is kept: each step writes its result straight into the
      // next checkpoint slot (the last one into d_u), no copies; two steps per
      // launch where the context runs two, the launch writing both states
      double* ck = (double*)(c->ws + c->L.ckpt);
      ADG_HIP(hipMemcpyAsync(ck, d_u, 8 * tot, hipMemcpyDeviceToDevice, c->stream));
      auto slot = [&](int64_t j) { return j < n_steps ? ck + tot * j : d_u; };
      while (done < n_steps) {
        const int32_t m = (int32_t)std::min<int64_t>(n_steps - done, kGraphSteps);
        for (int32_t i = 0; i < m;) {
          const int64_t n = done + i;
          if (c->fused_steps == 2 && i + 1 < m) {
            if ((rc = launch_fused(c, 2, ck + tot * n, slot(n + 2), slot(n + 1), i, c->stream))) return rc;
            i += 2;
          } else {
            if ((rc = launch_fused(c, 1, ck + tot * n, slot(n + 1), nullptr, i, c->stream))) return rc;
            i += 1;
          }
        }
        ADG_HIP(launch_advance((int64_t*)(c->ws + c->L.ctr), m, c->stream));
        done += m;
      }
      c->steps += n_steps;
      c->rec_steps = n_steps;
      if (flags & ADG_RUN_CHECK_FINITE) return adg_run(c, d_u, 0, ADG_RUN_CHECK_FINITE);
      return ADG_OK;
    }
    for (int64_t k = 0; done < n_steps; ++k) {
      ADG_HIP(hipMemcpyAsync(c->ws + c->L.ckpt + 8 * tot * k, d_u, 8 * tot, hipMemcpyDeviceToDevice, c->stream));
      if ((rc = c->save_records(k, false))) return rc;
      const int64_t m = std::min<int64_t>(C, n_steps - done);
      if ((rc = adg_run(c, d_u, m, flags & ~(ADG_RUN_RECORD | ADG_RUN_CHECK_FINITE)))) return rc;
      done += m;
    }
    c->rec_steps = n_steps;
    if (flags & ADG_RUN_CHECK_FINITE) return adg_run(c, d_u, 0, ADG_RUN_CHECK_FINITE);
    return ADG_OK;
  }
  int rc;
  if (n_steps == 0 && (flags & ADG_RUN_GRAPH) && (c->graph_u != d_u || !c->graph)) {
    // capture only: the step graph for d_u, replayed by later runs
    if ((rc = build_graph(c, d_u))) return rc;
  }
  if (n_steps > 0) c->rec_steps = 0;  // any further step invalidates a recording
  double* cur = d_u;
  double* other = c->kernel == ADG_KERNEL_FUSED ? c->state2() : nullptr;
  int64_t left = n_steps;
  if ((flags & ADG_RUN_GRAPH) && left >= kGraphSteps) {
    if (c->graph_u != d_u || !c->graph) {
      if ((rc = build_graph(c, d_u))) return rc;
    }
    while (left >= c->graph_steps) {
      ADG_HIP(hipGraphLaunch(c->graph, c->stream));
      left -= c->graph_steps;
    }
  }
  // remaining steps in batches of at most kGraphSteps, each closed by one
  // counter advance
  while (left > 0) {
    const int32_t m = (int32_t)std::min<int64_t>(left, kGraphSteps);
    if ((rc = enqueue_batch(c, &cur, &other, m, c->stream))) return rc;
    ADG_HIP(launch_advance((int64_t*)(c->ws + c->L.ctr), m, c->stream));
    left -= m;
  }
  if (cur != d_u)
    ADG_HIP(hipMemcpyAsync(d_u, cur, 8 * c->L.total_doubles, hipMemcpyDeviceToDevice, c->stream));
  c->steps += n_steps;
  if (flags & ADG_RUN_CHECK_FINITE) {
    int64_t* ctr = (int64_t*)(c->ws + c->L.ctr);
    ADG_HIP(launch_zero(ctr + 2, sizeof(int64_t), c->stream));
    ADG_HIP(launch_check_finite(c->stage_args(), d_u, c->stream));
    int64_t flag = 0;
    ADG_HIP(hipMemcpyAsync(&flag, ctr + 2, sizeof(int64_t), hipMemcpyDeviceToHost, c->stream));
    ADG_HIP(hipStreamSynchronize(c->stream));
    if (flag) return fail(ADG_E_NONFINITE, "state contains NaN or Inf");
  }
  return ADG_OK;
}

int adg_step(adg_ctx* c, double* d_u) { return adg_run(c, d_u, 1, 0); }

namespace {

// Per-problem sums of the per-work-item dJ/da shares, in work-list order.
void sum_speed_parts(const adg_ctx* c, const std::vector<double>& part, const std::vector<WorkItem>& items,
                     double* h_grad_speed) {
  std::vector<double> acc(c->probs.size(), 0.0);
  for (size_t t = 0; t < items.size(); ++t) acc[items[t].prob] += part[t];
  for (size_t i = 0; i < c->probs.size(); ++i)
    h_grad_speed[i] = c->probs[i].equation == ADG_EQ_ADVECTION ? acc[i] : 0.0;
}

// Adjoint with the per-stage kernels: the segment is recomputed stage by
// stage, and every reverse stage is one launch with its RK registers in HBM.
int adjoint_stage(adg_ctx* c, const double* d_cot_uT, double* d_grad_u0, double* h_grad_speed) {
  const Layout& L = c->L;
  const int64_t tot = L.total_doubles, C = L.ckpt_every, N = c->rec_steps;
  const int S = c->S;
  char* ws = c->ws;
  hipStream_t st = c->stream;
  const StepArgs sa = c->stage_args();
  double* lam = (double*)(ws + L.lam);
  double* lamu = lam + tot;
  double* Q = (double*)(ws + L.q);
  double* adjring = (double*)(ws + L.adjring);
  double* cpart = (double*)(ws + L.cpart);
  double* ring = (double*)(ws + L.ring);
  double* useg = (double*)(ws + L.useg);
  double* ybuf = (double*)(ws + L.ybuf);
  double* abuf = (double*)(ws + L.acc);
  double* y0 = (double*)(ws + L.y0);
  double* y1 = (double*)(ws + L.y1);
  int64_t* ctr = (int64_t*)(ws + L.ctr);
  const size_t bytes = 8 * (size_t)tot;

  ADG_HIP(hipMemcpyAsync(lam, d_cot_uT, bytes, hipMemcpyDeviceToDevice, st));
  ADG_HIP(launch_zero(adjring, 8 * std::max<int64_t>(L.ring_doubles, 1), st));
  ADG_HIP(launch_zero(cpart, 8 * (size_t)L.n_work_s, st));
  ADG_HIP(launch_set_counter(ctr, 0, st));  // launches below pass absolute step indices

  for (int64_t k = L.n_ckpt - 1; k >= 0; --k) {
    const int64_t n0 = k * C;
    const int64_t len = std::min<int64_t>(C, N - n0);
    if (len <= 0) continue;
    // recompute the segment's states u^{n0}, ..., u^{n0+len-1}
    ADG_HIP(hipMemcpyAsync(useg, ws + L.ckpt + 8 * tot * k, bytes, hipMemcpyDeviceToDevice, st));
    for (int64_t i = 1; i < len; ++i) {
      double* u = useg + tot * i;
      ADG_HIP(hipMemcpyAsync(u, u - tot, bytes, hipMemcpyDeviceToDevice, st));
      for (int s = 0; s < S; ++s) {
        const double* yin = s == 0 ? u : ((s & 1) ? y0 : y1);
        double* yout = (s & 1) ? y1 : y0;
        ADG_HIP(launch_stage(c->rk, c->phys, s, sa, yin, yout, u, abuf, (int32_t)(n0 + i - 1), st));
      }
    }
    for (int64_t i = len - 1; i >= 0; --i) {
      const int32_t n = (int32_t)(n0 + i);
      double* u = useg + tot * i;
      // stage inputs Y_1 = u^n, Y_2..Y_S
      for (int s = 0; s + 1 < S; ++s) {
        const double* yin = s == 0 ? u : ybuf + tot * (s - 1);
        ADG_HIP(launch_stage(c->rk, c->phys, s, sa, yin, ybuf + tot * s, u, abuf, n, st));
      }
      if (S > 1) ADG_HIP(launch_zero(Q, bytes * (S - 1), st));
      ADG_HIP(hipMemcpyAsync(lamu, lam, bytes, hipMemcpyDeviceToDevice, st));
      for (int s = S - 1; s >= 0; --s) {
        const double* Y = s == 0 ? u : ybuf + tot * (s - 1);
        ADG_HIP(launch_adj_stage(c->rk, c->phys, s, sa, Y, lam, lamu, Q, tot, ring, adjring, cpart, n, st));
      }
      std::swap(lam, lamu);
    }
  }
  ADG_HIP(hipMemcpyAsync(d_grad_u0, lam, bytes, hipMemcpyDeviceToDevice, st));
  ADG_HIP(launch_set_counter(ctr, c->steps, st));
  if (h_grad_speed) {
    std::vector<double> part(L.n_work_s);
    ADG_HIP(hipMemcpyAsync(part.data(), cpart, 8 * part.size(), hipMemcpyDeviceToHost, st));
    ADG_HIP(hipStreamSynchronize(st));
    std::vector<WorkItem> items;  // stage work list: contiguous per problem, in problem order
    items.reserve(L.n_work_s);
    for (size_t i = 0; i < c->probs.size(); ++i) {
      const int64_t nt = (c->probs[i].n_elem + kBlock - 1) / kBlock;
      for (int64_t t = 0; t < nt; ++t) items.push_back(WorkItem{(int32_t)i, (int32_t)t});
    }
    sum_speed_parts(c, part, items, h_grad_speed);
  }
  return ADG_OK;
}

// Adjoint with the fused kernels: each segment is recomputed out of place by
// the fused step kernel (from the checkpointed state and PE-face records, so
// the states are bitwise those of the recorded run), then every reverse step
// is one launch per degree group.  The records of the current step are kept
// in the spare checkpoint slot and restored at the end, so the context can
// keep stepping afterwards.
int adjoint_fused(adg_ctx* c, const double* d_cot_uT, double* d_grad_u0, double* h_grad_speed) {
  const Layout& L = c->L;
  const int64_t tot = L.total_doubles, C = L.ckpt_every, N = c->rec_steps;
  char* ws = c->ws;
  hipStream_t st = c->stream;
  const AdjArgs aa = c->adj_args();
  double* lam = (double*)(ws + L.lam);
  double* lamu = lam + tot;
  double* adjring = (double*)(ws + L.adjring);
  double* cpart = (double*)(ws + L.cpart);
  const double* ring = (const double*)(ws + L.ring);
  double* useg = (double*)(ws + L.useg);
  int64_t* ctr = (int64_t*)(ws + L.ctr);
  const size_t bytes = 8 * (size_t)tot;
  int rc;

  if ((rc = c->save_records(L.n_ckpt, false))) return rc;
  ADG_HIP(hipMemcpyAsync(lam, d_cot_uT, bytes, hipMemcpyDeviceToDevice, st));
  ADG_HIP(launch_zero(adjring, 8 * std::max<int64_t>(L.ring_doubles, 1), st));
  ADG_HIP(launch_zero(cpart, 8 * (size_t)std::max<int32_t>(L.n_work_a, 1), st));
  ADG_HIP(launch_set_counter(ctr, 0, st));  // launches below pass absolute step indices

  // linear advection: the reverse sweep does not depend on the forward states;
  // they are recomputed only for dJ/da
  const bool need_fwd = c->phys == PHYS_BURGERS_LLF || h_grad_speed != nullptr;
  if (!need_fwd) {
    const AdjArgs aa2 = c->adj_args(2);
    for (int64_t n = N - 1; n >= 0;) {
      if (c->fused_steps == 2 && L.work_a2 >= 0 && n >= 1) {  // steps n and n - 1 in one launch
        ADG_HIP(launch_adj_fused2(c->rk, c->phys, aa2, lam, lamu, adjring, (int32_t)(n - 1), st));
        n -= 2;
      } else {
        ADG_HIP(launch_adj_fused(c->rk, c->phys, aa, nullptr, lam, lamu, ring, adjring, cpart, (int32_t)n, st));
        n -= 1;
      }
      std::swap(lam, lamu);
    }
  }
  for (int64_t k = need_fwd ? L.n_ckpt - 1 : -1; k >= 0; --k) {
    const int64_t n0 = k * C;
    const int64_t len = std::min<int64_t>(C, N - n0);
    if (len <= 0) continue;
    // u^{n0+i}: the checkpoint itself for i = 0, recomputed into useg[i-1] after
    double* ck = (double*)(ws + L.ckpt) + tot * k;
    auto state = [&](int64_t i) { return i == 0 ? ck : useg + tot * (i - 1); };
    if (len > 1 && (rc = c->save_records(k, true))) return rc;
    for (int64_t i = 1; i < len;) {
      if (c->fused_steps == 2 && i + 1 < len) {  // two steps per launch, the first one written too
        if ((rc = launch_fused(c, 2, state(i - 1), state(i + 1), state(i), (int32_t)(n0 + i - 1), st))) return rc;
        i += 2;
      } else {
        if ((rc = launch_fused(c, 1, state(i - 1), state(i), nullptr, (int32_t)(n0 + i - 1), st))) return rc;
        i += 1;
      }
    }
    for (int64_t i = len - 1; i >= 0; --i) {
      ADG_HIP(launch_adj_fused(c->rk, c->phys, aa, state(i), lam, lamu, ring, adjring, cpart, (int32_t)(n0 + i),
                               st));
      std::swap(lam, lamu);
    }
  }
  ADG_HIP(hipMemcpyAsync(d_grad_u0, lam, bytes, hipMemcpyDeviceToDevice, st));
  if ((rc = c->save_records(L.n_ckpt, true))) return rc;
  ADG_HIP(launch_set_counter(ctr, c->steps, st));
  if (h_grad_speed) {
    std::vector<double> part(c->work_a.size());
    ADG_HIP(hipMemcpyAsync(part.data(), cpart, 8 * part.size(), hipMemcpyDeviceToHost, st));
    ADG_HIP(hipStreamSynchronize(st));
    sum_speed_parts(c, part, c->work_a, h_grad_speed);
  }
  return ADG_OK;
}

}  // namespace

int adg_adjoint(adg_ctx* c, const double* d_cot_uT, double* d_grad_u0, double* h_grad_speed) {
  if (!c || !d_cot_uT || !d_grad_u0) return fail(ADG_E_INVALID, "null argument");
  if (int rc = check_live(c)) return rc;
  if (!state_aligned(d_cot_uT) || !state_aligned(d_grad_u0))
    return fail(ADG_E_INVALID, "d_cot_uT and d_grad_u0 must be 16-byte aligned");
  if (c->rec_steps <= 0) return fail(ADG_E_STATE, "adg_adjoint needs a run recorded with ADG_RUN_RECORD");
  return c->kernel == ADG_KERNEL_FUSED ? adjoint_fused(c, d_cot_uT, d_grad_u0, h_grad_speed)
                                       : adjoint_stage(c, d_cot_uT, d_grad_u0, h_grad_speed);
}

int adg_error_stats(adg_ctx* c, const double* d_u, const double* d_ref, double* h_out) {
  if (!c || !d_u || !d_ref || !h_out) return fail(ADG_E_INVALID, "null argument");
  if (!state_aligned(d_u) || !state_aligned(d_ref)) return fail(ADG_E_INVALID, "d_u and d_ref must be 16-byte aligned");
  if (int rc = check_live(c)) return rc;
  const int32_t n = (int32_t)c->probs.size();
  double* part = (double*)(c->ws + c->L.part);
  double* dout = (double*)(c->ws + c->L.stats_out);
  ADG_HIP(launch_stats(c->stage_args(), d_u, d_ref, part, (const int32_t*)(c->ws + c->L.first_s), n, dout, c->stream));
  ADG_HIP(hipMemcpyAsync(h_out, dout, 3 * sizeof(double) * n, hipMemcpyDeviceToHost, c->stream));
  ADG_HIP(hipStreamSynchronize(c->stream));
  return ADG_OK;
}

int adg_ensemble_stats(adg_ctx* c, const double* d_u, const double* d_ref, const int32_t* h_group_of,
                       int32_t n_groups, double* h_out) {
  if (!c || !d_u || !d_ref || !h_group_of || !h_out) return fail(ADG_E_INVALID, "null argument");
  if (!state_aligned(d_u) || !state_aligned(d_ref)) return fail(ADG_E_INVALID, "d_u and d_ref must be 16-byte aligned");
  if (int rc = check_live(c)) return rc;
  const int32_t n = (int32_t)c->probs.size();
  if (n_groups < 1 || n_groups > n) return fail(ADG_E_INVALID, "n_groups must be in 1..n_probs");
  std::vector<int32_t> csr(2 * (size_t)n + 1, 0);  // [gstart (n_groups+1) | members (n)]
  std::vector<int32_t> count(n_groups, 0);
  for (int32_t i = 0; i < n; ++i) {
    if (h_group_of[i] < 0 || h_group_of[i] >= n_groups) return fail(ADG_E_INVALID, "group index out of range");
    ++count[h_group_of[i]];
  }
  int32_t* gstart = csr.data();
  int32_t* members = csr.data() + n + 1;
  for (int32_t g = 0; g < n_groups; ++g) gstart[g + 1] = gstart[g] + count[g];
  std::vector<int32_t> fill(gstart, gstart + n_groups);
  for (int32_t i = 0; i < n; ++i) members[fill[h_group_of[i]]++] = i;
  int32_t* d_csr = (int32_t*)(c->ws + c->L.groups);
  double* part = (double*)(c->ws + c->L.part);
  double* pstats = (double*)(c->ws + c->L.stats_out);
  double* gout = (double*)(c->ws + c->L.gstats);
  ADG_HIP(hipMemcpyAsync(d_csr, csr.data(), 4 * csr.size(), hipMemcpyHostToDevice, c->stream));
  ADG_HIP(launch_stats(c->stage_args(), d_u, d_ref, part, (const int32_t*)(c->ws + c->L.first_s), n, pstats,
                       c->stream));
  ADG_HIP(launch_group_stats(pstats, d_csr, d_csr + n + 1, n_groups, gout, c->stream));
  ADG_HIP(hipMemcpyAsync(h_out, gout, 4 * sizeof(double) * n_groups, hipMemcpyDeviceToHost, c->stream));
  ADG_HIP(hipStreamSynchronize(c->stream));
  return ADG_OK;
}

int adg_delay_schedule(const adg_problem* p, int64_t step0, int64_t n_steps, int32_t* h_k) {
  int rc = validate(p, 1);
  if (rc) return rc;
  if (!h_k || step0 < 0 || n_steps < 0) return fail(ADG_E_INVALID, "bad schedule arguments");
  const int S = rk_stages((int)p->rk);
  const int64_t P = p->n_elem / p->pe_size;
  if (P <= 1) return ADG_OK;
  const int q = q_of(*p);
  for (int64_t i = 0; i < n_steps; ++i) {
    const int64_t n = step0 + i;
    for (int s = 0; s < S; ++s) {
      const int key = p->delay_granularity == ADG_DELAY_PER_STAGE ? s : 0;
      for (int64_t b = 0; b < P; ++b) {
        int k = 0;
        if (p->scheme != ADG_SCHEME_DG) {
          k = p->delay_granularity == ADG_DELAY_CAA
                  ? caa_delay(n)
                  : draw_delay(p->seed, n, key, b, p->delay_threshold, (int)p->n_delays);
          k = clamp_delay(k, n, q);
        }
        h_k[(i * S + s) * P + b] = k;
      }
    }
  }
  return ADG_OK;
}

int adg_destroy(adg_ctx* c) {
  if (!c) return ADG_OK;
  drop_graph(c);
  delete c;
  return ADG_OK;
}

}  // extern "C"
