/*
 * adg.h -- C ABI of the MI355X (gfx950) asynchronous discontinuous Galerkin
 * stepper with asynchrony-tolerant (AT) fluxes.
 *
 * Method: Goswami & Aditya, "An asynchronous discontinuous Galerkin method
 * for massively parallel PDE solvers", arXiv 2404.03399.
 *   - u_t + f(u)_x = 0 on a periodic interval (Sec. 2, model problem);
 *     f = a u (linear advection) or f = u^2/2 (inviscid Burgers); and the
 *     viscous Burgers equation u_t + (u^2/2)_x = nu u_xx of Sec. 6 in local
 *     DG form (q = u_x; alternating fluxes: u-hat from the left element, q-hat
 *     from the right; LLF for u^2/2; AT at PE faces on both face values).
 *   - N_E uniform elements, nodal Lagrange basis of degree N_p on
 *     Gauss-Lobatto-Legendre nodes, exact mass matrix (Sec. 2, element-wise
 *     weak form and reference matrices).
 *   - The elements are split into P = n_elem / pe_size processing elements
 *     (PEs); only the P faces between PEs see delayed data (Sec. 2 parallel
 *     implementation, Sec. 3).
 *   - Delays k in {0..L-1} with probabilities p_k are emulated by a
 *     counter-based draw (Sec. 6.1 delay emulation): one draw per PE
 *     boundary per step (or per RK stage), SplitMix64 chained over
 *     (seed, step, stage key, boundary), 53-bit uniform, binned by
 *     integer thresholds.
 *   - Conservative ADG: both neighbours use the flux of the common delayed
 *     level (Sec. 4.1).  ADG-AT: flux = sum_{j<q} c_j(k) F^{n-k-j} with the
 *     AT coefficients of Sec. 5 / Table 1 (q = N_p + 1 by default).
 *
 * Conventions
 *   - Every call returns an int status (adg_status); nothing throws or aborts
 *     across the ABI.  adg_last_error() returns a thread-local message.
 *   - The library never allocates device memory.  All device buffers (state,
 *     workspace, adjoint outputs) are caller-owned; the workspace must stay
 *     alive and untouched until adg_destroy.
 *   - Work is enqueued on the caller's HIP stream and the call returns
 *     without synchronising (except adg_run with ADG_RUN_CHECK_FINITE and
 *     adg_adjoint's final scalar read, which synchronise the stream).  A kernel
 *     fault surfaces as ADG_E_HIP from a later call or from the caller's own
 *     stream synchronisation.
 *   - State layout: structure of arrays per problem.  Problem i owns
 *     u[offset_i + j * ld_i + e], node plane j in [0, degree], element
 *     e in [0, n_elem); ld_i = n_elem rounded up to 64.  Padding entries are
 *     never read; their contents after a stepping call are unspecified.
 *     Offsets/lds come from adg_state_layout.
 *   - A context is not thread-safe.  All problems of one context advance
 *     together and must share equation, flux, rk and scheme; degree, mesh,
 *     PE size, delays, seed, speed and dt may differ (batched ensembles).
 *     Each problem of a batch advances bitwise as in a context of its own.
 */
#ifndef ADG_H
#define ADG_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define ADG_ABI_VERSION 2

enum adg_status {
  ADG_OK = 0,
  ADG_E_INVALID = -1,      /* bad argument or unsupported combination           */
  ADG_E_ABI = -2,          /* adg_problem.abi_version != ADG_ABI_VERSION        */
  ADG_E_WORKSPACE = -3,    /* workspace missing, too small or misaligned        */
  ADG_E_HIP = -4,          /* a HIP runtime call failed                         */
  ADG_E_STATE = -5,        /* call sequence invalid (e.g. adjoint w/o record)   */
  ADG_E_NONFINITE = -6,    /* ADG_RUN_CHECK_FINITE found a NaN/Inf              */
  ADG_E_UNSUPPORTED = -7   /* valid request the library does not implement     */
};

/* VISCOUS_BURGERS: the fused kernel (local DG form, Sec. 7) runs one, two or
 * four elements per lane and one or two steps per launch; the per-stage
 * kernels run it too; adjoint recording returns ADG_E_UNSUPPORTED. */
enum adg_equation { ADG_EQ_ADVECTION = 0, ADG_EQ_BURGERS = 1, ADG_EQ_VISCOUS_BURGERS = 2 };
enum adg_scheme { ADG_SCHEME_DG = 0, ADG_SCHEME_ADG = 1, ADG_SCHEME_ADG_AT = 2 };
/* upwind / central: f^ = a (B+ u- + B- u+) (Sec. 2);  llf: local Lax-Friedrichs
 * 1/2 (f(u-) + f(u+)) - lambda/2 (u+ - u-), lambda = max(|u-|, |u+|) (Sec. 6.1). */
enum adg_flux { ADG_FLUX_UPWIND = 0, ADG_FLUX_CENTRAL = 1, ADG_FLUX_LLF = 2 };
/* Heun RK2 as in Sec. 4.2.1; Shu-Osher SSP-RK3; classical RK4; and two
 * 2N-storage schemes of the low-storage family of Sec. 6.1,
 * dU_s = A_s dU_{s-1} + dt L(U_{s-1}), U_s = U_{s-1} + B_s dU_s:
 * Williamson's three-stage third-order scheme (1980),
 * A = (0, -5/9, -153/128), B = (1/3, 15/16, 8/15), and Carpenter & Kennedy's
 * five-stage fourth-order scheme (1994) with its published coefficients. */
enum adg_rk { ADG_RK2_HEUN = 0, ADG_SSPRK3 = 1, ADG_RK4 = 2, ADG_LSRK3 = 3, ADG_LSRK4 = 4 };
/* PER_STEP / PER_STAGE: random delays drawn per step or per (step, stage);
 * CAA: the deterministic communication-avoiding cycle of Sec. 7 (of every five
 * steps the first two synchronise, the next three do not): delays
 * (0, 0, 0, 1, 2) by step mod 5 at every PE face, thresholds and seed ignored,
 * n_delays must be 3. */
enum adg_delay_granularity { ADG_DELAY_PER_STEP = 0, ADG_DELAY_PER_STAGE = 1, ADG_DELAY_CAA = 2 };
/* Kernel family: one launch per RK stage with the RK registers in HBM, or one
 * launch per time step with all stages kept on chip (halo recompute). */
enum adg_kernel { ADG_KERNEL_AUTO = 0, ADG_KERNEL_STAGE = 1, ADG_KERNEL_FUSED = 2 };

#define ADG_RUN_GRAPH 1u         /* capture the step loop in a hipGraph and replay it */
#define ADG_RUN_RECORD 2u        /* keep checkpoints for adg_adjoint (run must start at step 0) */
#define ADG_RUN_CHECK_FINITE 4u  /* fail with ADG_E_NONFINITE if the final state has NaN/Inf */

/* One problem (plain data, copied by adg_init). */
typedef struct adg_problem {
  uint32_t abi_version;        /* = ADG_ABI_VERSION */
  uint32_t equation;           /* adg_equation */
  uint32_t scheme;             /* adg_scheme */
  uint32_t flux;               /* adg_flux: upwind/central need advection, llf needs (viscous) Burgers */
  uint32_t rk;                 /* adg_rk */
  uint32_t degree;             /* N_p in 1..4 */
  uint32_t at_levels;          /* q of the AT flux, 1..5; 0 -> degree + 1; must be 0 unless ADG-AT */
  uint32_t n_delays;           /* L in 1..8 (delays 0..L-1) */
  uint32_t delay_granularity;  /* adg_delay_granularity */
  uint32_t reserved;           /* must be 0 */
  int64_t n_elem;              /* N_E >= 2 */
  int64_t pe_size;             /* elements per PE, divides n_elem; P = n_elem / pe_size; P == 1: no PE faces */
  uint64_t seed;               /* delay-stream seed */
  uint64_t delay_threshold[7]; /* L-1 non-decreasing cut-offs T_1..T_{L-1} <= 2^53 on the 53-bit uniform;
                                  delay = #{k : U >= T_k}; unused entries ignored */
  double x_left;               /* left end of the periodic interval */
  double length;               /* interval length (> 0) */
  double speed;                /* advection speed a (advection only; != 0) */
  double dt;                   /* fixed time step (> 0) */
  double viscosity;            /* nu >= 0 of the viscous Burgers equation; must be 0 otherwise */
} adg_problem;

typedef struct adg_options {
  int64_t ckpt_every;          /* adjoint checkpoint interval C in steps; 0 -> 64.  The recording keeps
                                  ceil(n_steps_record / C) states and adg_adjoint recomputes each segment
                                  once; C = 1 keeps every state (fused kernel: each recorded step writes
                                  straight into its slot, and the adjoint recomputes nothing) */
  int32_t kernel;              /* adg_kernel; AUTO -> FUSED */
  int32_t lane_elems;          /* fused kernel: consecutive elements per lane, 1, 2 or 4 (<= every
                                  asynchronous problem's pe_size); 0 -> 2, or 1 for a PE size of 1 */
  uint32_t flags;              /* ADG_OPT_* bits, 0 = defaults */
  uint32_t fused_steps;        /* fused kernel: time steps per launch, 1 or 2 (halo of 2S elements per side,
                                  half the state traffic per step); 0 -> 2.  Every (lane_elems,
                                  fused_steps) pair gives bitwise the same results. */
} adg_options;

/* adg_options.flags.  Fused kernel, PE-face split (only PE faces see
 * delayed data, Secs. 3, 5): within one launch, tile waves without any
 * PE-face handling advance every tile, and window waves recompute windows of
 * 4 K S elements around each PE face (K steps per launch, S stages), owning
 * the 2 K S elements that the face's delayed flux can reach, which the tile
 * waves leave alone; the result is bitwise that of the unsplit kernel.  By default the split is
 * used when a wave holds at least two windows of the longest launch and
 * every asynchronous problem's PE size holds four (RK4 with two steps per
 * launch: PE size >= 128); ADG_OPT_PE_SPLIT_OFF never splits,
 * ADG_OPT_PE_SPLIT_ON splits whenever the PE sizes hold one window.  Bits
 * other than those defined here: ADG_E_INVALID. */
#define ADG_OPT_PE_SPLIT_OFF 1u
#define ADG_OPT_PE_SPLIT_ON 2u
/* ADG_OPT_ONE_LAUNCH: the fused kernel advances every problem of a batch in
 * one launch per step batch instead of one launch per degree range (Sec. 4.3
 * ensembles mix degrees): each wave takes its range's tile with the PE-face
 * paths compiled in, so every range runs at the register footprint of the
 * degree-4 tile; the results are bitwise those of the per-range launches.
 * Needs the fused kernel with lane_elems 0 or 2 and no PE-face split
 * (together with ADG_OPT_PE_SPLIT_ON: ADG_E_INVALID); viscous Burgers:
 * ADG_E_UNSUPPORTED. */
#define ADG_OPT_ONE_LAUNCH 4u

typedef struct adg_ctx adg_ctx;  /* opaque, host side, library owned */

/* Returns ADG_ABI_VERSION. */
int adg_abi_version(void);

/* Thread-local description of the last failure in this thread ("" if none). */
const char* adg_last_error(void);

/* Identity of the library binary: a hash of its source files (kernels,
 * host code and this header), fixed when the library is compiled, so that a
 * caller can refuse a library built from other sources.  Static string. */
const char* adg_build_id(void);

/* Nodes of the reference element [-1, 1] of the Lagrange basis (Sec. 2,
 * reference element and basis; Gauss-Lobatto-Legendre points, end points
 * included) for the given degree (1..4): writes degree+1 doubles to host
 * array xi.  Lets callers build nodal initial data (the DOFs are nodal
 * values, Sec. 2) u[j*ld+e] = u0(x_left + e*dx + (xi[j]+1)*dx/2).
 * ADG_E_INVALID for another degree or a null xi. */
int adg_nodes(int32_t degree, double* xi);

/* Layout of the state vector for n_probs problems (the nodal DOFs u^e_j of
 * every element, Sec. 2): per-problem offsets and leading dimensions (host
 * arrays of n_probs int64, caller-owned), and the total number of doubles
 * the caller must allocate on the device.  ADG_E_INVALID for an invalid
 * problem (see adg_init). */
int adg_state_layout(const adg_problem* probs, int32_t n_probs, int64_t* offsets, int64_t* lds,
                     int64_t* total_doubles);

/* Device workspace bytes needed by adg_init for these problems, options and
 * an adjoint recording horizon of n_steps_record steps (0 if adg_adjoint
 * is not used): descriptors, work lists, the per-PE-boundary rings of past
 * face fluxes (depth L + q levels, Secs. 3, 5), the fused kernel's second
 * state, and with a horizon the checkpoints.  Host-only; ADG_E_INVALID for
 * invalid problems or options. */
int adg_workspace_size(const adg_problem* probs, int32_t n_probs, const adg_options* opt,
                       int64_t n_steps_record, int64_t* bytes_out);

/* Set up the problem statement: u_t + f(u)_x = 0 on a periodic interval
 * split into n_elem elements (Sec. 2, model problem and mesh), grouped into
 * P = n_elem / pe_size processing elements (Sec. 2 parallel implementation,
 * Sec. 3), with delays k < L drawn with probabilities p_k (Sec. 6.1) and a
 * fixed time step.  Validates the problems, builds the reference operators
 * (Sec. 2), the AT coefficient table (Sec. 5, Table 1) and the tile work
 * lists on the host, uploads them into the caller's device workspace
 * (256-byte aligned, >= adg_workspace_size bytes; caller-owned, untouched
 * by the caller until adg_destroy) on hip_stream (a hipStream_t, NULL =
 * default stream) and clears the step counter and delay history.
 * n_steps_record must match the value given to adg_workspace_size.  On
 * success *out owns a host-side context.  Errors: ADG_E_INVALID (see the
 * field comments of adg_problem / adg_options), ADG_E_ABI,
 * ADG_E_WORKSPACE (missing, small or misaligned workspace),
 * ADG_E_UNSUPPORTED, ADG_E_HIP. */
int adg_init(adg_ctx** out, const adg_problem* probs, int32_t n_probs, const adg_options* opt,
             int64_t n_steps_record, void* d_workspace, int64_t workspace_bytes, void* hip_stream);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): adg_init
 * with no recording horizon (n_steps_record = 0) whose workspace is a
 * file-scope static device array of the library, ADG_SCRATCH_BYTES bytes
 * (64 MiB) per GPU, held from first use until the process ends.  No device
 * memory is allocated or freed by this call; the caller still owns the state
 * vectors.  Problems whose workspace (adg_workspace_size with
 * n_steps_record = 0) exceeds the array are rejected with ADG_E_WORKSPACE
 * before any device call.  One array per GPU: a later adg_init_scratch on
 * the same device takes it over, after which every call on the earlier
 * context except adg_step_count and adg_destroy returns ADG_E_STATE; calls
 * that overlap in time on one GPU (several threads or streams) race on the
 * array.  The step counter, rings and records are cleared as by adg_init.
 * adg_run with ADG_RUN_GRAPH creates a capture stream and a graph; run
 * without that flag when nothing may be created. */
#define ADG_SCRATCH_BYTES (64ll << 20)
int adg_init_scratch(adg_ctx** out, const adg_problem* probs, int32_t n_probs, const adg_options* opt,
                     void* hip_stream);

/* Back to t = 0 (Sec. 2 problem statement): step counter := 0, delay
 * history (rings, Sec. 3) := 0, recorded checkpoints dropped.  Enqueued on
 * the context's stream.  ADG_E_INVALID for a null context. */
int adg_reset(adg_ctx* ctx);

/* Number of steps taken since init/reset (host mirror of the device step
 * counter that keys the delay draws of Sec. 6.1).  ADG_E_INVALID for null
 * arguments. */
int adg_step_count(const adg_ctx* ctx, int64_t* steps);

/* One RK time step of every problem, in place on the device state d_u:
 * adg_run with n_steps = 1 and no flags (see there). */
int adg_step(adg_ctx* ctx, double* d_u);

/* n_steps RK time steps in place on d_u (device, state layout, 16-byte
 * aligned): the RK stages of Sec. 4.2.1 (and the integrators of adg_rk) with
 * the element update of Sec. 2, PE faces reading the AT combination of
 * delayed levels (Secs. 4.1, 5), delays drawn as in Sec. 6.1.  flags:
 * ADG_RUN_GRAPH (steps in batches of 16 replayed from a hipGraph captured
 * for this d_u on first use; with n_steps = 0 the graph is only captured, so
 * that a later timed run replays it without capture cost), ADG_RUN_RECORD
 * (the context must be at step 0 and n_steps <= the recording horizon given
 * to adg_init), ADG_RUN_CHECK_FINITE.  Errors: ADG_E_INVALID (null or
 * misaligned d_u, n_steps < 0, step index past 2^31 - 1, unknown flags),
 * ADG_E_STATE (recording misuse), ADG_E_HIP, ADG_E_NONFINITE. */
int adg_run(adg_ctx* ctx, double* d_u, int64_t n_steps, uint32_t flags);

/* Discrete adjoint (not in the paper: the target's differentiation
 * addition) of the recorded run of the scheme of Secs. 2-5 (delay schedule
 * held fixed) for
 * J(u(T)) with cotangent d_cot_uT = dJ/du(T) (device, state layout).
 * Writes dJ/du(0) to d_grad_u0 (device, state layout) and, for advection,
 * dJ/da per problem to the host array h_grad_speed (n_probs doubles; dt is
 * held fixed; 0 for Burgers).  h_grad_speed may be NULL: for linear
 * advection the reverse sweep then skips the forward recomputation, which
 * only dJ/da needs, and with fused_steps = 2 reverses two steps per launch;
 * dJ/du(0) is bitwise the same either way.  Requires the last adg_run to have used ADG_RUN_RECORD;
 * the recording stays valid (the adjoint may be called again) and the
 * context may keep stepping afterwards.  Synchronises the stream when
 * h_grad_speed is given. */
int adg_adjoint(adg_ctx* ctx, const double* d_cot_uT, double* d_grad_u0, double* h_grad_speed);

/* Per-problem error statistics against a reference state (same layout;
 * Sec. 6.2 measures the error as the mean absolute pointwise error):
 * for each problem i writes h_out[3*i + 0] = mean |u - ref| over all nodal
 * values, h_out[3*i + 1] = max |u - ref|, h_out[3*i + 2] = (dx/2) sum_e w^T u^e
 * (the discrete integral).  Deterministic (fixed reduction order).
 * Synchronises the stream. */
int adg_error_stats(adg_ctx* ctx, const double* d_u, const double* d_ref, double* h_out);

/* Ensemble statistics over groups of problems (Sec. 4.3: spatial average
 * <E> = mean |u - ref| over all nodal values of a problem, and its ensemble
 * average over realizations).  h_group_of[i] in [0, n_groups) assigns
 * problem i to a group (e.g. one mesh, many delay realizations).  For each
 * group g writes h_out[4*g + 0] = mean of <E> over the group,
 * h_out[4*g + 1] = population variance of <E>, h_out[4*g + 2] = mean of
 * max |u - ref|, h_out[4*g + 3] = its population variance.  Two-pass,
 * fixed summation order (deterministic).  Synchronises the stream. */
int adg_ensemble_stats(adg_ctx* ctx, const double* d_u, const double* d_ref, const int32_t* h_group_of,
                       int32_t n_groups, double* h_out);

/* Host-side delay schedule of one problem (Sec. 6.1 delay emulation, or the
 * Sec. 7 communication-avoiding cycle; same integers the kernels use; the
 * start-up clamp k <= n - q + 1 applied):
 * h_k[((n - step0) * S + s) * P + b] = clamped delay at step n, RK stage s,
 * boundary b, for n in [step0, step0 + n_steps).  S = number of RK stages,
 * P = number of PEs (P == 1: nothing written); h_k is caller-owned host
 * memory of n_steps * S * P int32.  ADG_E_INVALID for an invalid problem or
 * arguments. */
int adg_delay_schedule(const adg_problem* prob, int64_t step0, int64_t n_steps, int32_t* h_k);

/* Release the context (host memory and hipGraphs).  The workspace may be
 * freed afterwards; a null context is accepted. */
int adg_destroy(adg_ctx* ctx);

#ifdef __cplusplus
}
#endif

#endif /* ADG_H */
