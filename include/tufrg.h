/*
 * tufrg.h - C ABI of the MI355X (gfx950) TUfRG flow right-hand-side library.
 *
 * The library evaluates the increment of the truncated-unity functional
 * renormalization group (TUfRG) for the pairing (P), crossed particle-hole
 * (C) and direct particle-hole (D) exchange propagators of the t-t'
 * Hubbard model in a bond form-factor basis, in the three steps of the
 * paper's Sec. 2.4 list:
 *   i.)  projections of the couplings onto each channel, eqns. proj_VP,
 *        proj_VC, proj_VD (position-space form eqn. proj_pos);
 *   ii.) form-factor projected loops, eqn. chis;
 *   iii.) per-momentum products, eqns. matmul-P, matmul-C, matmul-D;
 * and integrates the flow with an explicit ODE solver (Sec. 3) until the
 * largest exchange propagator exceeds a threshold (Sec. 4).
 *
 * The regulator is the temperature T: loops are T * sum over Matsubara
 * frequencies of G G with G(i w, eps) = 1/(i w - eps), and every
 * derivative is d/dT.  Transfer momenta live on a uniform Lq x Lq grid
 * q_i = 2 pi (i - Lq/2)/Lq per axis (flat index ix*Lq + iy); loops are
 * plain averages over the unshifted uniform Lk x Lk grid p_j = 2 pi j/Lk.
 *
 * Form factors (Sec. 3, footnote on C4v irreps): shells of bond length
 * 0, 1, sqrt2, 2, sqrt5; per shell ordered A1, B1, B2, A2, E:
 *   shell 0: 1
 *   shell 1: cos kx + cos ky, cos kx - cos ky, sqrt2 sin kx, sqrt2 sin ky
 *   shell 2: 2 cos kx cos ky, 2 sin kx sin ky, 2 sin kx cos ky, 2 cos kx sin ky
 *   shell 3: cos 2kx + cos 2ky, cos 2kx - cos 2ky, sqrt2 sin 2kx, sqrt2 sin 2ky
 *   shell 4: sqrt2(cos2kx cos ky + cos kx cos2ky), sqrt2(cos2kx cos ky - cos kx cos2ky),
 *            sqrt2(sin2kx sin ky + sin kx sin2ky), sqrt2(sin2kx sin ky - sin kx sin2ky),
 *            2 sin2kx cos ky, 2 cos kx sin2ky, 2 sin kx cos2ky, 2 cos2kx sin ky
 * giving N_ff = 1, 5, 9, 13, 21 for shells = 0..4.
 *
 * Data layout (all FP64, row-major, device memory owned by the caller):
 *   exchange propagators X  [3][S]   channels (P, C, D)
 *   loops dchi              [2][S]   channels (pp, ph)
 * where, for a context of npts points, S = sum_p Nq_p * Nff_p^2 and the
 * block of point p starts at offset_p (tufrg_layout) and is [Nq][Nff][Nff].
 * Full (not triangular) matrices are stored; no symmetry is assumed.
 *
 * Errors: every call returns a tufrg_status; none aborts.  The message of
 * the last failure is available from tufrg_last_error.  Kernel launches are
 * asynchronous on the context's stream; faults surface at the next
 * synchronising call (tufrg_sync, tufrg_flow).
 *
 * Concurrency: a context belongs to one host thread and one HIP stream.
 * Calls on one context must not overlap.  The step calls (bubbles, project,
 * rhs) allocate nothing; all their workspace is allocated by tufrg_init.
 * tufrg_flow allocates its RK4 step tables the first time a larger nsteps
 * is asked for, and instantiates (then destroys) a HIP graph when use_graph
 * is set.
 */
#ifndef TUFRG_H
#define TUFRG_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  TUFRG_OK = 0,
  TUFRG_EINVAL = -1,       /* invalid argument (message says which) */
  TUFRG_ENOMEM = -2,       /* device allocation failed in tufrg_init */
  TUFRG_EHIP = -3,         /* a HIP runtime call failed */
  TUFRG_ENONFINITE = -4,   /* a non-finite value appeared in the flow state */
  TUFRG_EUNSUPPORTED = -5  /* option combination not available */
} tufrg_status;

/* One model / discretisation point: eps(k) = -2t(cos kx + cos ky)
 * - 4t' cos kx cos ky - mu (eqn. hubb-disp) with onsite interaction U.
 * Requirements: t > 0; Lq even and Lq > 4 * (largest bond component of the
 * truncation: 0 for shells 0, 1 for shells 1-2, 2 for shells 3-4);
 * Lk even and >= 4; shells in 0..4. */
typedef struct {
  double t, tp, mu, U;
  int32_t Lq, Lk, shells;
  int32_t reserved;
} tufrg_point;

enum {
  TUFRG_FP64 = 0,          /* every step in FP64 */
  TUFRG_MIXED = 1          /* loops in FP32 with compensated sums; projections
                              and products with BF16 hi/lo split operands and
                              FP32 accumulation; flow state FP64 */
};

enum {
  TUFRG_NO_CROSS = 1u << 0, /* drop every inter-channel projection term: V^P = U - P,
                               V^C = U + C, V^D = U + D (decoupled channels; a test
                               seam for closed forms, not part of the method) */
  TUFRG_AUTOTUNE = 1u << 1, /* time candidate loop-kernel geometries (row slices per
                               momentum x row chunks per column) for every distinct
                               point shape, then both launch forms of the whole
                               batch, during tufrg_init and keep the fastest;
                               choices are read from and appended to the text file
                               named by the environment variable TUFRG_TUNE_CACHE
                               when it is set.  Results differ from the default
                               geometry only by summation order. */
  TUFRG_LOOP_QUEUE = 1u << 2 /* run the loop kernel as persistent blocks that take
                               work items from a queue (default: one block per work
                               item, items ordered costliest first); bit-identical
                               results.  TUFRG_AUTOTUNE times both forms and keeps
                               the faster, whatever this bit says. */
};

typedef struct {
  int32_t precision;       /* TUFRG_FP64 or TUFRG_MIXED */
  uint32_t flags;          /* TUFRG_NO_CROSS | TUFRG_AUTOTUNE | TUFRG_LOOP_QUEUE */
} tufrg_options;

enum { TUFRG_RK4_LOG = 0, TUFRG_DOPRI5_LOG = 1 };

/* Flow in s = ln T from T0 down to Tmin; dX/ds = T dX/dT.  Stops after the
 * first accepted step with max |X| > Xmax (divergence, Sec. 4). */
typedef struct {
  double T0, Tmin, Xmax;
  int32_t scheme;          /* TUFRG_RK4_LOG: nsteps uniform steps in s.
                              TUFRG_DOPRI5_LOG: Dormand-Prince 5(4), RMS error norm
                              with atol + rtol*max(|y|,|y_new|), step factor
                              0.9 err^(-1/5) in [0.2, 5], first step h0 (0: (ln Tmin
                              - ln T0)/200) */
  int32_t nsteps;
  double rtol, atol, h0;
  int32_t max_steps;       /* DOPRI5 step budget (0: 100000) */
  int32_t use_graph;       /* RK4: capture one step of all points in a HIP graph and
                              replay it (1), or launch every step eagerly (0).  Both
                              give identical results: stage temperatures come from a
                              device table indexed by a device step counter, and a
                              point stops (is skipped by every kernel) at the end of
                              the first step with max|X| > Xmax. */
} tufrg_flow_opts;

enum { TUFRG_FLOW_DIVERGED = 1, TUFRG_FLOW_REACHED_TMIN = 2, TUFRG_FLOW_NONFINITE = 3 };

/* Per-point flow result.  Tc: linear interpolation of ln max|X| in s to
 * ln Xmax between the last two accepted steps (only when DIVERGED).
 * channel 0/1/2 = P/C/D of the largest |X_mn(q)|; q_index its momentum;
 * irrep 0..4 = A1, B1, B2, A2, E of the form factors carrying most weight
 * of the leading eigenvector of that channel's matrix at q_index. */
typedef struct {
  int32_t status;
  int32_t channel, q_index, irrep;
  double Tc, max_abs_X;
  int64_t n_rhs, n_steps;
} tufrg_flow_result;

typedef struct tufrg_ctx tufrg_ctx;

/* Build the scale-independent tables of every point (bonds, form-factor
 * coefficients, harmonic and projection index tables - the reusable part
 * of the projections noted in Sec. 2.5), upload them once, and allocate
 * all workspace.  stream: a hipStream_t, or NULL for the default stream.
 * pts: host array [npts].  On success *out owns device memory until
 * tufrg_free.  Errors: EINVAL (bad point, message names it), ENOMEM, EHIP. */
tufrg_status tufrg_init(const tufrg_point* pts, int32_t npts, const tufrg_options* opt,
                        void* stream, tufrg_ctx** out);

/* Offset (in elements, within one channel), Nq and Nff of point `point`;
 * any output pointer may be NULL.  *total (if non-NULL) receives S. */
tufrg_status tufrg_layout(const tufrg_ctx* ctx, int32_t point, int64_t* offset,
                          int32_t* Nq, int32_t* Nff, int64_t* total);

/* Loop-kernel geometry chosen for point `point` (default heuristic or the
 * autotuner): row slices of the half fine grid per transfer momentum, row
 * chunks per fine-grid column, the block size shared by all points of the
 * context, and the launch form (1: persistent blocks taking work items from
 * a queue; 0: one block per work item, items ordered costliest first).  Any
 * output pointer may be NULL.  Host-only. */
tufrg_status tufrg_geometry(const tufrg_ctx* ctx, int32_t point, int32_t* nsplit,
                            int32_t* nchunk, int32_t* threads, int32_t* persistent);

/* Step ii.): dchi[2][S] = d/dT of the loops chi^pp, chi^ph of eqn. chis at
 * temperature T_host[p] > 0 for every point p.  dchi: device pointer. */
tufrg_status tufrg_bubbles(tufrg_ctx* ctx, const double* T_host, double* dchi);

/* Step i.): V[3][S] = (V^P, V^C, V^D) from X[3][S] (eqns. proj_VP/VC/VD).
 * X, V: device pointers (may not alias). */
tufrg_status tufrg_project(tufrg_ctx* ctx, const double* X, double* V);

/* Steps i.)-iii.): dXdT[3][S] = (dP/dT, dC/dT, dD/dT) at temperatures
 * T_host[p] (eqns. matmul-P/C/D).  X, dXdT: device pointers (no alias). */
tufrg_status tufrg_rhs(tufrg_ctx* ctx, const double* T_host, const double* X, double* dXdT);

/* Integrate the flow for every point; X (device, [3][S]) holds X(T0) on
 * entry and the state at the stop on return.  res: host array [npts].
 * Synchronises the stream.  Returns ENONFINITE if any point's state became
 * non-finite (its result status says NONFINITE too); divergence is a result,
 * not an error. */
tufrg_status tufrg_flow(tufrg_ctx* ctx, const tufrg_flow_opts* opts, double* X,
                        tufrg_flow_result* res);

/* Wait for all work issued on the context's stream; reports kernel faults. */
tufrg_status tufrg_sync(tufrg_ctx* ctx);

/* Number of FP64 (or FP32 in MIXED mode) flops one tufrg_rhs call performs
 * by the library's algorithmic count, per step: out[0] loops, out[1]
 * projections, out[2] products.  Host-only. */
tufrg_status tufrg_flop_count(const tufrg_ctx* ctx, double out[3]);

/* Chemical potential for electron density n (both spins) at temperature T:
 * n = (2/L^2) sum_k n_F(eps_k) on the unshifted L x L grid, by bisection to
 * |dmu| < 1e-13.  Host-only; no context needed.  EINVAL for n outside (0, 2),
 * T <= 0, L < 2. */
tufrg_status tufrg_mu_from_filling(double t, double tp, double n, double T, int32_t L,
                                   double* mu);

/* Release everything tufrg_init allocated.  NULL is ignored. */
void tufrg_free(tufrg_ctx* ctx);

/* Message of the last failing call on ctx (or of the last failing
 * tufrg_init / host-only call when ctx is NULL).  Never NULL. */
const char* tufrg_last_error(const tufrg_ctx* ctx);

#ifdef __cplusplus
}
#endif

#endif /* TUFRG_H */
