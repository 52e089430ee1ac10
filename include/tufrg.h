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
 * The regulator is the temperature T by default: loops are T * sum over
 * Matsubara frequencies of G G with G(i w, eps) = 1/(i w - eps), and every
 * derivative is d/dT.  With TUFRG_OMEGA_CUTOFF it is the Omega cutoff at
 * zero temperature (the regulator the paper's Sec. 3 names for its runs):
 * G(i w, eps) = chi(w)/(i w - eps) with chi(w) = w^2/(w^2 + Omega^2), loops
 * are integrals over real frequencies, every derivative is d/dOmega, and
 * every argument named T below (temperatures, T0, Tmin, Tc) is Omega.
 * With TUFRG_SYMMETRIC_STATE the states are taken to be C4v-symmetric (as
 * every state of a flow started at zero is) and part of the work runs at one
 * transfer momentum per point-group orbit; see the flag.
 * Transfer momenta live on a uniform Lq x Lq grid
 * q_i = 2 pi (i - Lq/2)/Lq per axis (flat index ix*Lq + iy), or on a
 * non-uniform mesh given to tufrg_init_mesh; loops are plain averages over
 * the unshifted uniform Lk x Lk grid p_j = 2 pi j/Lk.
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
 * tufrg_flow allocates its state buffers on its first call, its RK4 step
 * tables the first time a larger nsteps is asked for, and for the adaptive
 * scheme the step-control state and a small pinned, mapped host array of the
 * points' status words (which its control kernel writes, so that the host
 * follows the flow without synchronising the stream each step) on its first
 * adaptive call; it instantiates (then destroys) a HIP graph when use_graph
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
                               point shape alone; with several points, then the
                               slice counts of all points divided by 1, 2, 4, 8 on
                               the whole batch; then both launch forms of the whole
                               batch; during tufrg_init, keeping the fastest.
                               Choices (per shape and per batch of shapes) are read
                               from and appended to the text file named by the
                               environment variable TUFRG_TUNE_CACHE when it is set.
                               Results differ from the default geometry only by
                               summation order. */
  TUFRG_NO_SYMMETRY = 1u << 3, /* integrate the loops at every transfer momentum
                               instead of one representative per C4v orbit (a
                               test seam: the point-group reduction is exact up
                               to rounding) */
  TUFRG_LOOP_QUEUE = 1u << 2, /* run the loop kernel as persistent blocks that take
                               work items from a queue (default: one block per work
                               item, items ordered costliest first); bit-identical
                               results.  TUFRG_AUTOTUNE times both forms and keeps
                               the faster, whatever this bit says. */
  TUFRG_OMEGA_CUTOFF = 1u << 5, /* the flow's scale is the Omega cutoff at T = 0
                               instead of the temperature (see the top of this
                               file); only the loops change.  Not available with
                               a surrogate (tufrg_surrogate_attach returns
                               EUNSUPPORTED). */
  TUFRG_SYMMETRIC_STATE = 1u << 6, /* the caller's states are C4v-symmetric:
                               X(q) = T X(q') T^T whenever an operation h of C4v
                               gives h q = q' + G (G in {0, 2 pi}^2, the zone
                               edge), T being the signed permutation of the form
                               factors with f_m(h^-1 (k - G/2)) = sum_n T_mn f_n(k)
                               (Sec. 3: the lattice symmetries; every state of a
                               flow started at zero is symmetric, and the
                               increment of a symmetric state is).  The inverse
                               transform and the products then run at one
                               transfer momentum per orbit and the results are
                               copied to the rest of the orbit with that law:
                               every member is an exact signed copy of its
                               representative.  For a state that is not
                               symmetric the step calls return its
                               representatives' increments copied by the law:
                               validate states with tufrg_symmetry_defect;
                               tufrg_flow checks its initial state and returns
                               EINVAL when its relative defect exceeds 1e-12. */
  TUFRG_DENSE_PROJECTION = 1u << 7, /* precompute the projections' cross terms as
                               one dense operator per point (the reusable
                               projection data of Sec. 2.5, the stored tensors of
                               the appendix on symmetries): tufrg_init applies the
                               factored projections to every unit state
                               (3 Nq Nff^2 of them) and stores the results, a
                               (3 Nq Nff^2)^2 FP64 matrix; the step calls then
                               replace forward transform, bond basis, gather and
                               inverse transform by one operator product.  Small
                               points only (3 Nq Nff^2 <= 8192, else EINVAL); FP64
                               per-momentum contexts (EUNSUPPORTED with
                               TUFRG_MIXED or TUFRG_SYMMETRIC_STATE).  Results equal
                               the factored path's up to summation order. */
  TUFRG_NO_LOOP_REUSE = 1u << 8, /* flows: evaluate the loops at every stage.  By
                               default a stage at the temperature of the stage
                               just before it (RK4's second and third, RK4's
                               first and the last stage of the step before,
                               Dormand-Prince's sixth and seventh) takes that
                               stage's loops, still in the workspace, instead of
                               evaluating them again (the loops depend on T
                               alone).  Bit-identical results. */
  TUFRG_NO_FUSE = 1u << 4  /* never run the right-hand side in fused launches.  By
                               default a context whose channel state (sum of
                               Nq Nff^2 over its points) is at most 2^18 runs the
                               loops and the projections in shared launches on one
                               stream (small problems are bound by launch and
                               synchronisation cost); larger ones, and every
                               context with this bit, the surrogate or the loop
                               queue, run the loops on a second stream alongside
                               the projections.  Bit-identical results. */
};

typedef struct {
  int32_t precision;       /* TUFRG_FP64 or TUFRG_MIXED */
  uint32_t flags;          /* TUFRG_NO_CROSS | TUFRG_AUTOTUNE | TUFRG_LOOP_QUEUE |
                              TUFRG_NO_SYMMETRY | TUFRG_NO_FUSE | TUFRG_OMEGA_CUTOFF |
                              TUFRG_SYMMETRIC_STATE | TUFRG_DENSE_PROJECTION |
                              TUFRG_NO_LOOP_REUSE */
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
                              - ln T0)/200; otherwise it must be negative, pointing
                              from T0 towards Tmin, else EINVAL) */
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

/* MAX_STEPS: a DOPRI5 flow used up max_steps attempted steps before it
 * diverged or reached Tmin (the state is the last accepted one). */
enum { TUFRG_FLOW_DIVERGED = 1, TUFRG_FLOW_REACHED_TMIN = 2, TUFRG_FLOW_NONFINITE = 3,
       TUFRG_FLOW_MAX_STEPS = 4 };

/* Per-point flow result.  Tc: linear interpolation of ln max|X| in s to
 * ln Xmax between the last two accepted steps (only when DIVERGED).
 * channel 0/1/2 = P/C/D of the largest |X_mn(q)|; q_index its momentum;
 * irrep 0..4 = A1, B1, B2, A2, E of the form factors carrying most weight
 * of the leading eigenvector of that channel's matrix at q_index. */
typedef struct {
  int32_t status;
  int32_t channel, q_index, irrep;
  double Tc, max_abs_X;
  double max_abs_V;   /* max |V| of the point's projected couplings (eqns.
                         proj_VP/VC/VD, as tufrg_project) at the end state */
  int64_t n_rhs, n_steps;
} tufrg_flow_result;

typedef struct tufrg_ctx tufrg_ctx;
typedef struct tufrg_mlp tufrg_mlp;

/* Build the scale-independent tables of every point (bonds, form-factor
 * coefficients, harmonic and projection index tables - the reusable part
 * of the projections noted in Sec. 2.5), upload them once, and allocate
 * all workspace.  stream: a hipStream_t, or NULL for the default stream.
 * pts: host array [npts].  On success *out owns device memory until
 * tufrg_free.  Errors: EINVAL (bad point, message names it), ENOMEM, EHIP. */
tufrg_status tufrg_init(const tufrg_point* pts, int32_t npts, const tufrg_options* opt,
                        void* stream, tufrg_ctx** out);

/* A non-uniform transfer-momentum mesh (Sec. 4: the exchange propagators on
 * an adaptively dense set of momenta, denser where they are expected to
 * peak).  nq momenta (qx[i], qy[i]) in [-pi, pi)^2 with quadrature weights
 * w[i] > 0, the fractions of the zone's area their cells cover (sum 1 to
 * 1e-12); host arrays, copied by the init call.  The loops and the products
 * are evaluated at the mesh momenta; the projections' Fourier coefficients of
 * the gauged exchange propagators (the Fourier series of the appendix on
 * symmetries) are the mesh quadrature
 *   Yhat_{R1R2}(W) = sum_u w_u X_{R1R2}(u) exp(i u.(W - (R1+R2)/2)),
 * which on the uniform Lq grid (w = 1/Lq^2) is the transform tufrg_init uses.
 * The point's Lq names the coarse grid the mesh refines (the same condition
 * Lq > 4 * largest bond component applies).  Flat index: the mesh order. */
typedef struct {
  int32_t nq;              /* 1 .. 65535; 0 selects the uniform Lq x Lq grid */
  const double* qx;
  const double* qy;
  const double* w;
} tufrg_mesh;

/* tufrg_init with a transfer mesh per point (meshes: host array [npts]; an
 * entry with nq = 0, or meshes = NULL, keeps the uniform grid).  A point on a
 * non-uniform mesh integrates its loops at every mesh momentum (no
 * point-group reduction); TUFRG_SYMMETRIC_STATE and the surrogate are not
 * available for it (EUNSUPPORTED).  EINVAL for a mesh outside the zone,
 * non-positive or non-finite weights, or weights not summing to 1. */
tufrg_status tufrg_init_mesh(const tufrg_point* pts, const tufrg_mesh* meshes, int32_t npts,
                             const tufrg_options* opt, void* stream, tufrg_ctx** out);

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

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the same
 * right-hand side as tufrg_rhs (same kernels, same bits), with its
 * workspace (loops, transforms, bond basis, loop harmonics) in a 32 MiB
 * static device array of the library instead of the context's workspace.
 * The call allocates nothing.  EINVAL when the context's workspace exceeds
 * 32 MiB (the message gives the size: at N_ff = 13 on 24x24 it is about
 * 6 MB); EUNSUPPORTED with a surrogate attached.  The array is shared by
 * every context on a device and holds the last call's workspace: calls that
 * overlap on one device (other streams, other host threads) race.  Nothing in
 * it needs to start at zero. */
tufrg_status tufrg_rhs_noalloc(tufrg_ctx* ctx, const double* T_host, const double* X, double* dXdT);

/* Integrate the flow for every point; X (device, [3][S]) holds X(T0) on
 * entry and the state at the stop on return.  res: host array [npts].
 * Synchronises the stream.  Returns ENONFINITE if any point's state became
 * non-finite (its result status says NONFINITE too); divergence is a result,
 * not an error. */
tufrg_status tufrg_flow(tufrg_ctx* ctx, const tufrg_flow_opts* opts, double* X,
                        tufrg_flow_result* res);

/* Largest relative deviation of X (device, [3][S]) from the C4v covariance
 * law of TUFRG_SYMMETRIC_STATE (Sec. 3, the lattice symmetries):
 * *rel = max over points of max|X(q)_mn - s_m s_n X(r)_{pi(m) pi(n)}| / max|X|,
 * the maximum over channels, orbit members q of their representative r and
 * (m, n); 0 for X = 0, NaN for a non-finite state.  A state with *rel below
 * about 1e-12 is symmetric up to rounding.  Synchronises the stream. */
tufrg_status tufrg_symmetry_defect(tufrg_ctx* ctx, const double* X, double* rel);

/* Wait for all work issued on the context's stream; reports kernel faults. */
tufrg_status tufrg_sync(tufrg_ctx* ctx);

/* Number of FP64 (or FP32 in MIXED mode) flops one tufrg_rhs call performs
 * by the library's algorithmic count, per step: out[0] loops, out[1]
 * projections, out[2] products.  Host-only. */
tufrg_status tufrg_flop_count(const tufrg_ctx* ctx, double out[3]);

/* Diagnostic: average duration in microseconds (*us) of the loop kernel
 * alone, from HIP events recorded on the context's stream around `reps`
 * back-to-back launches at temperatures T_host[p] (after one warm-up
 * launch), and its algorithmic flop count per launch (*flops, may be NULL;
 * the loop part of tufrg_flop_count without the chi' expansion).
 * Synchronises the stream. */
tufrg_status tufrg_loop_kernel_time(tufrg_ctx* ctx, const double* T_host, int32_t reps, double* us,
                                    double* flops);

/* Diagnostic: average duration in microseconds of each kernel of the
 * projections (Sec. 2.5: forward transform, bond basis, gather, inverse
 * transform) and of the products (the right-hand side of Sec. 2.4), each
 * measured alone: one right-hand side at temperatures T_host fills the
 * workspace, then per stage `reps` back-to-back launches are captured in a
 * HIP graph on the context's own capture stream (ordered after the
 * caller's), replayed once as warm-up and once between HIP events: the GPU's
 * time per launch, the gap to the next launch included, without the host's
 * launch costs.  Stage i: 0 forward
 * transform, 1 bond basis, 2 gather, 3 inverse transform, 4 products (which
 * write dX/dT into dXdT, device, caller-owned, the size of X; X and dXdT must
 * not alias).  us[i] is that stage's average per launch (the launch and its
 * kernels; several kernels where a stage is launched per class of points),
 * flops[i] (may be NULL) its algorithmic flop count per launch, FMA = 2
 * (parts of tufrg_flop_count's out[1] and out[2]; with symmetric states the
 * inverse transform and the products count the orbit representatives only).
 * TUFRG_EUNSUPPORTED with a surrogate attached, a dense projection operator
 * or TUFRG_NO_CROSS.  Synchronises the stream. */
tufrg_status tufrg_kernel_times(tufrg_ctx* ctx, const double* T_host, const double* X, double* dXdT,
                                int32_t reps, double us[5], double flops[5]);

/* Chemical potential for electron density n (both spins) at temperature T:
 * n = (2/L^2) sum_k n_F(eps_k) on the unshifted L x L grid, by bisection to
 * |dmu| < 1e-13.  Host-only; no context needed.  EINVAL for n outside (0, 2),
 * T <= 0, L < 2. */
tufrg_status tufrg_mu_from_filling(double t, double tp, double n, double T, int32_t L,
                                   double* mu);

/* ---------------------------------------------------------------------
 * Loop harmonics and the learned loop surrogate.
 *
 * With f_m(p) = sum_b c_mb exp(-i p.R_b), the loops of eqn. chis are
 *   chi'_mn(q) = sum_{a,b} c_ma c_nb ghat(q, R_a + R_b),
 *   ghat_X(q, S) = (1/N_k) sum_p dL^X/dT(eps(p+q/2), eps(p-q/2)) cos(p.S),
 * real and even in S, so one value per (q, S) with S in the half set of
 * bonds + bonds (S_x > 0, or S_x = 0 and S_y >= 0; N_S' = 1, 7, 13, 21, 35
 * for shells 0..4) carries the loops of every form-factor pair.
 *
 * The surrogate (not part of the paper) predicts ghat from 9 features
 *   (qx/pi, qy/pi, log10 T, mu/t, t'/t, R_a/2, R_b/2),
 * (R_a, R_b) the canonical bond pair of S (the first pair in the bond
 * order of the form-factor table with R_a + R_b = S), as 4 targets
 *   (T (1 + 4T) ghat_pp, (1 + 4T^2) ghat_ph, 0, 0)
 * (the last two: the imaginary parts, identically zero).
 * ------------------------------------------------------------------- */

/* Half-set harmonics of point `point`: *n receives N_S'; table (if not
 * NULL, host [N_S'][6]) receives (S_x, S_y, R_a,x, R_a,y, R_b,x, R_b,y) per
 * harmonic, the canonical pair included; *offset (if not NULL) the offset
 * of the point in [sum_p Nq_p * 2 * N_S'_p] harmonic arrays. */
tufrg_status tufrg_harmonics(const tufrg_ctx* ctx, int32_t point, int32_t* n, int32_t* table,
                             int64_t* offset);

/* ghat (device, [sum_p Nq_p][2][N_S'_p] per point block, channels pp, ph)
 * at temperatures T_host[p], from the exact FP64 loop kernel.  FP64
 * contexts only (EUNSUPPORTED otherwise). */
tufrg_status tufrg_loop_harmonics(tufrg_ctx* ctx, const double* T_host, double* ghat);

/* n training samples of the surrogate drawn uniformly over (point, q, S)
 * with a counter-based hash of (seed, sample index), labels from the exact
 * FP64 loop kernel at T_host[p]: x (device float [n][9]) features, y
 * (device float [n][4]) targets, idx (device int32 [n][3] or NULL) the
 * (point, q, harmonic) of each sample.  FP64 contexts only. */
tufrg_status tufrg_surrogate_dataset(tufrg_ctx* ctx, const double* T_host, int64_t n, uint64_t seed,
                                     float* x, float* y, int32_t* idx);

/* Route the loops of tufrg_bubbles, tufrg_rhs and tufrg_flow through one or
 * two surrogate networks (9 inputs, 4 outputs) with an exact fallback, or
 * detach (a = b = NULL).  Per call, momentum q takes the exact loop kernel
 * when the networks' predicted harmonics differ by more than
 * tol * max_S |prediction at q| (two networks only), when q = phase (mod
 * check_stride) with the phase advancing by one per call, or while q is
 * flagged; a checked q whose prediction misses the exact harmonics by more
 * than tol * max_S |exact| is flagged together with its 8 neighbours, and a
 * later passing check clears the flag.  With b = NULL (one network, half the
 * inference cost) acceptance rests on the rotating check and the flags.
 * Either way a prediction is verified at most check_stride calls before it
 * is used: predictions that are wrong everywhere are all flagged within
 * check_stride calls, but in between they are used unverified.  Single-point FP64 contexts only (EUNSUPPORTED otherwise).  The
 * networks must outlive the attachment and are used on the context's
 * streams.  Allocates the surrogate's buffers. */
tufrg_status tufrg_surrogate_attach(tufrg_ctx* ctx, tufrg_mlp* a, tufrg_mlp* b, double tol,
                                    int32_t check_stride);

/* Cumulative surrogate counters since the attachment: out[0] momenta
 * evaluated exactly, out[1] momenta queried, out[2] failed checks.
 * Synchronises the stream. */
tufrg_status tufrg_surrogate_stats(tufrg_ctx* ctx, int64_t out[3]);

/* Release everything tufrg_init allocated.  NULL is ignored. */
void tufrg_free(tufrg_ctx* ctx);

/* Message of the last failing call on ctx (or of the last failing
 * tufrg_init / host-only call when ctx is NULL).  Never NULL. */
const char* tufrg_last_error(const tufrg_ctx* ctx);

/* ---------------------------------------------------------------------
 * Multilayer perceptron (the surrogate's network; not part of the paper).
 *
 * Layers l = 1..L: z_l = a_{l-1} W_l^T + b_l, a_l = silu(z_l) = z_l
 * sigmoid(z_l) on hidden layers, a linear output.  Loss: mean over all
 * rows and outputs of (a_L - y)^2.  Matrix products run on the matrix cores
 * with FP32 accumulation: forward products with BF16 hi/lo split operands
 * (about 16 mantissa bits), gradient products with plain BF16 operands;
 * parameters and Adam moments are FP32.  Flat parameter layout: per layer
 * W_l [out][in] row-major, then b_l [out].  All arrays are device memory,
 * row-major [rows][width].  Calls are asynchronous on the network's stream
 * unless stated otherwise.
 * ------------------------------------------------------------------- */

/* widths [nwidths] (input, hidden..., output), each 1..4096; max_rows: the
 * largest batch of tufrg_mlp_gradient / tufrg_mlp_train and the chunk size
 * of tufrg_mlp_forward.  Weights Glorot-uniform from a SplitMix64 counter
 * hash of (seed, parameter index), biases zero.  Synchronises. */
tufrg_status tufrg_mlp_create(const int32_t* widths, int32_t nwidths, int32_t max_rows, uint64_t seed,
                              void* stream, tufrg_mlp** out);
tufrg_status tufrg_mlp_nparams(const tufrg_mlp* net, int64_t* count);
/* copy the FP32 parameters to / from a device array [nparams] */
tufrg_status tufrg_mlp_get_params(tufrg_mlp* net, float* dst);
tufrg_status tufrg_mlp_set_params(tufrg_mlp* net, const float* src);
/* y [rows][out] = network(x [rows][in]) */
tufrg_status tufrg_mlp_forward(tufrg_mlp* net, const float* x, float* y, int64_t rows);
/* loss and gradient (device [nparams], may be NULL) of rows <= max_rows
 * samples; *loss (host, may be NULL) synchronises. */
tufrg_status tufrg_mlp_gradient(tufrg_mlp* net, const float* x, const float* y, int64_t rows,
                                float* grad, double* loss);
/* `steps` Adam steps (beta1 0.9, beta2 0.999, eps 1e-8; learning rate lr
 * with cosine decay to lr/100 over the call) on minibatches of `batch`
 * rows drawn with replacement from (x, y) [rows] by a counter hash of
 * (seed, step, row); loss_hist (host [steps] or NULL) receives each step's
 * minibatch loss.  Synchronises. */
tufrg_status tufrg_mlp_train(tufrg_mlp* net, const float* x, const float* y, int64_t rows, int32_t steps,
                             int32_t batch, float lr, uint64_t seed, double* loss_hist);
void tufrg_mlp_free(tufrg_mlp* net);
const char* tufrg_mlp_last_error(const tufrg_mlp* net);

#ifdef __cplusplus
}
#endif

#endif /* TUFRG_H */
