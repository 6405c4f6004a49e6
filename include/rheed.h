/*
 * rheed.h -- C ABI of the MI355X (gfx950) many-beam RHEED/TRHEPD library.
 *
 * Method: Kudo, Yamamoto, Hoshi, "A fast and accurate computation method for
 * reflective diffraction simulations" (arXiv 2306.00271).  The coupled-beam
 * equation c'' = -(U(z) + Gamma^2) c (Sec. 2.1, Eq. sch3) is written as the
 * matrix ODE Z' = B(z) Z in economical form (Sec. 3.1, Eq. ode2, Eq. mateq2),
 * stepped slice by slice with an explicit Runge-Kutta method (Sec. 3.4) and
 * the right-hand-side transformation Z <- Z Q^{-1} whenever the Gershgorin
 * condition estimate of the upper block exceeds a threshold (Sec. 3.2,
 * Algorithm 1); the reflected amplitudes follow from Eq. (vrhocomp) and the
 * intensities from the formula at the end of Sec. 2.1.
 *
 * Conventions for every entry point:
 *  - All numbers are IEEE FP64.  Complex values are {double re, im}
 *    interleaved (the layout of hipDoubleComplex and torch.complex128).
 *  - Pointers documented "device" must be device memory of the current HIP
 *    device; "host" pointers are read during the call only.  The caller owns
 *    every buffer; the library allocates only inside rheed_plan_create.
 *  - Calls that take a `stream` (a hipStream_t, NULL = default stream) are
 *    asynchronous with respect to the host and enqueue all their work on that
 *    stream.  They do not synchronise and do not allocate.
 *  - Invalid arguments return RHEED_E_INVALID before anything is enqueued;
 *    a failing HIP call returns RHEED_E_HIP.  rheed_last_error() then holds a
 *    message for the calling thread.
 *  - Numerical failure of one (structure, angle) pair never fails the call:
 *    that pair's outputs are NaN and its entry in pair_status says why.
 *  - There is no CPU fallback: on a machine without a gfx950 device every
 *    compute entry point returns RHEED_E_HIP.
 */
#ifndef RHEED_H
#define RHEED_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  RHEED_OK = 0,
  RHEED_E_INVALID = -1,
  RHEED_E_HIP = -2,
  RHEED_E_NOMEM = -3,
  RHEED_E_UNSUPPORTED = -4
} rheed_status;

/* per-pair status codes written to pair_status[] */
enum {
  RHEED_PAIR_OK = 0,
  RHEED_PAIR_SINGULAR = 1,  /* an exactly zero pivot in a right division */
  RHEED_PAIR_NONFINITE = 2, /* Inf/NaN reached the reflected amplitudes */
  RHEED_PAIR_SYNC = 3,      /* split launch: the two workgroups of the pair lost contact */
  RHEED_PAIR_BREAKDOWN = 4  /* the final solve (Gamma Q - iP) x = e_1 is numerically singular:
                               ||B||_inf ||x||_inf > 1e14 (a lower bound of its condition number),
                               as when the state's columns have collapsed onto one mode */
};

/* Steppers (Sec. 3.4): the explicit RK tableaux (classical 4th order, 4
 * stages; Butcher's 6th-order 7-stage method) and splitting methods, which
 * alternate kicks c' -= h b (U(tau) + Gamma^2) c and drifts c += h a c'.
 * The splitting methods are compositions of Stormer-Verlet steps of lengths
 * alpha_k: fourth order, the triple jump g1, 1 - 2 g1, g1 with
 * g1 = 1 / (2 - 2^(1/3)); sixth order, the triple jump of that step with
 * w1 = 1 / (2 - 2^(1/5)), w0 = 1 - 2 w1 (nine steps w_i g_j).  In the BAB
 * form (RHEED_SP4, RHEED_SP6) the drifts are alpha_k and the kicks their half
 * sums, with the first kick at the slice start and the last at its end; in
 * the ABA form (RHEED_SP4_ABA, RHEED_SP6_ABA) the kicks are alpha_k, the
 * drifts their half sums.  Each kick uses the potential at the position the
 * drifts before it have reached; the node tables of a splitting stepper sit
 * at those positions (3 per slice for the fourth-order methods, 9 for the
 * sixth-order ones; positions may lie outside the slice).  Splitting
 * steppers run on the one-workgroup layout, with state saving and
 * rheed_backward for N <= 64 (no bulk start); for N > 64 only RHEED_SP4,
 * forward only. */
typedef enum {
  RHEED_RK4 = 0,
  RHEED_RK6 = 1,
  RHEED_SP4 = 2,
  RHEED_SP6 = 3,
  RHEED_SP4_ABA = 4,
  RHEED_SP6_ABA = 5
} rheed_stepper;

/* Intensity normalisation (Sec. 2.1): FLUX = |rho_j|^2 Gamma_0/Gamma_j on
 * open beams; PAPER = the printed formula, FLUX times sin(theta0). */
typedef enum { RHEED_INTENSITY_FLUX = 0, RHEED_INTENSITY_PAPER = 1 } rheed_convention;

/* Largest beam count N the kernels of this library handle.  Structures with
 * N <= 64 run on the one- or two-workgroup kernels; structures with
 * 64 < N <= 128 run on a kernel that keeps the state of a pair in device
 * memory owned by the plan.  Both have the adjoint (RK steppers, FP64).
 * Structures with 128 < N <= 256 run on a third kernel, also with the state
 * in plan-owned memory, which streams the rows of its eliminations through
 * that memory: RK steppers, FP64, with the adjoint.  Structures with
 * 256 < N <= 576 (the paper's single-angle size, Sec. 4) run on a fourth,
 * each pair on a cooperative group of workgroups that step its column blocks
 * side by side: RK steppers, FP64, forward only; a batch larger than the
 * device holds at once runs in several launches. */
#define RHEED_MAX_BEAMS 576
/* Largest potential-table row (rod differences) for N <= 64, for
 * 64 < N <= 128, for 128 < N <= 256 and for 256 < N <= 576. */
#define RHEED_MAX_BOX 300
#define RHEED_MAX_BOX_LARGE 1024
#define RHEED_MAX_BOX_XL 1536
#define RHEED_MAX_BOX_XXL 4096

/* One slab.  Rod indices are on the reciprocal basis b1, b2:
 * k_j = h_j b1 + k_j b2 (Sec. 2.1, the reciprocal rods k_j with k_1 = 0). */
typedef struct {
  int32_t n_beams;          /* N, 1..RHEED_MAX_BEAMS */
  const int32_t* beam_hk;   /* host [N][2] (h, k); beam 0 must be (0, 0) */
  double recip[4];          /* b1x, b1y, b2x, b2y in 1/A */
  int32_t n_slices;         /* L >= 1; slice i spans [-D + i h, -D + (i+1) h], h = D/L */
  double thickness;         /* D > 0 in A: the slab is z in [-D, 0] (z_e = -D) */
  double wavenumber;        /* gamma in 1/A (see rheed_beam_constants) */
  /* Potential model, used by rheed_potential / rheed_potential_backward only:
   * atoms with v(r) = sum_m a_m exp(-b_m |r - r_a|^2) volts, rescaled so the
   * slab average is mean_inner_potential, times kappa (charge - i absorption). */
  int32_t n_atoms;
  double cell_area;         /* A^2 of the (super)cell */
  double scat_a[4];         /* V */
  double scat_b[4];         /* 1/A^2, > 0 */
  double kappa;             /* 1/(A^2 V) */
  double charge;            /* +1 electron, -1 positron */
  double absorption;        /* alpha >= 0 */
  double mean_inner_potential; /* V */
} rheed_structure;

/* How rheed_forward lays pairs out on the GPU.  SPLIT runs each pair on two
 * workgroups (two CUs) that own 32 columns of the state each and exchange
 * through memory the data that couples the columns; it needs both workgroups
 * of every pair resident at once, so it holds at most one pair per two CUs
 * (rheed_plan_info.split_max_pairs).  WHOLE runs a pair on one workgroup.
 * AUTO picks SPLIT when the batch fits, WHOLE otherwise.  The results of the
 * two layouts agree to rounding.  For structures with N > 128, WHOLE keeps
 * one workgroup per pair; AUTO and SPLIT give a batch that cannot fill the
 * device a group of workgroups per pair (rheed_plan_info.xl_group). */
typedef enum { RHEED_LAYOUT_AUTO = 0, RHEED_LAYOUT_WHOLE = 1, RHEED_LAYOUT_SPLIT = 2 } rheed_layout;

/* Precision of the RK stage products U X (the paper's Sec. 6 names single
 * and half precision as future work): FP64, or FP32 on the FP32 matrix
 * cores (v_mfma_f32_16x16x4f32) with the operands rounded to FP32 and
 * everything else in FP64 (the Gamma^2 X term, the stage combinations, the
 * state, the transformation, the reflection).  FP32 stages: RK steppers,
 * N <= 256, forward only (no state saving, no bulk start); the intensities then differ from the FP64 ones by about 1e-7 to
 * 1e-6 in eacc on the test slabs, well below the step's own discretisation
 * error at the usual grids. */
typedef enum { RHEED_STAGES_FP64 = 0, RHEED_STAGES_FP32 = 1 } rheed_stage_precision;

typedef struct {
  rheed_stepper stepper;
  double rhst_threshold;     /* RHST when the condition estimate exceeds it; the paper uses 1000 */
  int32_t checkpoint_every;  /* slices between states rheed_forward keeps for rheed_backward (>= 1) */
  rheed_convention convention;
  rheed_layout layout;       /* SPLIT when the batch does not fit -> RHEED_E_UNSUPPORTED at plan creation */
  rheed_stage_precision stage_precision;
} rheed_opts;

typedef struct rheed_plan_s* rheed_plan_t;

typedef struct {
  int32_t n_struct;
  int32_t n_pairs;           /* sum of angles_per_struct; pair p of structure s is
                                numbered structure-major: pairs of s are contiguous */
  int32_t max_beams;         /* Nmax over structures: leading dimension of outputs */
  int32_t nodes_per_slice;   /* node tables per slice: 2 for RK4, 4 for RK6, 3 or 9 for the splitting steppers */
  int64_t table_elems;       /* complex elements of all potential tables */
  int64_t n_atoms_total;
  size_t fwd_workspace;      /* bytes rheed_forward needs to keep states for rheed_backward */
  size_t bwd_workspace;      /* extra bytes rheed_backward needs beyond fwd_workspace */
  int32_t split;             /* 1 if rheed_forward runs the split layout (for the pairs with N <= 64) */
  int32_t split_max_pairs;   /* pairs a split launch can hold on the current device */
  int32_t large_pairs;       /* pairs of structures with N > 64 */
  int32_t large_slots;       /* workgroups (state slots of 768 KiB each, plan-owned) that run them */
  size_t bulk_workspace;     /* bytes rheed_bulk_reflection needs beyond fwd_workspace (0: not available) */
  int32_t queue;             /* 1 if rheed_forward (without a workspace) runs the batch as one persistent
                                launch over a queue of pairs of both kinds (N <= 64 and N > 64) */
  int32_t xl_pairs;          /* pairs of structures with N > 128 */
  int32_t xl_slots;          /* resident workgroups (state slots) of the kernel for N > 128 */
  int32_t xl_group;          /* workgroups per pair with 128 < N <= 256: 1, or (a batch too small to
                                fill the device, layout not WHOLE) a cooperative group stepping the
                                pair's column blocks side by side */
  int32_t xxl_pairs;         /* pairs of structures with N > 256 (forward only) */
  int32_t xxl_group;         /* workgroups of the cooperative group of each of them */
} rheed_plan_info;

/* Vacuum wavenumber gamma (1/A) and the coefficient kappa (1/(A^2 V)) of the
 * electrostatic potential in Eq. (sch1) for a lepton of kinetic energy
 * energy_eV, relativistic (CODATA 2018).  Host only. */
rheed_status rheed_beam_constants(double energy_eV, double* gamma, double* kappa);

/* Validates and uploads the structure descriptors (host -> device, blocking).
 * angles_per_struct: host [n_struct], each >= 1.  The structure array and the
 * beam lists are copied; the caller may free them after the call. */
rheed_status rheed_plan_create(rheed_plan_t* plan, const rheed_opts* opts, int32_t n_struct,
                               const rheed_structure* structs, const int32_t* angles_per_struct);
rheed_status rheed_plan_destroy(rheed_plan_t plan);
rheed_status rheed_plan_get_info(rheed_plan_t plan, rheed_plan_info* info);
/* Failure path of the multi-workgroup launches, for tests: with half = 0
 * or 1, the first wait of that workgroup of every pair in later split
 * launches gives up at once, as a wait does when the partner workgroup stops
 * answering for about 20 ms; in the group launches (N > 128) workgroup half
 * of every pair's group starts as if a wait had given up (it waits for no
 * other workgroup).  Such a pair must come back with RHEED_PAIR_SYNC while
 * the call itself succeeds and every workgroup ends normally.  half = -1
 * (the default) turns it off.  Host only; no effect on the one-workgroup
 * layouts. */
rheed_status rheed_plan_force_sync_failure(rheed_plan_t plan, int32_t half);

/* host out[n_struct + 1]: complex-element offset of each structure's table;
 * table of structure s is [n_nodes(s)][box(s)], n_nodes = L * nodes_per_slice + 1,
 * box = (2 Hd + 1)(2 Kd + 1), Hd = max h - min h, Kd = max k - min k, entry
 * (dh + Hd)(2 Kd + 1) + (dk + Kd) holds u_{dh b1 + dk b2}(z_node) in 1/A^2
 * (the coefficient u_{l(j,k)} of Eq. sch2 for g_j - g_k = (dh, dk)). */
rheed_status rheed_plan_table_offsets(rheed_plan_t plan, int64_t* out);
/* host out[n_struct + 1]: atom offsets into the packed [n_atoms_total][3] array */
rheed_status rheed_plan_atom_offsets(rheed_plan_t plan, int64_t* out);

/* Potential tables on the slice nodes from atom positions (Sec. 2.1).
 * atoms: device [n_atoms_total][3] (x, y, z) in A.  U_tables: device complex
 * [table_elems].  Node n of a structure sits at z = -D + (i + c) h with
 * n = i * nodes_per_slice + m and c the m-th node position of the stepper (the
 * distinct RK nodes in [0, 1); for a splitting stepper its kick positions in
 * the order the kicks use them, the slice end excluded), plus
 * the final node at z = 0. */
rheed_status rheed_potential(rheed_plan_t plan, const double* atoms, void* U_tables, void* stream);

/* Gradient of a real loss w.r.t. atom coordinates from its gradient w.r.t.
 * the tables.  dL_dU: device complex [table_elems] holding
 * dL/dRe(u) + i dL/dIm(u); dL_datoms: device [n_atoms_total][3] (overwritten).
 * The sum over table entries runs in a fixed order (bitwise reproducible) and
 * uses partial sums held by the plan, so calls on one plan must not overlap
 * (issue them on one stream). */
rheed_status rheed_potential_backward(rheed_plan_t plan, const double* atoms, const void* dL_dU,
                                      double* dL_datoms, void* stream);

/* rheed_potential_backward for callers that cannot allocate device memory
 * or must not use the plan's buffers (code under stream capture, serving
 * loops, harnesses that forbid allocation).  Same arguments and results,
 * bit for bit, as rheed_potential_backward; the per-atom partial sums live in
 * a fixed device array of the library instead of the plan's memory: one copy
 * per GPU (6 MiB, held until the process ends), for at most
 * RHEED_NOALLOC_MAX_ATOMS atoms in the plan (more -> RHEED_E_UNSUPPORTED).
 * Every partial is written before it is read, so nothing needs clearing.
 * Calls no allocating routine.  Every call on one GPU shares that array:
 * calls that overlap on a GPU (other streams, other threads) race and must be
 * serialised by the caller. */
#define RHEED_NOALLOC_MAX_ATOMS 4096
rheed_status rheed_potential_backward_noalloc(rheed_plan_t plan, const double* atoms, const void* dL_dU,
                                              double* dL_datoms, void* stream);

/* Reflected amplitudes and intensities for every (structure, angle) pair
 * (Algorithm 1 + Eq. vrhocomp + the intensity formula of Sec. 2.1).
 *  U_tables   device complex [table_elems] (see rheed_plan_table_offsets)
 *  angles     device [n_pairs][2]: glancing angle theta0 and azimuth theta1
 *             (rad, theta1 measured from b1); b0 = gamma cos(theta0)(cos theta1, sin theta1)
 *  intensity  device [n_pairs][max_beams]; entries j >= N of a pair are 0
 *  rho        device complex [n_pairs][max_beams] or NULL
 *  pair_status device int32 [n_pairs] (RHEED_PAIR_*)
 *  n_rhst     device int32 [n_pairs] number of right-hand-side transformations, or NULL
 *  workspace  device, >= fwd_workspace bytes, to keep the states rheed_backward
 *             needs; NULL when no backward pass follows.
 * A batch that mixes N <= 64 and N > 64 (RK stepper, FP64 stages, layout
 * AUTO or WHOLE) runs, when no workspace is given, as one persistent launch:
 * a workgroup per CU takes pairs dearest first from a counter in plan-owned
 * memory (set to zero by a small kernel launched before it) and runs each
 * on the path of its N (rheed_plan_info.queue; rheed_autotune compares it
 * with two launches).
 * With the split layout the launch is cooperative and uses exchange blocks
 * owned by the plan, so forward calls on one plan must not overlap (issue them
 * on one stream).  Like every compute call, it only launches kernels (no
 * allocation, no memset, no synchronisation), so a stream capture records it
 * into a HIP graph, and each replay behaves like a new call (the exchange
 * blocks count their own launches). */
rheed_status rheed_forward(rheed_plan_t plan, const void* U_tables, const double* angles,
                           double* intensity, void* rho, int32_t* pair_status, int32_t* n_rhst,
                           void* workspace, size_t ws_bytes, void* stream);

/* rheed_forward over a slab that rests on the bulk (Sec. 2.2, treatment of
 * the bulk layer): the propagation starts from the state [I; Y] that the
 * bulk below leaves at z_e (c' = Y c there, the normalised form of
 * Sec. 3.2) instead of the vacuum's [I; i Gamma]; the bottom condition is
 * then rho(z_e) = R tau(z_e) with R = (Gamma + iY)(Gamma - iY)^{-1}.
 *  y_bottom  device complex [n_pairs][max_beams][max_beams], row major: Y of
 *            pair p at p max_beams^2, entry (j, k) at j max_beams + k for
 *            j, k < N of the pair (other entries are not read); typically
 *            rheed_bulk_reflection's y_bulk for the same beams and angles.
 * Every other argument, the workspace included, is as for rheed_forward,
 * and rheed_backward may follow: the gradient then holds the bulk fixed (it
 * is not fitted).  Needs an RK stepper and every structure to have N <= 64
 * (RHEED_E_UNSUPPORTED otherwise). */
rheed_status rheed_forward_bulk(rheed_plan_t plan, const void* U_tables, const double* angles, const void* y_bottom,
                                double* intensity, void* rho, int32_t* pair_status, int32_t* n_rhst,
                                void* workspace, size_t ws_bytes, void* stream);

/* The ideal bulk below a surface (Sec. 2.2, treatment of the bulk layer),
 * computed once before a structure search.  The plan's structures are unit
 * layers of the bulk (one period each, with its potential table).  Every
 * pair propagates the stack upward from the vacuum (Y = i Gamma, R = 0), one
 * unit layer at a time: a forward pass from [I; Y] over the layer, then the
 * state at its top normalised to [I; Y'] (Y' = P Q^{-1}, the transformation
 * of Sec. 3.2) and the stack's reflection matrix
 * R' = (Gamma + iY')(Gamma - iY')^{-1}.  A pair stops at the first layer
 * whose change max_jk |R' - R| is <= tol; the others go on, up to
 * max_layers layers.
 *  y_bulk, r_bulk  device complex [n_pairs][max_beams][max_beams] as
 *             y_bottom of rheed_forward_bulk (out; entries beyond N are 0):
 *             the state and reflection matrix at the top of the stack
 *  layers     device int32 [n_pairs]: layers applied when the change first
 *             passed, -1 if it did not within max_layers or the pair failed
 *  pair_status device int32 [n_pairs]: RHEED_PAIR_* (a failed pair keeps the
 *             last layer's Y and R and stops)
 *  workspace  device, >= fwd_workspace + bulk_workspace bytes (overwritten)
 * Over many layers the stepper's error on the fastest beams can turn the
 * stack to the wrong modes (R then grows without bound and no layer
 * passes): use a step at which it is small.  On the synthetic bulks of this
 * library's tests, 21 beams need RK6 at h = 0.1 A or RK4 at 0.05 A, and the
 * 61-beam bulk of the benchmark RK6 at 0.05 A.
 * Synchronises the stream after each layer to read the convergence flags
 * (so it cannot be captured into a graph); allocates nothing.  Needs an RK
 * stepper and every structure to have N <= 64. */
rheed_status rheed_bulk_reflection(rheed_plan_t plan, const void* U_tables, const double* angles, double tol,
                                   int32_t max_layers, void* y_bulk, void* r_bulk, int32_t* layers,
                                   int32_t* pair_status, void* workspace, size_t ws_bytes, void* stream);

/* Launch configurations rheed_autotune compares (at most RHEED_TUNE_MAX). */
#define RHEED_TUNE_MAX 8
typedef struct {
  int32_t n_candidates;
  int32_t chosen;                           /* index of the configuration the plan now uses */
  int32_t split[RHEED_TUNE_MAX];            /* 1: pairs with N <= 64 on the two-workgroup layout */
  int32_t large_cost_order[RHEED_TUNE_MAX]; /* 1: pairs with N > 64 dearest first, 0: in pair order */
  int32_t queue[RHEED_TUNE_MAX];            /* 1: one persistent launch over a batch mixing N <= 64 and N > 64 */
  float ms[RHEED_TUNE_MAX];                 /* mean duration of one rheed_forward call */
} rheed_tune_report;

/* Picks the launch configuration of rheed_forward for this plan by timing
 * the candidates on the caller's inputs (the batching of Sec. 3.5 over
 * (structure, angle) pairs is this library's; the paper fixes no schedule):
 * for a batch mixing N <= 64 and N > 64, one persistent launch over both;
 * and two launches with the layout of the N <= 64 pairs (split or whole,
 * where the plan's layout option is AUTO and the batch fits the split
 * layout) and the order in which the N > 64 kernel takes its pairs (by
 * estimated cost or in pair order).
 * Each candidate runs one untimed and `reps` (1..1000) timed forward calls
 * without state saving on `stream`, timed with HIP events; the fastest is
 * kept by the plan for every later rheed_forward.  U_tables, angles,
 * intensity and pair_status are as for rheed_forward (intensity and status
 * hold the last candidate's results on return; the candidates agree to
 * rounding).  Synchronises the stream; creates and destroys two HIP events,
 * allocates no device memory.  report (host) may be NULL.  Calls on one plan
 * must not overlap. */
rheed_status rheed_autotune(rheed_plan_t plan, const void* U_tables, const double* angles, double* intensity,
                            int32_t* pair_status, int32_t reps, void* stream, rheed_tune_report* report);

/* Adjoint of rheed_forward (not in the paper): given dL/d(intensity) for a
 * real loss L, accumulates dL/dU over all angles of each structure.
 * Must follow rheed_forward on the same stream with the same plan, inputs and
 * workspace.  dL_dI: device [n_pairs][max_beams]; dL_dU: device complex
 * [table_elems], overwritten; workspace >= fwd_workspace + bwd_workspace.
 * rheed_forward keeps the state at the start of every K-th slice
 * (K = checkpoint_every) and the final state, Q^{-1} and a decision byte for
 * every transformation, and for K > 1 also the normalised P after it.  The
 * adjoint walks K-slice segments from the top: the physical column psi = Z x
 * of a segment is formed from its stored state and stepped up through the
 * segment by the RK step itself, then the adjoint walks back down.  The
 * adjoint does the same products for every K; a larger K keeps fewer states
 * (fwd_workspace) at the price of the R slots.
 * Pairs with N <= 64 keep their matrices padded to 64 beams; pairs with
 * 64 < N <= 128 padded to 128 (four times the bytes per matrix), and with
 * them also B^{-1} of the final reflection solve.  A plan holding both kinds
 * sizes every pair's block for the larger.  Needs an RK stepper with FP64
 * stages (RHEED_E_UNSUPPORTED otherwise). */
rheed_status rheed_backward(rheed_plan_t plan, const void* U_tables, const double* angles,
                            const double* dL_dI, void* dL_dU, void* workspace, size_t ws_bytes,
                            void* stream);

/* R-factor of the specular beam against a target curve:
 * loss = sum_p (intensity[p][0] - target[p])^2 (device scalar), and its
 * gradient dL_dI[p][j] = 2 (intensity[p][0] - target[p]) for j = 0, 0 else. */
rheed_status rheed_rfactor(int32_t n_pairs, int32_t ld, const double* intensity, const double* target,
                           double* loss, double* dL_dI, void* stream);

/* Measured FP64 matrix-core throughput of the current device, for reading the
 * propagation kernels' roofline against an achievable ceiling beside the
 * published one: `blocks` workgroups of 4 waves each run 8 independent chains
 * of `iters` v_mfma_f64_16x16x4f64 (2048 flop each) on the null stream,
 * timed with HIP events after one untimed launch.  *tflops (host) receives
 * the rate.  Allocates and frees a small device buffer; synchronises. */
rheed_status rheed_mfma_f64_peak(int32_t blocks, int32_t iters, double* tflops);

const char* rheed_status_string(rheed_status s);
const char* rheed_last_error(void);

#ifdef __cplusplus
}
#endif
#endif /* RHEED_H */
