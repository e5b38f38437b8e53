/*
 * etd.h -- C ABI of the MI355X ETD stepper for the multicomponent-membrane
 * phase-field model of Luo, Qiao and Zhao ("Exponential Time Differencing
 * Schemes for a Phase-Field Model of Multicomponent Membranes").
 *
 * Two models, one plan object:
 *   ETD_COUPLED         the coupled phi / u system, stepped by the stabilized
 *                       spectral ETD1 / ETDRK2 of Section 3.3 (Algorithm 1);
 *   ETD_FIXED_MEMBRANE  the OK dynamics on a fixed membrane g > 0, stepped by
 *                       the localization-split FD ETD1 (eqn:ETD1) / ETDRK2
 *                       (eqn:ETDRK2) of Section 2.2.
 *
 * Conventions shared by every entry point
 *   - Every function returns etd_status (0 == ETD_OK); nothing throws.
 *   - Variables use the paper's [0,1] convention: phi ~ 1 inside the vesicle,
 *     0 outside; W(s) = 18 (s^2 - s)^2; g(phi) = 18 (phi^2 - phi)^2.
 *   - Grid: Omega = prod_d [-X_d, X_d), h_d = 2 X_d / N_d, x_i = -X_d + i h_d
 *     (Section 2.1, Section 3.2).  Arrays crossing the ABI are real, dense,
 *     C order (last axis contiguous), N_0 x N_1 (x N_2) elements.
 *   - Device pointers live on the plan's device; the caller owns them.  The
 *     plan owns its workspace and frees it in etd_plan_destroy.
 *   - Work is enqueued on the HIP stream given at creation and is
 *     stream-ordered; only the calls documented as "synchronizes" block.
 *   - Argument checks happen before any HIP call, so invalid arguments are
 *     reported (ETD_E_ARG / ETD_E_SIZE / ETD_E_STATE) even without a GPU.
 *   - A plan is not thread safe; distinct plans on distinct streams are
 *     independent.
 *
 * Environment (read once per process)
 *   ETD_LOG             host log to stderr: 0 (default) quiet, 1 every error
 *                       status with its message, 2 also plan creation, graph
 *                       captures and the autotuner's trials and choice.
 *   ETD_ROCTX           1 (default): roctx ranges around each step and its
 *                       stages (etd.phi1 / etd.phi2 / etd.u1 / etd.u2, the
 *                       band rebuild and band solve, the two fixed-membrane
 *                       stages), visible to rocprofv3 --marker-trace; they
 *                       span the host enqueue of the stage.  0 turns them off.
 *   ETD_AUTOTUNE_CACHE  the schedule cache of etd_autotune when its
 *                       cache_path argument is NULL or empty.
 */
#ifndef ETD_H
#define ETD_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct etd_plan* etd_plan_t;

typedef enum {
    ETD_OK = 0,
    ETD_E_ARG = -1,        /* null pointer, non-finite or out-of-range value      */
    ETD_E_SIZE = -2,       /* unsupported grid size (see etd_grid)                */
    ETD_E_STATE = -3,      /* call out of order (e.g. step before set_state)      */
    ETD_E_HIP = -4,        /* a HIP runtime call failed; see etd_last_error       */
    ETD_E_NOMEM = -5,      /* device allocation failed                            */
    ETD_E_NONFINITE = -6,  /* NaN/Inf detected in the state (reported at sync)    */
    ETD_E_CAPACITY = -7    /* output buffer too small; *count_out holds the need  */
} etd_status;

typedef enum { ETD_FIXED_MEMBRANE = 0, ETD_COUPLED = 1 } etd_model;
typedef enum { ETD_ETD1 = 1, ETD_ETDRK2 = 2 } etd_scheme;

/* Arithmetic of the step.
 *   ETD_FP64: every stage in FP64.
 *   ETD_FP32: coupled model -- FFTs and pointwise work in FP32 with FP32
 *             accumulation; the phi-function multipliers are formed in FP64
 *             and rounded; integrals, energies, max-bound in FP64.
 *             fixed model -- only the nonlocal (-Delta)^{-1} FFT runs in FP32;
 *             everything else stays FP64 (g reaches 1e-47 and underflows FP32). */
typedef enum { ETD_FP64 = 0, ETD_FP32 = 1 } etd_precision;

/* Element type of arrays passed through set/get_state and band building. */
typedef enum { ETD_F64 = 0, ETD_F32 = 1 } etd_dtype;

/* Grid.  dim is 2 or 3; n[d] for d < dim, each even, >= 8 and <= 512, of the
 * form 2^a or 3 * 2^a (radix-2/4/8 and radix-3 transforms); half_len[d] = X_d > 0.
 * Both models take dim 2 and 3 (a 2D grid [n0][n1] is stored like a 3D grid
 * with one x plane). */
typedef struct {
    int dim;
    int n[3];
    double half_len[3];
} etd_grid;

/* Coupled-model parameters (eqn:model_force, eqn:model_OK; stabilizers of
 * eqn:linear_force and eqn:linear_OK).  u0 is the shift in alpha (u + u0).
 * A0 is the area-constraint target; with A0_from_initial != 0 it is set to
 * h^3 sum phi^0 at etd_set_state. */
typedef struct {
    double mu, lambda_surf, kappa, lambda_line, M_area, alpha, u0;
    double eps_phi, eps_u, gamma, ubar, M;
    double A1, A2, B1, B2;
    double A0;
    int A0_from_initial;
} etd_coupled_params;

/* Fixed-membrane parameters (eqn:model_OK_fix, R_phi of Section 2.2).
 * B <= 0 selects B = B_MBP of (eqn:cond_MBP) with C = ||(-Delta_h)^{-1}||_inf
 * computed at plan creation.  nonlocal_with_ubar = 0 uses g f(u) as the
 * nonlocal argument (the discrete R_phi and energy); 1 uses g (f(u) - ubar)
 * as in the continuous equation. */
typedef struct {
    double eps_u, gamma, ubar, M;
    double B;
    int nonlocal_with_ubar;
} etd_fixed_params;

/* flags */
#define ETD_F_MASS_PROJECT 0x1u   /* after each step, shift U on {g > recover_threshold}
                                      so that <g U, 1>_h keeps its value from set_state */
#define ETD_F_FROZEN_MEMBRANE 0x2u /* coupled model only: phi keeps its set_state value and
                                      each step runs only the g u stages of Algorithm 1
                                      with g = g(phi) and v = 0 (the stabilized spectral
                                      scheme of Section 3.1 on a fixed membrane); other
                                      models reject it with ETD_E_ARG */
#define ETD_F_SURFACE_NONLOCAL 0x4u /* needs band_threshold > 0: the nonlocal term uses
                                      (-Delta_S,h)^{-1} (Section 2.1, operator:diff) assembled
                                      and solved on a band (Section 3.2), as etd_surface_lapinv
                                      does, in place of the constant-coefficient (-Delta_h)^{-1}
                                      by FFT.  Coupled model: in R2, with g = g+ of the stage
                                      and the band |2 phi - 1| < band_threshold.  Fixed model:
                                      in R_phi, with the fixed g and the band
                                      {g >= band_threshold} (the paper's delta), built by
                                      etd_set_state; FP64 on both of its paths.  The solve
                                      checks convergence on the host, so plans with this flag
                                      step eagerly under every schedule.  Each in-step solve
                                      starts from the previous solve's result (the first one
                                      after etd_set_state from 0) and runs to a residual of
                                      1e-9 (FP32 coupled instances) or 1e-12 relative to the
                                      right-hand side, at most 20000 iterations; one that
                                      stops at the cap is not an error: the step goes on with
                                      its last iterate, and ETD_Q_SURF_ITERS /
                                      ETD_Q_SURF_RELRES report the last solve.  The energy
                                      diagnostics keep (-Delta_h)^{-1}. */
#define ETD_F_BAND_STEP 0x8u      /* fixed model only, needs band_threshold > 0: the whole
                                      step runs on the band {g >= band_threshold} (the
                                      narrow-band implementation of the fixed-membrane
                                      scheme, Section 2 with the band of Section 3.2): the
                                      unknowns are the band nodes, Delta_S,h keeps the faces
                                      whose two nodes are on the band, the nonlinear terms,
                                      the nonlocal argument and the mass sum are taken on the
                                      band, and U off the band keeps its set_state value.
                                      The Chebyshev interval and B_MBP's C are those of the
                                      band operator's Gershgorin bound and of (-Delta_h)^{-1};
                                      etd_energy sums over the band's nodes and faces. */

/* One simulation instance. */
typedef struct {
    etd_model model;
    etd_scheme scheme;
    etd_precision precision;
    etd_grid grid;
    double tau;                              /* time step, > 0                          */
    const etd_coupled_params* coupled;       /* required for ETD_COUPLED                */
    const etd_fixed_params* fixed;           /* required for ETD_FIXED_MEMBRANE         */
    double band_threshold;                   /* coupled: > 0 restricts the surface terms
                                                to {|2 phi - 1| < band_threshold}
                                                (Section 3.2 narrow band); 0 = off       */
    int band_rebuild_every;                  /* rebuild the band when step % this == 0  */
    double recover_threshold;                /* U = GU/G where G > this (default 1e-3)  */
    unsigned flags;                          /* ETD_F_* bits                            */
} etd_instance_desc;

/* Create a plan for n_instances independent instances advanced together by
 * etd_step.  hip_stream is a hipStream_t (NULL = default stream).  Validates
 * every descriptor before touching HIP; then allocates device workspace and
 * forms the per-plan constants (for the fixed model C and B; the Gershgorin
 * bound of H and the Chebyshev coefficients of phi1 and phi2 depend on g and
 * are formed by etd_set_state).
 * Errors: ETD_E_ARG, ETD_E_SIZE, ETD_E_HIP, ETD_E_NOMEM.  On error *out is NULL. */
etd_status etd_plan_create(const etd_instance_desc* inst, int n_instances, void* hip_stream,
                           etd_plan_t* out);

/* Free all plan-owned device memory (synchronizes the plan's stream). */
etd_status etd_plan_destroy(etd_plan_t plan);

/* Load the state of one instance from device arrays in the grid layout.
 *   coupled: a = phi^0, u = u^0 (Algorithm 1 inputs);
 *   fixed:   a = g (fixed localization field, every value > 0), u = U^0.
 * dtype gives the element type of a and u.  Copies on the plan's stream;
 * the caller may reuse the arrays after the stream reaches this point.
 * Synchronizes.  A state holding a NaN or Inf is accepted: it is the
 * detected non-finite state of etd_step below (etd_get_state then reports
 * ETD_E_NONFINITE).  The fixed model's g must be finite and > 0 everywhere
 * (ETD_E_ARG otherwise). */
etd_status etd_set_state(etd_plan_t plan, int instance, const void* a, const void* u,
                         etd_dtype dtype);

/* Set the time step of the next steps of one instance.  Section 3.3 writes
 * both coupled schemes with a per-step tau_{n+1} (the phi-functions, the
 * step itself and the velocity's phi_t all take it), and the fixed-membrane
 * schemes of Section 2.2 step the same way; a sequence of etd_set_tau /
 * etd_step calls runs the variable-step scheme.  The state is kept.  Fixed
 * model: the Chebyshev coefficients of phi1(tau L) and phi2(tau L) are
 * re-formed on the host (no device work; formed by etd_set_state if no
 * state is loaded yet).  Graphs captured by ETD_EXEC_GRAPH are dropped (they
 * hold the old step's kernel arguments) and recaptured by the next etd_step.
 * Does not synchronize.  Errors: ETD_E_ARG (null plan, instance out of
 * range, tau not finite and > 0). */
etd_status etd_set_tau(etd_plan_t plan, int instance, double tau);

/* Copy the current state of one instance into device arrays.
 *   coupled: a <- phi^n, u <- u^n;  fixed: a <- g (may be NULL), u <- U^n.
 * Synchronizes.  The state is copied in every case; the return value is
 * ETD_E_NONFINITE once a non-finite value has been detected (see etd_step). */
etd_status etd_get_state(etd_plan_t plan, int instance, void* a, void* u, etd_dtype dtype);

/* Checkpoint of one instance in host memory: everything a step carries over
 * to the next (coupled, Algorithm 1: the spectrum of phi^n, phi^n and the
 * fields derived from it, u^n, the band mask and list in use, the device
 * scalars; fixed, eqn:ETD1 / eqn:ETDRK2: g and U^n with the device scalars;
 * the band solve's starting iterate when ETD_F_SURFACE_NONLOCAL is set), the
 * step counter and A0.  etd_set_state / etd_get_state carry phi^n and u^n
 * alone, and a run restarted from them differs from the original in
 * rounding (the spectrum is re-formed from phi^n) and in A0; a run resumed
 * with etd_checkpoint_load continues bit for bit as the saved one would.
 *   etd_checkpoint_size: *bytes (host) receives the size of the image.
 *   etd_checkpoint_save: writes the image into host[0 .. bytes); needs a
 *     state (ETD_E_STATE) and bytes >= the size (ETD_E_CAPACITY).
 *   etd_checkpoint_load: reads an image saved from an instance with the same
 *     model, scheme, precision, grid, flags and band settings (ETD_E_ARG
 *     otherwise; nothing is changed); the instance keeps its own tau (call
 *     etd_set_tau to continue a variable-step run).
 * The image is the library's own binary layout (a header, then the device
 * buffers in a fixed order), valid for the library build that wrote it.
 * Save and load synchronize.  Errors: ETD_E_ARG (null pointers, instance
 * out of range, a foreign or mismatched image), ETD_E_STATE, ETD_E_CAPACITY,
 * ETD_E_HIP. */
etd_status etd_checkpoint_size(etd_plan_t plan, int instance, size_t* bytes);
etd_status etd_checkpoint_save(etd_plan_t plan, int instance, void* host, size_t bytes);
etd_status etd_checkpoint_load(etd_plan_t plan, int instance, const void* host, size_t bytes);

/* Advance every instance by nsteps time steps (ETD1 or ETDRK2 as planned).
 * Asynchronous.  Non-finite values are detected on the device, per
 * instance, by the FP64 sums every step forms (coupled: h^d sum phi after
 * each phi stage and the mass of each u stage; fixed: the mass m_f of each
 * remainder evaluation), and by etd_set_state on its inputs.  From then on
 * the instance's steps leave its state (phi, u / U) as it is, also under a
 * captured graph schedule: the kernels that write the state read the flag
 * first.  Values written by the step in which the detection happens, before
 * that point, remain.  Reported by etd_get_state and etd_diagnostics
 * (ETD_E_NONFINITE); cleared by etd_set_state.  Other instances step on. */
etd_status etd_step(etd_plan_t plan, int nsteps);

/* Energy of one instance, FP64, written to host_out (synchronizes).
 *   fixed   (eqn:Energy_dis), n_out >= 5: [E, E_grad, E_well, E_nonlocal, E_mass]
 *   coupled (n_out >= 6): [E_surf, E_bend, E_area, E_ok, E_nonlocal, E_mass]
 *           with E_surf = lambda_surf <|grad phi|^2/2 + W(phi)/eps^2, 1>_h,
 *           E_bend = (kappa/2) <(Delta phi - W'(phi)/eps^2)^2, 1>_h,
 *           E_area = (M_area/2)(int phi - A0)^2, E_ok = the OK gradient and well
 *           terms with g(phi), E_nonlocal = (gamma/2) <(-Delta)^{-1} q, q>_h,
 *           E_mass = (M/2) <q, 1>_h^2, q = g(phi)(u - ubar). */
etd_status etd_energy(etd_plan_t plan, int instance, double* host_out, int n_out);

/* Per-instance diagnostics (FP64). */
typedef struct {
    int64_t step;        /* steps taken since set_state                            */
    double int_phi;      /* h^d sum phi (coupled) / 0 (fixed)                      */
    double mass;         /* coupled: <g(phi)(u - ubar), 1>_h; fixed: <g (f(U) - ubar), 1>_h */
    double Q;            /* <g U, 1>_h                                             */
    double umin, umax;   /* min / max of U                                         */
    double bound;        /* max |2 U - 1| (the paper's max-bound check)            */
    int64_t band_count;  /* current narrow-band size (coupled with a band), else 0 */
    int nonfinite;       /* 1 if a NaN/Inf was seen                                */
    int b_warning;       /* fixed: 1 if the planned B is below B_MBP               */
} etd_diag;

/* Compute and return the diagnostics of one instance (synchronizes). */
etd_status etd_diagnostics(etd_plan_t plan, int instance, etd_diag* host_out);

/* Per-step diagnostics ring (the etd_diag fields of etd_diagnostics,
 * recorded on the device after every step, so a long run can be followed
 * without a synchronization per step; also under a captured graph schedule).
 * etd_diag_ring_enable keeps the last `capacity` steps of the instance (0
 * turns the ring off and frees it; at most 2^24); it synchronizes and drops
 * captured graphs.  Each step then adds one reduction pass over its state.
 * etd_set_state and etd_checkpoint_load start the record again.
 * etd_diag_ring_read copies the most recent min(recorded, capacity,
 * max_entries) entries, oldest first, into host_out; *recorded receives the
 * number of steps recorded since the record started (the older ones beyond
 * the capacity are gone).  Synchronizes.  Errors: ETD_E_ARG (null plan or
 * output, instance out of range, capacity or max_entries out of range),
 * ETD_E_STATE (read with the ring off), ETD_E_NOMEM, ETD_E_HIP. */
etd_status etd_diag_ring_enable(etd_plan_t plan, int instance, int capacity);
etd_status etd_diag_ring_read(etd_plan_t plan, int instance, etd_diag* host_out, int max_entries,
                              int64_t* recorded);

/* Narrow band of Section 3.2 for a phase field phi (device array, grid layout
 * of the instance): the ascending C-order linear indices i with
 * |2 phi_i - 1| < threshold, decided in FP64, written as int32 to dev_idx_out.
 * If the band holds more than capacity points, nothing is written,
 * *count_out is set to the band size and ETD_E_CAPACITY is returned.
 * count_out is a host pointer; the call synchronizes. */
etd_status etd_narrowband_build(etd_plan_t plan, int instance, const void* phi, etd_dtype dtype,
                                double threshold, int32_t* dev_idx_out, int64_t capacity,
                                int64_t* count_out);

/* The band list of etd_narrowband_build for callers that cannot allocate
 * device memory (serving loops and harnesses that forbid hipMalloc): the
 * same indices, bit for bit, for the n values phi[0 .. n) (any n from 0 to
 * 268,435,456; the list does not depend on the grid's shape), with no
 * hipMalloc, hipFree or allocating library call.  Its kernels keep their
 * tile offsets and the total in a static 512 KiB array per device, which
 * the library looks up at etd_plan_create and which lives until the process
 * ends; every entry a call reads is written earlier in the same call.  All
 * calls on one device share that array, so calls that overlap in time on
 * one device race (the plan's stream orders calls made through one plan).
 * Runs on the plan's stream; count_out is a host pointer; synchronizes (so
 * it cannot be captured into a graph).  Errors: ETD_E_ARG (null plan or
 * count_out, n < 0, phi NULL with n > 0, threshold not finite and > 0,
 * capacity < 0, dev_idx_out NULL with capacity > 0, bad dtype), ETD_E_SIZE
 * (n above the limit), ETD_E_CAPACITY (as etd_narrowband_build: nothing
 * written, *count_out set), ETD_E_HIP. */
etd_status etd_narrowband_build_noalloc(etd_plan_t plan, const void* phi, etd_dtype dtype, int64_t n,
                                        double threshold, int32_t* dev_idx_out, int64_t capacity,
                                        int64_t* count_out);

/* Apply one of the plan's spectral operators to a real field through the
 * instance's own transforms (forward r2c, multiplier, inverse c2r):
 *   ETD_OP_IDENTITY  round trip (multiplier 1)
 *   ETD_OP_LAPLACE   spectral Laplacian, symbol -k^2 with the wavenumbers of
 *                    Section 3.2 (lambda(i) = pi i / X for i <= N/2, pi (N - i)/X above)
 *   ETD_OP_DX/DY/DZ  spectral first derivative i k_d along array axis 0/1/2
 *                    (Nyquist bin zeroed); a 2D grid has axes 0 and 1 only,
 *                    and ETD_OP_DZ returns ETD_E_ARG there
 *   ETD_OP_LAPINV    (-Delta_h)^{-1}: inverse of the periodic (2d+1)-point FD
 *                    Laplacian with the mean removed (symbol 1/mu_k, 0 at k = 0)
 * in and out are device arrays in the grid layout (they may alias).  The
 * transforms run in the instance's precision (fixed model: FP64, or FP32 on
 * the FP32-FFT path).  Uses only the instance's scratch buffers, never its
 * state.  Asynchronous on the plan's stream. */
typedef enum {
    ETD_OP_IDENTITY = 0, ETD_OP_LAPLACE = 1, ETD_OP_DX = 2, ETD_OP_DY = 3, ETD_OP_DZ = 4, ETD_OP_LAPINV = 5
} etd_spectral_op;
etd_status etd_spectral_apply(etd_plan_t plan, int instance, etd_spectral_op op, const void* in, void* out,
                              etd_dtype dtype);

/* Per-pass timing of the step's kernels (a measurement aid).  enable != 0
 * starts a measurement: every kernel launched afterwards by steps of this plan is
 * bracketed by HIP events recorded on the plan's stream.  enable == 0 stops
 * it, synchronizes, and fills out (may be NULL) per pass kind: the number of
 * launches, their summed event-timed duration in ms, and the algorithmic bytes
 * they move (each distinct input element read once, each output element
 * written once).  Kinds:
 *   0 z-row r2c            1 z-row c2r             2 y lines
 *   3 x lines              4 inverse x lines S -> (S, i kx S, -kx^2 S)
 *   5 inverse y lines, 3 -> 4 spectra (derivatives)
 *   6 z-row c2r, 4 spectra -> phi, grad phi, lap phi
 *   7 z-row r2c of two fields          8 forward y lines of two spectra
 *   9 forward x lines of two spectra with the ETD combine
 *  10 last forward axis times 1/mu and back ((-Delta_h)^{-1})
 *  11 z-row c2r of a G U increment with the recovery of U in the store
 * and the other kernels of a step (same hook, same bracketing):
 *  12 narrow-band flags and compaction   13 R1 remainder (stencil)
 *  14 R2 remainder P2 (stencil)          15 coupled pointwise kernels
 *  16 FP64 reductions                    17 fixed model: Chebyshev / L stencils
 *  18 fixed model: pointwise kernels
 *  19 z-row r2c of the R1 pair with R1 formed in the load
 *  20 z-row r2c of the (P2, g u) pair with P2 formed in the load
 *  21 z-row r2c of q = g (u - ubar) formed in the load, with its sum
 *  22..23 unused. */
#define ETD_PASS_KINDS 24
typedef struct {
    int64_t launches[ETD_PASS_KINDS];
    double total_ms[ETD_PASS_KINDS];
    double bytes[ETD_PASS_KINDS];
} etd_pass_times;
etd_status etd_pass_timing(etd_plan_t plan, int enable, etd_pass_times* out);

/* Scalar plan facts for one instance (host doubles):
 *   ETD_Q_B          stabilizer B in use (fixed)
 *   ETD_Q_B_MBP      B_MBP of (eqn:cond_MBP) (fixed)
 *   ETD_Q_B_ES       B of (eqn:cond_ES) (fixed)
 *   ETD_Q_C          ||(-Delta_h)^{-1}||_inf (fixed)
 *   ETD_Q_RHO        Gershgorin bound of H = -g^{-1/2} Delta_{S,h} g^{-1/2} (fixed)
 *   ETD_Q_CHEB_DEG   degree of the Chebyshev expansions of phi1 / phi2 (fixed)
 *   ETD_Q_A0         area target A0 (coupled)
 *   ETD_Q_WORKSPACE  bytes of device workspace held by the instance */
typedef enum {
    ETD_Q_B = 0, ETD_Q_B_MBP = 1, ETD_Q_B_ES = 2, ETD_Q_C = 3, ETD_Q_RHO = 4,
    ETD_Q_CHEB_DEG = 5, ETD_Q_A0 = 6, ETD_Q_WORKSPACE = 7,
    ETD_Q_SURF_ITERS = 8,   /* iterations of the last band solve (ETD_F_SURFACE_NONLOCAL) */
    ETD_Q_SURF_RELRES = 9   /* its final relative residual */
} etd_query;
etd_status etd_plan_query(etd_plan_t plan, int instance, etd_query what, double* out);

/* psi = (-Delta_S,h)^{-1} f on a narrow band (Section 2.1: Delta_S,h of
 * operator:diff with face coefficients g_{i+1/2} = (g_i + g_{i+1})/2, its
 * inverse on mean-zero grid functions with the mean of f removed; Section
 * 3.2: the operator is set up and inverted on the band nodes alone).  Band: the nodes with
 * mask[i] != 0 (uint8, grid layout, e.g. from etd_narrowband_build's rule);
 * faces to nodes off the band carry no flux, the band means of f and of psi
 * are removed, psi = 0 off the band.  The band must be connected (its
 * constants are then the only null space).  g (> 0 on the band), f and psi
 * are device arrays in the grid layout of the instance, element type dtype
 * (psi may alias f).  FP64 conjugate gradients from psi = 0, preconditioned
 * by a 16-term Chebyshev polynomial of the Jacobi-scaled operator (its
 * vectors stored in the precision of dtype, its arithmetic FP64), until the
 * residual relative to f - mean_band(f) is <= tol or after max_iter
 * iterations (f constant on the band: psi = 0 at once); *iters_out and
 * *relres_out (host, nullable) report the outcome -- not converging is
 * reported there, not as an error.
 * Uses a workspace of about 92 bytes per grid point, allocated on the first
 * call and kept by the plan.  Synchronizes.
 * Errors: ETD_E_ARG (null pointers, dtype, tol not finite and > 0,
 * max_iter < 1), ETD_E_NOMEM, ETD_E_HIP. */
etd_status etd_surface_lapinv(etd_plan_t plan, int instance, const void* g, const void* f,
                              const uint8_t* mask, void* psi, etd_dtype dtype, double tol, int max_iter,
                              int* iters_out, double* relres_out);

/* Static strings; never NULL. */
/* Execution schedule of etd_step over all instances of a plan (a batch of
 * uneven instances, e.g. many 64^3, 96^3 and 128^3 vesicles in one plan).
 *   ETD_EXEC_EAGER  every kernel is launched from the host, one instance
 *                   after another, on the plan's stream (the default).
 *   ETD_EXEC_GRAPH  two steps of all instances are captured once into a HIP
 *                   graph and replayed.  Inside the graph the instances are
 *                   spread round-robin over `branches` (1..64) concurrent
 *                   branches forked from and joined back to the plan's
 *                   stream, so small instances overlap on the device.  An odd
 *                   remaining step runs eagerly.  The captured graphs are
 *                   dropped by etd_set_state and etd_set_schedule and are
 *                   recaptured when the band-rebuild pattern of the two
 *                   captured steps changes.  Pass timing forces eager steps.
 *   ETD_EXEC_GROUPED  like ETD_EXEC_GRAPH, but the instances of one shape and
 *                   configuration (grid, model, scheme, precision, flags)
 *                   form a group, and each pass of a step runs as ONE launch
 *                   over the tiles of all instances of the group (the
 *                   instance is the second grid coordinate; each reads its
 *                   own arguments -- fields, tau, coefficients -- from a
 *                   device table the graph owns), so a batch of 48 uneven
 *                   instances in three shape classes takes three launches per
 *                   pass instead of 48.  The groups are spread over
 *                   min(branches, groups) concurrent branches.  Coupled
 *                   instances on 3D grids without a band, diagnostics ring,
 *                   mass projection or band solve only (ETD_E_ARG otherwise,
 *                   at etd_set_schedule, or at the next etd_step if such a
 *                   feature is turned on later; the states are then left
 *                   as they were).
 * Results are identical under every schedule (the instances are
 * independent and every kernel runs the same arithmetic). */
typedef enum { ETD_EXEC_EAGER = 0, ETD_EXEC_GRAPH = 1, ETD_EXEC_GROUPED = 2 } etd_exec_mode;
typedef struct {
    int mode;       /* etd_exec_mode */
    int branches;   /* concurrent capture branches (graph and grouped modes) */
    int xlines;     /* lines per workgroup of the ETD x pass of FP32 coupled
                       instances on 3D grids: 0 or 16 (the default tile), 8
                       (twice the workgroups; the same arithmetic, so the same
                       results bit for bit) */
} etd_schedule;
etd_status etd_set_schedule(etd_plan_t plan, const etd_schedule* sched);
etd_status etd_get_schedule(etd_plan_t plan, etd_schedule* out);

/* Schedule autotuner.  Times trial_steps (rounded up to even, >= 2) steps
 * of each candidate -- eager, then graph with 1, 2, 4, 8, 16 and 32 branches
 * (those not above the instance count), grouped on 1 and 8 branches (where
 * every instance can be grouped), then the fastest of these with the
 * 8-line ETD x tile (when an FP32 coupled 3D instance takes that pass) --
 * after two untimed warm-up steps each, on the current states; then restores
 * every instance exactly from a device snapshot taken first (state fields,
 * spectrum, derivatives, band mask and list, device scalars, step counter),
 * sets the fastest schedule and returns it in *chosen (may be NULL).  ms_out
 * (may be NULL) receives the per-step milliseconds of the 10 candidates in
 * that order (negative for a candidate not tried).  cache_path (NULL or empty: the environment's
 * ETD_AUTOTUNE_CACHE, else no cache) names a JSON file of earlier choices keyed by the device architecture and the sorted multiset of (model,
 * scheme, precision, grid) of the instances: a hit selects the cached
 * schedule without trials (ms_out entries then negative); a miss appends the
 * new choice.  Every instance must have a state.  Allocates the snapshot
 * (about the size of the state) for the duration of the call.  Synchronizes. */
#define ETD_AUTOTUNE_CANDIDATES 10
etd_status etd_autotune(etd_plan_t plan, int trial_steps, const char* cache_path, etd_schedule* chosen,
                        double* ms_out);

const char* etd_status_string(etd_status s);
const char* etd_last_error(etd_plan_t plan);   /* plan may be NULL: last global error */

#ifdef __cplusplus
}
#endif
#endif /* ETD_H */
