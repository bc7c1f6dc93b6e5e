/*
 * cpic.h -- C ABI of libcpic, an MI355X (gfx950) implementation of the
 * data-parallel hot path of the colored particle-in-cell (CPIC) method of
 * arXiv:2303.05599: leapfrog evolution of boost-invariant SU(3) Glasma fields
 * on a periodic transverse lattice (Sec. II.A) coupled to a Wong-equation push
 * of test particles whose colour charges are parallel-transported with the
 * links (Sec. III.B).
 *
 * General conventions
 *   - Every function returns cpic_status: 0 on success, a negative code on
 *     failure; nothing aborts.  cpic_last_error() gives a message.
 *   - A context owns all device memory it allocates and frees it in
 *     cpic_destroy().  Host buffers passed in are owned by the caller; the
 *     library reads/writes them only during the call, after synchronising
 *     its stream.
 *   - All device work of a context is enqueued on the HIP stream given to
 *     cpic_create (NULL: the library creates its own default-priority
 *     stream).  Functions that return data synchronise that stream.
 *   - One context must not be used from two threads at once.
 *   - Fixed seeds give bitwise-identical results from run to run.
 *   - Units: inputs in fm and GeV as documented; internally everything is
 *     in lattice ("hat") units: t = tau/a, p_hat = a p, m_hat = a m,
 *     p^eta_hat = a^2 p^eta, fields g a^2 F.
 */
#ifndef CPIC_H
#define CPIC_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef int32_t cpic_status;
#define CPIC_OK 0
#define CPIC_E_INVALID (-1)    /* bad argument or call order                        */
#define CPIC_E_NOMEM (-2)      /* device or host allocation failed                  */
#define CPIC_E_HIP (-3)        /* a HIP runtime call failed                         */
#define CPIC_E_IC_NEWTON (-4)  /* initial-link Newton solve did not converge        */
#define CPIC_E_NAN (-5)        /* NaN/Inf found by the diagnostics                  */
#define CPIC_E_DRIFT (-6)      /* unitarity / Gauss / Casimir drift over threshold (cpic_set_watchdog) */
#define CPIC_E_CAPACITY (-7)   /* caller buffer too small                           */
#define CPIC_E_CELL_JUMP (-8)  /* a particle moved more than one cell in one step   */
#define CPIC_E_IO (-9)         /* checkpoint file could not be read or written      */

typedef struct cpic_ctx cpic_ctx;
typedef struct cpic_batch cpic_batch;

#define CPIC_FP64 0
#define CPIC_FP32 1
#define CPIC_REP_FUND 0
#define CPIC_REP_ADJ 1

/*
 * Glasma event parameters (Sec. II.A for the lattice and the MV model with
 * N_s colour sheets [eq:MVchargecorrnum]; Sec. VII.A for the regulators).
 *   N            lattice sites per transverse direction (N = 2^p 3^q, 4..1024)
 *   L_fm         transverse box length; a = L/N
 *   g2mu_GeV     MV scale g^2 mu
 *   m_ir_GeV     infrared regulator of the Poisson kernel
 *   uv_GeV       ultraviolet cut of the Poisson kernel (<= 0: none)
 *   n_sheets     number of colour sheets per nucleus
 *   dtau_over_a  leapfrog step in units of a (1/8 in Sec. VII.A)
 *   tau_max_fm   end of the evolution; n_max = ceil(tau_max / dtau) steps
 *   seed         seed of the colour-charge stream
 *   precision    CPIC_FP64 or CPIC_FP32 (storage and update type)
 *   reunit_every FP32 only: project links to SU(3) and renormalise the
 *                colour charges every that many steps (0 = never)
 *   record_every steps between broadening samples (a sample is also taken
 *                after the last step)
 *   n_colors     gauge group SU(n_colors): 3 (or 0, the default) or 2.  The
 *                SU(2) variant (links as unit quaternions, three colour
 *                components, charges from the Darboux parametrisation of
 *                Sec. IV.A) runs single events with the rotation colour update;
 *                light-like paths, the matrix-logarithm update, batches and
 *                the launch tuner are SU(3) only.
 */
typedef struct {
    int32_t N;
    double L_fm;
    double g2mu_GeV;
    double m_ir_GeV;
    double uv_GeV;
    int32_t n_sheets;
    double dtau_over_a;
    double tau_max_fm;
    uint64_t seed;
    int32_t precision;
    int32_t reunit_every;
    int32_t record_every;
    int32_t n_colors;
} cpic_glasma_params;

/*
 * Test-particle species (toy-model initial conditions of Sec. III.B, colour
 * charges from the Haar measure of Sec. IV.B).
 *   n                number of test particles (0: fields only); at most
 *                    14,128,181 in FP64 and 28,256,363 in FP32 (the records,
 *                    19 reals each, stay below 2 GiB), else CPIC_E_INVALID
 *   mass_GeV         mass; INFINITY selects the static (infinite-mass) branch
 *                    of Sec. V.A: no motion, no colour rotation
 *   pT_min/max_GeV   initial |p_T| uniform in [min, max) (equal: fixed)
 *   azimuth_uniform  1: direction of p_T uniform; 0: along +x (the jets of Sec. VII.D)
 *   tau_form_fm      formation time; the push starts at n_form = ceil(tau_form/dtau)
 *   rep              CPIC_REP_FUND (q2 = 4, q3 = 10/3) or CPIC_REP_ADJ (q2 = 24, q3 = 0);
 *                    SU(2): q2 = 3/2 or 6, q3 = 0 ([eq:q23c23])
 *   seed             seed of the particle stream
 *   color_update     CPIC_COLOR_ROTATE (default): the charges are rotated with
 *                    the links crossed and the rapidity Wilson line
 *                    [eq:colorrotnum], which keeps their Casimirs exactly;
 *                    CPIC_COLOR_LOG: the alternative of Sec. III.B, dQ/dtau =
 *                    ig[Q, A_mu] p^mu/p^tau with the transverse gauge fields
 *                    from the matrix logarithm of the links (a A_i = -i log U_i
 *                    on the link whose midpoint is nearest), stepped by
 *                    explicit Euler with the rest of the particle (the Casimirs
 *                    then drift at first order in dtau; no renormalisation).
 *                    Single events only (cpic_batch_create rejects it).
 */
#define CPIC_COLOR_ROTATE 0
#define CPIC_COLOR_LOG 1
typedef struct {
    int64_t n;
    double mass_GeV;
    double pT_min_GeV;
    double pT_max_GeV;
    int32_t azimuth_uniform;
    double tau_form_fm;
    int32_t rep;
    uint64_t seed;
    int32_t color_update;
} cpic_particle_params;

/* Create a context: validates the parameters and allocates the ping-pong
 * field buffers (68 reals per site each), the particle records and the
 * observable buffers.  hip_stream: a hipStream_t or NULL.  No computation. */
cpic_status cpic_create(const cpic_glasma_params* glasma, const cpic_particle_params* particles, void* hip_stream,
                        cpic_ctx** out);

/* MV-model initial condition from the seeds (Sec. II and II.A; Haar colour
 * charges, Sec. IV.B): Gaussian charges per sheet, FFT Poisson solve with the
 * IR and UV regulators, Wilson lines, pure-gauge nucleus links, tau = 0 Glasma
 * links from the lattice initial condition (Newton per link), pi(0); E = phi = 0.
 * Particles: positions uniform, |p_T| and azimuth as configured, eta = p^eta = 0.
 * Resets the step counter and the recorded samples.  Runs on the GPU in double
 * precision and synchronises.  CPIC_E_IC_NEWTON if a link did not converge. */
cpic_status cpic_init_mv(cpic_ctx* ctx);

/* Advance n_steps leapfrog steps (Sec. II.A) with the particle push at each
 * step n >= n_form (Sec. III.B).  Asynchronous; fails with CPIC_E_INVALID if it
 * would pass n_max. */
cpic_status cpic_step(cpic_ctx* ctx, int32_t n_steps);

/* Advance until tau >= tau_target_fm (or n_max).  Asynchronous; every step
 * runs from a HIP graph: graphs of up to 16 steps, each ending at the next
 * particle reordering point or at the target, captured once per length and
 * buffer parity and replayed; a graph that starts at a reordering point of
 * moving particles starts with the reordering.  A no-op if already there. */
cpic_status cpic_evolve(cpic_ctx* ctx, double tau_target_fm);

/* Wait for the context's stream; reports CPIC_E_CELL_JUMP if any particle
 * moved more than one cell in one step since the last check, and a breach the
 * drift watchdog found (CPIC_E_DRIFT, or CPIC_E_NAN for a non-finite value;
 * cpic_last_error names the check, the step and the value).  A reported
 * breach is cleared. */
cpic_status cpic_sync(cpic_ctx* ctx);

/* Drift watchdog (on by default, every 64 steps).  After every `every`-th
 * step the device computes the Gauss, unitarity and Casimir columns of
 * cpic_diagnostics for the state (not the energies) and compares them,
 * without synchronising, with
 *   max_unitarity       max |U U^+ - 1| over all link entries (absolute);
 *   max_gauss_drift     the change of max |G| (the Gauss residual of Sec. II)
 *                       since the state was installed, relative to max(1, its
 *                       value then): the leapfrog keeps the lattice Gauss law
 *                       to rounding;
 *   max_casimir_drift   the change of max |q2 - q2(R)| and of max |q3 - q3(R)|
 *                       over the particles ([eq:q2_main], [eq:q3_main]) since
 *                       installation, relative to max(1, q2(R)) (SU(3) with the
 *                       rotation update, which keeps the Casimirs);
 * and any non-finite value.  The baseline is taken before the first step
 * after cpic_init_mv, cpic_set_state or cpic_load.  The first breach is kept
 * and reported by the next cpic_sync.  every = 0 switches it off.  Defaults:
 * 1e-8 for all three in double precision, 1e-2 in single precision. */
cpic_status cpic_set_watchdog(cpic_ctx* ctx, int32_t every, double max_unitarity, double max_gauss_drift,
                              double max_casimir_drift);

/* Current step n (tau = n dtau) and the number of broadening samples taken. */
cpic_status cpic_current_step(const cpic_ctx* ctx, int64_t* n);
cpic_status cpic_num_samples(const cpic_ctx* ctx, int32_t* n);

/*
 * Momentum broadening [eq:mombroad] averaged over the particles, raw classical
 * value in GeV^2 (divide by D_R for the quantum mapping of Sec. VI), one entry
 * per sample, oldest first:
 *   tau_fm[k], dpT2[k] = <p_x^2 + p_y^2 - p_T(form)^2>, dpL2[k] = <p_z^2>
 * with p^z = p^tau sinh(eta) + tau p^eta cosh(eta) (the tracked p_z for the
 * static branch).  Any pointer may be NULL.  CPIC_E_CAPACITY if cap is smaller
 * than the number of samples (nothing written).  Synchronises.
 */
cpic_status cpic_observables(cpic_ctx* ctx, double* tau_fm, double* dpT2_GeV2, double* dpL2_GeV2, int32_t cap);

/* As above with all columns: out[6*k + c], c = tau_fm, <dp_T^2>, <dp_L^2>,
 * <dp_par^2> (along the initial p_T direction), <dp_perp^2> (across it), and
 * the number of particles averaged.  GeV^2. */
cpic_status cpic_observables_full(cpic_ctx* ctx, double* out, int32_t cap);

/* Transport coefficients and anisotropies from the samples: the instantaneous
 * heavy-quark coefficients kappa_{L,T}(tau) = d<dp_{L,T}^2>/dtau
 * ([eq:kappalt]), the jet coefficients qhat_i = d<dp_i^2>/dtau ([eq:qhati];
 * for particles launched along x, i = x is the component along the initial
 * direction, y across it, z the longitudinal one, qhat_z = kappa_L), the
 * heavy-quark anisotropy <dp_L^2>/<dp_T^2> and the jet anisotropy
 * <dp_z^2>/<dp_y^2> ([eq:jetanisotropy]).  The derivatives are central
 * differences between consecutive samples, at the midpoint, the first interval
 * opening at the formation time, where every <dp^2> vanishes.  out[8*k + c]
 * for sample k: c = 0 tau_mid (fm/c), 1 kappa_T, 2 kappa_L, 3 qhat_x (par),
 * 4 qhat_y (perp) (GeV^2 c/fm, over [tau_{k-1}, tau_k]), 5 tau_k, 6 the
 * heavy-quark anisotropy, 7 the jet anisotropy at tau_k.  *n_samples (may be
 * NULL) receives the sample count; CPIC_E_CAPACITY if cap is smaller (nothing
 * written).  Synchronises. */
cpic_status cpic_transport(cpic_ctx* ctx, double* out, int32_t cap, int32_t* n_samples);

/*
 * Diagnostics at the current step n (double-precision reductions):
 *   out[0] sum_x |G(x)|^2, G the lattice Gauss residual
 *          sum_i [E_i(x) - U_i(x-i)^+ E_i(x-i) U_i(x-i)] + i[phi, pi]
 *          (the Gauss constraint of Sec. II)
 *   out[1] max_x |G(x)|
 *   out[2..5] lattice energy terms (1/t) sum Tr E^2, t sum Tr pi^2,
 *          2t sum Re Tr(1 - U_12), (1/t) sum Tr(phi->_i - phi)^2 with the
 *          momenta averaged to integer time (hat units, = g^2 a dE/deta)
 *   out[6] max |U U^+ - 1| over all link entries, out[7] sum of its squares
 *   out[8] max |q2 - q2(R)|, out[9] max |q3 - q3(R)| over the particles
 *          (classical Casimirs [eq:q2_main], [eq:q3_main])
 * Returns CPIC_E_NAN if any of them is not finite.  Synchronises.
 */
cpic_status cpic_diagnostics(cpic_ctx* ctx, double out[10]);

/* The four headline quantities of cpic_diagnostics at the current step:
 *   gauss_l2      = sqrt(out[0]), the L2 norm of the Gauss residual over the lattice;
 *   energy_lat    = out[2] + out[3] + out[4] + out[5], the lattice energy (hat units);
 *   unitarity_max = out[6];
 *   casimir_max   = max(out[8], out[9]) (0 without particles).
 * Any pointer may be NULL.  CPIC_E_NAN as cpic_diagnostics (nothing
 * written).  Synchronises. */
cpic_status cpic_diagnostics_summary(cpic_ctx* ctx, double* gauss_l2, double* energy_lat, double* unitarity_max,
                                     double* casimir_max);

/*
 * For callers that cannot allocate device memory (code under HIP graph
 * capture, serving loops, harnesses that forbid hipMalloc): the field columns
 * out[0..7] of cpic_diagnostics, computed on a caller-owned device buffer set
 * and written to caller-owned device memory, with no allocation of any kind.
 *   precision    CPIC_FP64 or CPIC_FP32: the element type of fields_dev
 *   N            lattice size, 4 <= N <= 1024 (any N; larger: CPIC_E_INVALID,
 *                nothing launched)
 *   dtau_over_a  leapfrog step in units of a; t = n dtau_over_a enters the
 *                energy terms and the half-step correction of the momenta
 *   n            step of the state (E and pi at n - 1/2, as the library keeps them)
 *   fields_dev   device buffer set of 68 N^2 reals, component-major (site
 *                s = y N + x innermost): U_x [18][N^2], U_y [18][N^2] (complex
 *                3x3, row-major, re/im; only the first two rows, components
 *                0..11, are read: the third row is rebuilt as the conjugate
 *                cross product), phi [8][N^2], E_x [8][N^2], E_y [8][N^2],
 *                pi [8][N^2].  Read only.
 *   out_dev      device array of 8 doubles, written in the order of
 *                cpic_diagnostics out[0..7] (non-finite values are written as
 *                they are: no CPIC_E_NAN, since the call does not synchronise)
 *   hip_stream   stream of the current device (NULL: the null stream)
 * Asynchronous: two kernels on hip_stream, no synchronisation, no memset.
 * The per-block partial sums go to a fixed 256 KiB device array of the
 * library (one per GPU, held until the process ends; its address on a device
 * is resolved by cpic_create or by this call's first use on that device).
 * Every call overwrites all the partials it reads, so no state carries over;
 * calls that overlap on one GPU (several streams or host threads) race on
 * that array and must be ordered by the caller.  Errors: CPIC_E_INVALID (bad
 * argument), CPIC_E_HIP (launch failure); message in cpic_last_error(NULL).
 */
cpic_status cpic_field_diagnostics_noalloc(int32_t precision, int32_t N, double dtau_over_a, int64_t n,
                                           const void* fields_dev, double* out_dev, void* hip_stream);

/*
 * Copy a part of the state to/from caller host memory, always as float64 in
 * this layout (site s = y*N + x, x along e1), whatever the device precision:
 *   CPIC_STATE_U         complex128 [2][N][N][3][3]  links U_x, U_y (row-major)
 *   CPIC_STATE_PHI       float64 [N][N][8]           phi = g A_eta components
 *   CPIC_STATE_E         float64 [2][N][N][8]        E_i = g a P^i at n - 1/2
 *   CPIC_STATE_PI        float64 [N][N][8]           pi = g a^2 P^eta at n - 1/2
 *                        (SU(2): [3][3] -> [2][2] and 8 -> 3 components; the
 *                        particle records keep 20 columns, Q^4..Q^8 zero)
 *   CPIC_STATE_PARTICLES float64 [n][20]             x, y, eta, p^x, p^y, p^eta
 *                        (p^z for the static branch), Q^1..Q^8, cell x, cell y,
 *                        last eta increment, initial direction (ux, uy), |p_T(form)|
 *   CPIC_STATE_STEP      int64 [1]                   n (setting it clears the samples)
 *   CPIC_STATE_JET_W     complex128 [N][N][3][3]     Wilson line of the light-like path
 *                        starting in site (y, x) (get only; cpic_jets_enable)
 *   CPIC_STATE_JET_F     float64 [N][N][3][8]        its integrated transported force
 *                        components F_x, F_y, F_z (get only)
 *   CPIC_STATE_PTAU      float64 [n][2]              the temporal-constraint check of
 *                        Appendix D (get only; SU(3), moving particles): p^tau at
 *                        step n from the constraint [eq:ptau], and p^tau integrated by
 *                        the push from its own equation of motion [eq:ptaueq] (Euler
 *                        with the rest of the particle, from the constraint at the
 *                        formation step, or at the step of the last set of
 *                        CPIC_STATE_PARTICLES; 0 before formation)
 * bytes must equal the exact size (CPIC_E_CAPACITY otherwise).  Synchronises.
 * The device keeps only the first two rows of each SU(3) link: a get returns
 * the third row as the conjugate cross product of the first two, and a set
 * uses the first two rows of each link (the third must agree with them, as it
 * does for a unitary matrix of unit determinant).
 */
#define CPIC_STATE_U 0
#define CPIC_STATE_PHI 1
#define CPIC_STATE_E 2
#define CPIC_STATE_PI 3
#define CPIC_STATE_PARTICLES 4
#define CPIC_STATE_STEP 5
#define CPIC_STATE_JET_W 6
#define CPIC_STATE_JET_F 7
#define CPIC_STATE_PTAU 8
cpic_status cpic_get_state(cpic_ctx* ctx, int32_t which, void* host_dst, size_t bytes);
cpic_status cpic_set_state(cpic_ctx* ctx, int32_t which, const void* host_src, size_t bytes);

/* Checkpoint: write / read the complete state (fields, particles, step, samples,
 * parameters) to a file.  cpic_load requires a context created with the same
 * lattice, precision and particle count.  A run resumed from a checkpoint is
 * bitwise identical to an uninterrupted one.  CPIC_E_IO on file errors. */
cpic_status cpic_save(cpic_ctx* ctx, const char* path);
cpic_status cpic_load(cpic_ctx* ctx, const char* path);

/* Field-kernel launch: tile shape in sites, whether consecutive tiles are
 * mapped onto one XCD, the occupancy the register allocator targets (waves per
 * SIMD; 1 = compiler default) and the kernel variant:
 *   0  one thread per site, stencil read from global memory (bx * by a
 *      multiple of 64, <= 256, waves 1..4);
 *   1  one thread per link (bx * by = 128, bx a multiple of 32, waves 1..3);
 *   2  one thread per site, links and scalars of the tile and its halo staged
 *      in LDS first (bx x by one of 64x4, 32x4, 64x2, 32x8, 16x8; waves 1);
 *   3  as 2 with only the first two rows of each link in LDS (the third is
 *      rebuilt) and the scalars read from global memory, so that two
 *      workgroups share a CU (64x4, 32x8, 16x16, 32x4; waves 1), or one
 *      workgroup of 512 threads with a smaller halo (64x8).
 *   4  the fused step: as 3, with the particle push of every tile in the same
 *      kernel (push mode CPIC_PUSH_TILE; 64x8, 32x8, 16x16 or 8x8; needs
 *      SU(3) particles with the rotation colour update and no light-like
 *      paths).  The particle records are reordered by these tiles before the
 *      next push step.
 * Used by the tuner; takes effect for the next launch. */
cpic_status cpic_set_launch(cpic_ctx* ctx, int32_t bx, int32_t by, int32_t xcd_remap, int32_t waves,
                            int32_t variant);

/* Push work split: wavefronts per group of 64 particles (1, 2 or 4).  The
 * helper wavefronts evaluate part of the colour fields at the particles' cells
 * while the owner wavefront rotates the charges, which shortens the chain of
 * dependent memory accesses per particle.  Default from n; cpic_tune times
 * all three. */
cpic_status cpic_set_push_lanes(cpic_ctx* ctx, int32_t lanes);

/* Where the push takes the colour fields at a particle's cell (the
 * interpolations of Sec. III.B from U(n), phi(n), E(n -+ 1/2), pi(n -+ 1/2)):
 *   CPIC_PUSH_GATHER  evaluated per particle from the two field buffer sets
 *                     of the step;
 *   CPIC_PUSH_TABLE   evaluated once per site into a force table (48 reals
 *                     per site, one more kernel per step) that the push reads
 *                     at the cell;
 *   CPIC_PUSH_TILE    the fused step (launch variant 4): the workgroup that
 *                     updates a tile of sites evaluates the fields at every
 *                     site of the tile from the values of its own update and
 *                     pushes the particles the last reordering put in the
 *                     tile, in the same kernel; particles that have left
 *                     their tile since then are pushed by a second, small
 *                     kernel that gathers their fields.  It pays where the
 *                     particles are dense enough that evaluating the fields
 *                     at every site costs less than at every particle.
 * The default is the gather push (the force table with more particles than
 * sites).
 * The three give the same arithmetic per particle up to rounding.  SU(3) with
 * the rotation colour update only for the table and tile modes; cpic_tune
 * times them.  Kernel timing counts the table kernel as push time, the fused
 * kernel as field time and the straggler kernel as push time. */
#define CPIC_PUSH_GATHER 0
#define CPIC_PUSH_TABLE 1
#define CPIC_PUSH_TILE 2
cpic_status cpic_set_push_mode(cpic_ctx* ctx, int32_t mode);
cpic_status cpic_get_push_mode(const cpic_ctx* ctx, int32_t* mode);

/* Current launch configuration: out = {bx, by, xcd_remap, waves, push lanes,
 * variant, non-temporal stores of the new state}.  The last is set at creation (and by
 * cpic_jets_enable, cpic_set_push_mode): 1 where the state, the new state
 * and what the rest of the step reads exceed the 256 MB last-level cache
 * together (FP64 at 512^2), so that the new links and phi, which only the
 * next step reads, do not displace what this step's push reads;
 * cpic_tune may change it.  Results are the same
 * either way. */
cpic_status cpic_get_launch(const cpic_ctx* ctx, int32_t out[7]);

/* Store policy of the new state in the compressed-tile field update:
 * 1 stores the new links and phi non-temporal, 0 with the default cache
 * policy (the choice cpic_get_launch reports in out[6]); the new E and pi,
 * which the push of the same step reads, always keep the default policy.
 * Results are the same either way; takes effect for the next launch. */
cpic_status cpic_set_store_policy(cpic_ctx* ctx, int32_t non_temporal);

/* Launch tuner: times every candidate field-kernel configuration (block shape x
 * occupancy target x XCD mapping) in place on the current state without
 * advancing it (the free buffer is overwritten), and, once particles are being
 * pushed, the push lanes and the force table on a saved copy of the
 * particles.  Then the three fastest field configurations, each with both
 * store policies, and the configuration before tuning run two whole steps
 * from a saved copy of the state (one extra field buffer set, allocated for
 * the duration), which is restored afterwards; the fastest step decides, but
 * the configuration before tuning stays unless another is at least 2 %
 * faster per step (timing noise does not flip between equals).  reps launches per candidate.  report
 * (may be NULL) receives a text table whose last line is the choice.
 * Synchronises. */
cpic_status cpic_tune(cpic_ctx* ctx, int32_t reps, char* report, size_t cap);

/* Kernel timing: when enabled, every field-update and particle-push launch
 * records its own start and stop times in HIP events attached to the launch
 * (steps are then launched one by one instead of from graphs).  cpic_timing
 * returns the summed kernel times in ms and the launch counts since enabling,
 * and synchronises. */
cpic_status cpic_set_timing(cpic_ctx* ctx, int32_t enable);
cpic_status cpic_timing(cpic_ctx* ctx, double* field_ms, double* push_ms, int64_t* n_field, int64_t* n_push);

/* Fused step (push mode CPIC_PUSH_TILE): the number of particle pushes the
 * straggler kernel has made since kernel timing was enabled (particles that
 * had left the tile the last reordering put them in, or that exceeded one per
 * thread of their tile); the tiles pushed the rest.  0 when timing is off or
 * the fused step did not run.  Synchronises. */
cpic_status cpic_straggler_pushes(cpic_ctx* ctx, int64_t* n);

/*
 * Light-like jet limit of the momentum broadening (Sec. V.B,
 * [eq:mombroadjets]).  A parton moving along +x at the speed of light feels
 * f_x = E_x, f_y = E_y - B_eta, f_z = E_eta + B_y (the fields of Sec. III.B at
 * its nearest grid point), seen through the Wilson line W of the x links it
 * has crossed: f~ = W f W^+.  Its broadening is g^2 times the double time
 * integral of the correlator of f~, i.e. <dp_i^2> = (q2/8) |F_i|^2 with
 * F_i = sum_n w f~_i(t_n) for charges rotated uniformly over their orbit
 * ([eq:qnpointfct_main]; q2 the classical quadratic Casimir of rep).
 *
 * The library follows one straight path per lattice site, through the same
 * event: path (y, x) starts at x + x_offset in row y at the first step n_f
 * with t_{n_f} >= tau_form / a.  After m steps it is at x + x_offset + m dt;
 * when its nearest grid point moves from c to c + x, W <- W U_x(c) with the
 * link at that step.  The force is evaluated every `stride` steps with
 * weight stride * dtau (stride 1: every step, as the particle push does;
 * stride = a / dtau: steps of one lattice spacing).  Samples are taken at
 * the same steps as the particle samples.
 *
 *   x_offset    start of every path inside its cell, in [0, 1)
 *   stride      >= 1
 *   tau_form_fm formation time of the paths (jets form at 0)
 *   rep         CPIC_REP_FUND or CPIC_REP_ADJ: the charges <dp^2> is quoted for
 *
 * The paths read the fields at their cells from the per-site force table of
 * the step (CPIC_PUSH_TABLE), which is then evaluated every step from the
 * paths' formation on, whatever the push mode.  cpic_jets_enable allocates
 * the paths' state (42 reals per site) and, if the context has none yet, the
 * force table (48 reals per site).  Call it once, before the paths'
 * formation step is reached; CPIC_E_INVALID otherwise, or if dtau > a.
 * Every later step then launches the table kernel (unless the push already
 * does) and the path kernel; kernel timing counts the table as path time
 * when the push does not read it.  Checkpoints include the paths.
 */
typedef struct {
    double x_offset;
    int32_t stride;
    double tau_form_fm;
    int32_t rep;
} cpic_jet_params;
cpic_status cpic_jets_enable(cpic_ctx* ctx, const cpic_jet_params* params);
/* Samples of the light-like broadening: out[4*k + c], c = tau_fm, <dp_x^2>,
 * <dp_y^2>, <dp_z^2> (GeV^2, averaged over the N^2 paths, fixed-order double
 * precision sums).  *n_samples (may be NULL) receives the sample count;
 * CPIC_E_CAPACITY if cap is smaller (nothing written).  Synchronises. */
cpic_status cpic_jets_observables(cpic_ctx* ctx, double* out, int32_t cap, int32_t* n_samples);
/* The light-like paths' qhat_i = d<dp_i^2>/dtau ([eq:qhati]) and the jet
 * anisotropy <dp_z^2>/<dp_y^2> ([eq:jetanisotropy]), as cpic_transport:
 * out[6*k + c], c = tau_mid, qhat_x, qhat_y, qhat_z (GeV^2 c/fm), tau_k, the
 * anisotropy at tau_k.  Synchronises. */
cpic_status cpic_jets_transport(cpic_ctx* ctx, double* out, int32_t cap, int32_t* n_samples);
/* Summed kernel time (ms) and launch count of the light-like path kernel
 * since cpic_set_timing enabled timing.  Synchronises. */
cpic_status cpic_jets_timing(cpic_ctx* ctx, double* ms, int64_t* launches);

/* Message of the last failure (never NULL; static storage for a NULL ctx). */
const char* cpic_last_error(const cpic_ctx* ctx);
void cpic_destroy(cpic_ctx* ctx);

/*
 * Batched events: n_events independent Glasma events (each with its own
 * lattice size, MV scale, particle species and step count; one precision for
 * all) evolved together.  Events are split into launch groups whose working
 * set fits the last-level cache (cpic_batch_set_group_bytes); the groups are
 * dealt to launch lanes (cpic_batch_set_lanes), and each lane runs its groups
 * one after the other, each to the end of its events.  One step of a group is
 * one batched field launch and one batched push launch (which also advances
 * the step counters) over its active events; each workgroup reads its (event, tile) or
 * (event, particle block) item from a device work map.  Runs of steps are
 * replayed from HIP graphs; events that reach their n_max drop out of the
 * work maps.  Parameter arrays have n_events entries (particles may be NULL:
 * no particles).  The batch's stream is hip_stream, or a new non-blocking
 * stream if NULL; with more than one launch lane the events also run on
 * streams of the library's own (cpic_batch_set_lanes).  Each event is also a full cpic_ctx
 * internally; per-event results are read with the functions below.  Not
 * thread-safe.
 */
cpic_status cpic_batch_create(int32_t n_events, const cpic_glasma_params* glasma,
                              const cpic_particle_params* particles, void* hip_stream, cpic_batch** out);
/* MV initial condition of every event (as cpic_init_mv); synchronises */
cpic_status cpic_batch_init_mv(cpic_batch* b);
/* run every event to its n_max; asynchronous */
cpic_status cpic_batch_run(cpic_batch* b);
/* advance every unfinished event by up to k steps (group by group); asynchronous */
cpic_status cpic_batch_step(cpic_batch* b, int32_t k);
/* wait for the batch's stream; reports the first event's particle error
 * (CPIC_E_CELL_JUMP) as cpic_sync does */
cpic_status cpic_batch_sync(cpic_batch* b);
/* Field-tile tuner: times the batched field launch for each tile shape and
 * XCD mapping over the current active events (state unchanged) and keeps the
 * fastest; report as in cpic_tune.  Synchronises. */
cpic_status cpic_batch_tune(cpic_batch* b, int32_t reps, char* report, size_t cap);
/* batched launch shape: compressed-link LDS field tiles bx x by (64x4, 32x8,
 * 16x16 or 32x4), xcd_remap 0/1, tpp = wavefronts per 64-particle group
 * (1, 2, 4) */
cpic_status cpic_batch_set_launch(cpic_batch* b, int32_t bx, int32_t by, int32_t xcd_remap, int32_t tpp);
/* Launch groups: events are taken by decreasing working set (both field
 * buffer sets and the particle records) and packed into groups of at most
 * `bytes` (a larger event forms a group of its own).  A group runs all its
 * steps before the next group of its lane starts, so its fields stay in the
 * last-level cache from one step to the next.  0 = all events in one group,
 * stepped together.  Default 96 MiB (with the default two lanes, the groups
 * running side by side share the 256 MB last-level cache). */
cpic_status cpic_batch_set_group_bytes(cpic_batch* b, int64_t bytes);
/* Launch lanes (1 to 4; default 2): the launch groups are dealt to the
 * batch stream and up to three streams of the library's own (default
 * priority), by their remaining work (largest first, each to the lane with
 * the least; odd lanes then run theirs smallest first), and the streams run
 * concurrently: the launches of small events leave most of the chip idle,
 * and a large event's latency-bound push leaves bandwidth unused, which the
 * other lane's groups take.  The events' results do not depend on the lanes
 * (each event's kernels run in the same order on one stream).
 * cpic_batch_run and cpic_batch_step end with the batch stream waiting for
 * the other lanes, so the batch stream orders everything after them
 * (cpic_batch_sync, reads of the results). */
cpic_status cpic_batch_set_lanes(cpic_batch* b, int32_t lanes);
/* out = {bx, by, xcd_remap, tpp} */
cpic_status cpic_batch_get_launch(const cpic_batch* b, int32_t out[4]);
cpic_status cpic_batch_num_events(const cpic_batch* b, int32_t* n);
cpic_status cpic_batch_current_step(const cpic_batch* b, int32_t event, int64_t* n);
/* per-event samples, layout of cpic_observables_full; synchronises */
cpic_status cpic_batch_observables(cpic_batch* b, int32_t event, double* out, int32_t cap, int32_t* n_samples);
/* per-event state access, as cpic_get_state; synchronises */
cpic_status cpic_batch_get_state(cpic_batch* b, int32_t event, int32_t which, void* host_dst, size_t bytes);
const char* cpic_batch_last_error(const cpic_batch* b);
void cpic_batch_destroy(cpic_batch* b);

#ifdef __cplusplus
}
#endif
#endif /* CPIC_H */
