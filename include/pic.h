/*
 * pic.h -- C ABI of the MI355X laser-dielectric particle-in-cell hot path.
 *
 * The library advances the particle-in-cell method of arXiv 2502.13695
 * ("A Fully Three-Dimensional Kinetic Particle-In-Cell Framework for Modeling
 * Laser-Dielectric Interactions: Few-Cycle Pulse Damage") on one AMD MI355X:
 * Yee field solve with a spatially varying permittivity (Sec. 2.3), shape-
 * function gather, relativistic Boris push, Esirkepov current deposit,
 * one-cycle rolling field-amplitude window and Keldysh photoionization with
 * Monte-Carlo single ionization of neutral molecule macroparticles (Sec. 2.1),
 * driven by a laser entering through the x_min boundary (Sec. 3).
 *
 * Conventions for every call:
 *  - Return value: PIC_OK (0) or a negative pic_status.  No exception or
 *    signal crosses the ABI.  A NULL pointer where one is required gives
 *    PIC_E_INVAL.
 *  - Host pointers are plain host memory owned by the caller; the library
 *    copies what it needs before returning.  Device memory is owned by the
 *    library (through the allocator callbacks of pic_config when given, else
 *    hipMalloc) and released by pic_destroy.
 *  - A context is bound to one HIP stream (pic_config.stream, NULL = the
 *    default stream) and must be used from one host thread at a time.
 *  - Work is enqueued asynchronously; pic_diag synchronises the stream.
 *  - Errors latch: after PIC_E_NUMERIC or PIC_E_CAPACITY only pic_diag and
 *    pic_destroy are accepted.
 *  - Units are SI unless stated.  The propagation axis is x (index 0); the
 *    laser enters at x = 0.  Transverse axes are y, z.
 */
#ifndef PIC_H
#define PIC_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define PIC_ABI_VERSION 2u

typedef enum {
  PIC_OK = 0,
  PIC_E_INVAL = -1,     /* bad argument or configuration */
  PIC_E_NOMEM = -2,     /* device allocation failed */
  PIC_E_DEVICE = -3,    /* HIP runtime error */
  PIC_E_STATE = -4,     /* call not valid in the current state (latched error) */
  PIC_E_NUMERIC = -5,   /* non-finite field or particle value detected */
  PIC_E_CAPACITY = -6,  /* charged-particle buffer full */
  PIC_E_VERSION = -7    /* struct_size / abi_version mismatch */
} pic_status;

typedef struct pic_ctx pic_ctx;
typedef struct pic_batch pic_batch;

/* One dielectric (paper Table 1): band gap [eV], linear refractive index n
 * (eps_r = n^2, Sec. 2.3), mass density [g/cm^3], molar mass [g/mol] (gives the
 * molecular density n0 = rho N_A / M), effective hole and electron masses in
 * units of m_e (reduced mass m* = 1/(1/m_e* + 1/m_h*), Sec. 3.2).  Ionized
 * electrons carry m_e* (Sec. 3.2).  pos_mass_kg: mass of the positive carrier
 * born with each electron; 0 selects the molecule mass M / N_A.
 *
 * Dispersive response (the linear response of Sec. 2.3 made frequency
 * dependent): lorentz_lambda_m > 0 selects a single-pole Lorentz medium,
 *   eps(w) = eps_inf + deps w0^2 / (w0^2 - w^2 - i g w),
 * w0 = 2 pi c / lorentz_lambda_m, g = lorentz_gamma_s [1/s], with deps chosen
 * so that Re eps at the laser frequency is n_index^2 (n stays the index at the
 * laser wavelength; the resonance must lie above the laser frequency and
 * eps_inf <= n^2).  Per E position the polarisation Q = P/eps0 and its current
 * K = dt J_p / eps0 advance as K^{n+1/2} = a K^{n-1/2} + c deps E^n - c Q^n,
 * Q^{n+1} = Q^n + K^{n+1/2} (a = (1 - g dt/2)/(1 + g dt/2), c = (w0 dt)^2 /
 * (1 + g dt/2)), and K enters the E update beside the free current with
 * 1/eps_inf.  pic_init returns PIC_E_INVAL when the coupled update is unstable
 * at the time step (lossless von Neumann bound: c < 4 and sum_d C_d^2 <=
 * eps_inf - c deps / (4 - c), with the vertex condition of that bound).
 * lorentz_lambda_m = 0: static eps_r = n^2 (eps_inf and lorentz_gamma_s unused).
 *
 * Impact ionization (the paper's future work, Sec. 2.2: Keldysh's impact
 * rate): impact_rate_s = P > 0 lets every electron of this material in a cell
 * of this material ionize, once per step at most, with probability
 * 1 - exp(-w dt), w = P (eps / E_th - 1)^2 above E_th = E_g (1 + 2 mu)/(1 + mu),
 * mu = m_e* / m_h*, eps its kinetic energy.  The decisions of a cell's electrons
 * are taken in a fixed order keyed by their ids; an event consumes the cell's
 * alive neutral of lowest index (a photoionization-like birth at its position)
 * and takes E_g from the impacting electron.  0: none; negative: PIC_E_INVAL.
 * Runs with impact ionization cannot join a batch.
 *
 * Kerr response (the nonlinear extension of the linear optics, which the
 * paper leaves out): kerr_n2_m2W = n2 > 0 adds chi3 E^3 to the displacement of
 * each E component, chi3 = (4/3) n^2 eps0 c n2 (a linearly polarised wave
 * then sees n + n2 I); the update advances the displacement by the curl and
 * the currents and solves the cubic for E at every interior position of the
 * material.  0: linear; negative: PIC_E_INVAL. */
typedef struct {
  double gap_eV, n_index, density_gcc, molar_mass_gmol, me_star, mh_star, pos_mass_kg;
  double lorentz_lambda_m, eps_inf, lorentz_gamma_s;
  double impact_rate_s;
  double kerr_n2_m2W;
} pic_material;

/* Optical region (Sec. 2.3): material `material` fills lo_m <= x < hi_m across
 * the whole transverse extent.  The first matching layer wins; no layer means
 * vacuum.  The same predicate places the neutral molecules (at cell centres)
 * and the permittivity (at each E component's own staggered position). */
typedef struct {
  int32_t material;
  int32_t reserved;
  double lo_m, hi_m;
} pic_layer;

enum { PIC_ENV_GAUSS = 0, PIC_ENV_SIN2 = 1 };

/* Laser pulse entering at x = 0 (Sec. 3).  Field at the boundary:
 *   E(t) = E0 env(t) cos(omega (t - t_peak) + cep)  x  exp(-r^2 / waist^2)
 * with env = exp(-2 ln2 (t - t_peak)^2 / fwhm^2) (PIC_ENV_GAUSS) or sin^2 with
 * intensity FWHM fwhm (PIC_ENV_SIN2, Sec. 3).  Peak intensity I0 from
 * peak_Wcm2, or from fluence_Jcm2 > 0 as I0 = F / int(env^2 dt) (peak on-axis
 * fluence F = 2 E_las / (pi w0^2), Sec. 3); E0 = sqrt(2 I0 / (c eps0)).
 * t_peak_s = 0 selects 3 fwhm (Gaussian) or the sin^2 centre.  waist_m = 0 is
 * a plane wave.  pol_axis: 1 = y, 2 = z. */
typedef struct {
  double lambda_m, fwhm_s, peak_Wcm2, fluence_Jcm2, waist_m, t_peak_s, cep_rad;
  int32_t envelope, pol_axis;
} pic_laser;

enum { PIC_BC_OUTFLOW = 0, PIC_BC_PERIODIC = 1 };

/* Run configuration.  Copied by pic_init; the caller keeps ownership. */
typedef struct {
  uint32_t struct_size;        /* sizeof(pic_config) */
  uint32_t abi_version;        /* PIC_ABI_VERSION */
  int32_t ndim;                /* 1, 2 or 3 */
  int32_t transverse_bc;       /* PIC_BC_OUTFLOW (Sec. 3.1) or PIC_BC_PERIODIC */
  int64_t n[3];                /* cells per axis (unused axes ignored) */
  double dx_m[3];              /* cell size per axis [m] */
  double cfl;                  /* fraction of the CFL limit (Sec. 3.1: 0.95) */
  int64_t nsteps;              /* planned steps (sizes the laser source table) */
  int32_t nmat, nlayer;
  const pic_material* mats;
  const pic_layer* layers;
  int32_t ppc;                 /* neutral macroparticles per material cell (Sec. 3.1) */
  int32_t shape_order;         /* 1 or 2 (B-spline order of the particle shape) */
  double T_K;                  /* neutral temperature (Sec. 3.1: 300 K) */
  int32_t keldysh_terms;       /* terms of the Eq. (3) series (Sec. 2.1: 500) */
  int32_t keldysh_tol_bits;    /* the series stops early once a bound of its
                                  remaining tail is below 2^-bits of the partial
                                  sum (the adaptive tolerance the paper names as
                                  future work); 0 = 60 (full FP64 accuracy);
                                  1 .. 60, else PIC_E_INVAL */
  uint64_t seed;               /* Philox key */
  pic_laser laser;
  int64_t particle_capacity;   /* charged-particle slots; 0 = 2 x neutrals + 4096 */
  double preionize_eV;         /* >0: every neutral starts ionized, carriers thermal at
                                  this temperature (charged-loop stress variant) */
  int32_t collisions;          /* 1: binary Coulomb collisions among all charged
                                  particles every step, after ionization (Sec. 2.2,
                                  Eq. 4: the Perez/Nanbu model; pairing per cell and
                                  kind, relativistic kinematics, Coulomb logarithm
                                  per collision with a lower bound of 1, the
                                  low-temperature cap).  0: none.  A run with
                                  collisions cannot join a batch (PIC_E_INVAL). */
  int32_t reserved2;
  void* stream;                /* hipStream_t, or NULL for the default stream */
  void* (*alloc)(size_t bytes, void* user);   /* optional device allocator */
  void (*free)(void* ptr, void* user);
  void* alloc_user;
} pic_config;

/* Canonical discrete problem derived from a configuration (host-only query).
 * dt is the largest value with c dt / dx_0 an FP32 number not above the
 * requested fraction of the CFL limit (Sec. 3.1); Cd[d] = c dt / dx_d and
 * kmur[d] = (Cd - 1)/(Cd + 1) are FP32 numbers; ie[m] = 1/n_m^2 as FP32
 * (a Lorentz material: 1/eps_inf); lor[m] = (a, c, c deps) of its oscillator
 * as FP32 numbers (zeros for a static material);
 * nwin = ceil(lambda / (c dt)) samples make one laser cycle (Sec. 2.1). */
typedef struct {
  double dt;
  double Cd[3];
  double kmur[3];
  double ie[8];
  int64_t nwin;
  double E0;                   /* peak boundary field [V/m] */
  double t_peak;               /* envelope centre [s] */
  double amp_cut[8];           /* per material: amplitudes below cannot ionize [V/m] */
  double amp_sat[8];           /* per material: amplitudes above ionize with P = 1 */
  int64_t n_neutral;           /* neutral macroparticles loaded */
  int64_t capacity;            /* charged slots */
  double lor[8][3];            /* per material: Lorentz oscillator coefficients */
  double chi3[8];              /* per material: Kerr chi3 [m^2/V^2] as FP32 (0: linear) */
} pic_params;

/* Diagnostic kinds for pic_diag.  Grids are FP64 unless stated, on the
 * positions inside the box, x fastest. */
enum {
  PIC_DIAG_SCALARS = 0,   /* double[PIC_SC_COUNT], see PIC_SC_* */
  PIC_DIAG_FIELDS = 1,    /* double: Ex, Ey, Ez, bx, by, bz (b = cB) on their own
                             staggered positions; per component the shape is
                             n_d (half-integer or periodic axis) or n_d + 1 */
  PIC_DIAG_NE_GRID = 2,   /* electron number density at nodes [m^-3] (Sec. 4.1) */
  PIC_DIAG_UE_GRID = 3,   /* electron kinetic energy density at nodes [J/m^3] (Sec. 4.2) */
  PIC_DIAG_EVENTS = 4,    /* int64 pairs (neutral id, step) of every ionization so far */
  PIC_DIAG_PARTICLES = 5, /* pic_particle records of live charged particles */
  PIC_DIAG_PARAMS = 6,    /* one pic_params */
  PIC_DIAG_AMP = 7,       /* float: windowed amplitude A at nodes [V/m] */
  PIC_DIAG_TIMERS = 8,    /* double[32]: [0..7] device ms per phase summed over the
                             timed launches, [8..15] launch counts (phases: 0 push,
                             1 field update with outflow faces and amplitude window,
                             2 ionization, 3 tile sort); [16..22] autotuner ms per field launch of
                             each tile shape (best block count), [23] the tile shape in
                             use, [24] field blocks per launch, [25] push blocks */
  PIC_DIAG_SORT = 9,      /* double[4]: charged slots held in tile order, tile
                             chunks, drifter-steps (a particle that deposited outside
                             its tile's window, counted per step) since the last
                             sort, sorts performed */
  PIC_DIAG_REGION = 10,   /* double[6]: charged region along x that the next step's
                             field update uses (first and last cell that held a
                             charged particle so far, together with the amplitude
                             window's cells; lo > hi when empty), then the field
                             tiles that read the current and the far tiles that
                             skip it (see pic_set_far_tiles), then the field front:
                             the last x node of a field tile that has held a
                             nonzero E or b, then the field tiles updated so far,
                             summed over the field launches */
  PIC_DIAG_IMAX = 11,     /* float: maximum accumulated intensity at nodes, the
                             largest node |E|^2 [V^2/m^2] over the samples taken
                             since pic_set_imax (zero when never enabled) */
  PIC_DIAG_TRACKS = 12,   /* pic_track records taken since pic_set_tracks, sorted
                             by (id, kind, step) */
  PIC_DIAG_HEALTH = 13,   /* double[4]: the device health word (bit 0 charged-slot
                             capacity exceeded by births, bit 1 a non-finite E value
                             stored by the field update, a non-finite particle
                             momentum or a non-finite window amplitude), the latched
                             pic_status, the device step index, the charged slots
                             in use.  Valid in every state, including after a
                             latched error. */
  PIC_DIAG_POL = 14       /* double: Qx, Qy, Qz (P / eps0 [V/m], at step n), then
                             Kx, Ky, Kz (dt J_p / eps0 [V/m], at step n - 1/2) of the
                             Lorentz media, each on its E component's positions
                             (shapes of the E part of PIC_DIAG_FIELDS); zero
                             outside Lorentz media and everywhere in runs without one */
};

/* PIC_DIAG_SCALARS layout (all double). */
enum {
  PIC_SC_STEP = 0, PIC_SC_TIME = 1, PIC_SC_N_NEUTRAL = 2, PIC_SC_N_E = 3, PIC_SC_N_POS = 4,
  PIC_SC_EVENTS = 5, PIC_SC_U_FIELD = 6, PIC_SC_KE_E = 7, PIC_SC_KE_POS = 8,
  PIC_SC_E_GAP = 9, PIC_SC_E_ABS = 10, PIC_SC_GAUSS_MAX = 11, PIC_SC_RHO_MAX = 12,
  PIC_SC_HEALTH = 13, PIC_SC_SLOTS = 14, PIC_SC_TRACKS_DROPPED = 15,
  PIC_SC_GAUSS_L2 = 16,   /* root mean square of the Gauss-law residual over the interior nodes [V/m^2];
                             the residual is div(E/ie + Q) - rho/eps0, Q = P/eps0 of Lorentz media */
  /* Field-side energy budget (a reading of Sec. 4.2's absorbed energy): field
   * energy carried through the flux surface since the start [J], entering and
   * leaving.  The surface bounds the box whose faces are the node planes one
   * cell inside the outflow faces (periodic axes: the whole period); on it the
   * Poynting vector eps0 c (E x b) uses E at the half step, (E^n + E^{n+1})/2,
   * and b^{n+1/2} averaged to the plane, integrated with the trapezoid rule
   * (absent axes count 1 m).  Each staggered product E_a b_b is one term; a
   * term's energy goes to E_IN when it points into the box, else to E_OUT.
   * E_IN - E_OUT - U_FIELD is the energy the charges took from the field (in
   * Lorentz media U_FIELD counts eps0/2 (eps_inf E^2 + b^2) only, so the
   * difference also holds the energy the oscillators store). */
  PIC_SC_E_IN = 17, PIC_SC_E_OUT = 18,
  PIC_SC_COUNT = 19
};

/* A charged macroparticle: cell indices, FP32 offsets in [0, 1) (position =
 * cell + offset, in cells), u = gamma v / c, kind = 2 * material (electron) or
 * 2 * material + 1 (positive carrier). */
typedef struct {
  int32_t cell[3];
  int32_t kind;
  float off[3];
  float u[3];
} pic_particle;

/* State written by pic_set_state: E and b (FP32, layout of PIC_DIAG_FIELDS),
 * the charged particles, and the step index.  Neutrals and the amplitude
 * window keep their values unless reset_window != 0 (window cleared).  The
 * polarisation of Lorentz media restarts from rest (Q = K = 0). */
typedef struct {
  int64_t step;
  const float* E[3];
  const float* b[3];
  int64_t n_particles;
  const pic_particle* particles;
  int32_t reset_window;
  int32_t reserved;
} pic_state;

/* Create a context: canonicalise the configuration, build the FP64 Keldysh
 * rate table per material (Sec. 2.1, Eq. 1-3), allocate device state, load the
 * neutrals (Sec. 3.1).  Returns PIC_E_VERSION on a struct_size/abi_version
 * mismatch, PIC_E_INVAL on a bad configuration (including a guarded grid of
 * 2^30 points or more, or a charged capacity above 2^30), PIC_E_NOMEM /
 * PIC_E_DEVICE. */
pic_status pic_init(const pic_config* cfg, pic_ctx** out);

/* Enqueue nsteps time steps (Sec. 1-2 loop: gather, push, deposit, field
 * update, amplitude window, ionization).  Asynchronous on the context stream. */
pic_status pic_step(pic_ctx* c, int64_t nsteps);

/* Copy a diagnostic into host_out (out_bytes available); *written gets the
 * byte count.  host_out == NULL queries the size only.  Synchronous.
 * Returns PIC_E_INVAL if out_bytes is too small. */
pic_status pic_diag(pic_ctx* c, int kind, void* host_out, size_t out_bytes, size_t* written);

/* Overwrite fields, charged particles and step index (parity tests, restarts). */
pic_status pic_set_state(pic_ctx* c, const pic_state* s);

/* Device bytes pic_init would allocate for this configuration (admission
 * control).  Host-only. */
pic_status pic_footprint(const pic_config* cfg, size_t* bytes);

/* Canonical parameters of a configuration without creating a context.
 * Host-only (no GPU needed). */
pic_status pic_canonical(const pic_config* cfg, pic_params* out);

/* FP64 Keldysh rate W(A) [m^-3 s^-1] of Eq. (2)-(3) for n amplitudes A [V/m]
 * with `terms` series terms, as the table builder evaluates it.  Host-only. */
pic_status pic_keldysh_rate(const pic_material* m, double lambda_m, int32_t terms,
                            const double* A, int64_t n, double* W_out);

/* Per-step ionization probability P(A) = 1 - exp(-W dt / n0) for material
 * `mat` of `cfg`, looked up in the FP32 table exactly as the device does, for
 * n FP32 amplitudes.  Host-only (builds the table on the host). */
pic_status pic_table_probe(const pic_config* cfg, int32_t mat, const float* A, int64_t n,
                           float* P_out);

/* Bound the ionization step uses to skip a neutral before it reads the
 * neutral's amplitude (Sec. 2.1, Eq. 1-3 through the table): for each of n
 * FP32 amplitudes A, a value B(A) >= the table lookup of every FP32 amplitude
 * A' <= A, nondecreasing in A, 0 below the cut and 1 from saturation on.  A
 * draw (w + 1/2) 2^-32 >= B(A) can fire for no amplitude up to A.  Host-only;
 * same arguments and errors as pic_table_probe. */
pic_status pic_table_bound_probe(const pic_config* cfg, int32_t mat, const float* A, int64_t n,
                                 float* B_out);

/* The same lookup executed on the device of context c (host in/out buffers). */
pic_status pic_table_probe_device(pic_ctx* c, int32_t mat, const float* A, int64_t n,
                                  float* P_out);

/* Batching of independent instances (fluence scans): one launch per phase
 * advances every member.  Members keep their own step counters; a member
 * added with pic_batch_add joins at the next step boundary.  pic_batch_step
 * replays one sort period of batch steps (8) as a HIP graph, captured on a
 * private stream at the first full period after a change of membership and
 * launched on the members' stream; the steps before the next period boundary
 * and the remainder run eagerly.  Results are those of eager stepping. */
pic_status pic_batch_create(pic_ctx* const* members, int32_t n, pic_batch** out);
pic_status pic_batch_step(pic_batch* b, int64_t nsteps);
/* Graph replay of batch steps on (default) or off; off steps eagerly. */
pic_status pic_batch_set_graph(pic_batch* b, int32_t on);
/* Graph replays launched so far (each is one sort period of batch steps). */
int64_t pic_batch_graph_replays(const pic_batch* b);
pic_status pic_batch_add(pic_batch* b, pic_ctx* c);
pic_status pic_batch_remove(pic_batch* b, pic_ctx* c);
void pic_batch_destroy(pic_batch* b);

/* Field-kernel autotuner: times each tile shape of the fused field update
 * (reps launches each, HIP events) on the context's real launch, keeps the
 * fastest and restores the initial (all-zero field) state.  Valid only before
 * the first step of a run without pre-ionization (else PIC_E_STATE).  The
 * measured ms per launch and the chosen variant are in PIC_DIAG_TIMERS. */
pic_status pic_autotune(pic_ctx* c, int32_t reps);

/* In-run variant of the tuner: the next reps x (number of shapes) steps of
 * pic_step cycle the tile shapes, reps consecutive steps each (every shape
 * computes identical fields), timing each field launch with HIP events; then
 * the shape with the fastest launch is kept for the rest of the run (one host
 * synchronisation when the tuning window ends).  Valid at any step of a single
 * run; reps in 1..16; PIC_E_STATE while a tuning window is open. */
pic_status pic_autotune_steps(pic_ctx* c, int32_t reps);

/* Device time of each step phase measured with HIP events that the phase's
 * own dispatches stamp (start of its first kernel, end of its last) on the
 * stream it runs on, for one step in every `on` consecutive steps (1 = every
 * step; 0 = off, the default); the sampled position inside each window of `on`
 * steps advances by one per window, so a phase that runs every r steps with r
 * dividing `on` (the tile sort check) is sampled in proportion.  No host synchronisation per
 * step.  Phases: 0 push, 1 field update, 2 ionization, 3 tile sort.
 * Switching resets the accumulators. */
pic_status pic_set_timing(pic_ctx* c, int32_t on);

/* Checkpoint and resume.  pic_snapshot writes the whole simulation state:
 * fields, currents, the amplitude window, the charged particles (with their
 * ids), the neutrals' alive bits and death steps, the device counters and the
 * step index, after an 80-byte header.  host_out = NULL: size query (written =
 * bytes needed).  Synchronous.  The maximum accumulated intensity and the
 * trajectory records are diagnostics, not part of it.  pic_restore loads such a
 * snapshot into a context created from the same configuration (the header
 * carries a key of the problem and the state layout), so that stepping
 * continues from it.  The random draws are keyed by (id, step) and carry no
 * state, so the continuation takes the same decisions; the fields agree with
 * an uninterrupted run to the rounding of FP32 atomic additions.  A restore
 * clears a latched error unless the snapshot itself carries one.  Errors:
 * PIC_E_INVAL (short buffer, another configuration), PIC_E_VERSION (not a
 * snapshot of this format), PIC_E_DEVICE. */
pic_status pic_snapshot(pic_ctx* c, void* host_out, size_t out_bytes, size_t* written);
pic_status pic_restore(pic_ctx* c, const void* host_in, size_t in_bytes);

/* Maximum accumulated intensity (Sec. 5, multilayer mirror: the intensity is
 * recorded at fixed intervals, 0.5 fs in the paper, and each point keeps its
 * largest value over the run).  every > 0: after the field update of each
 * step whose new step index is a multiple of `every`, every domain node's
 * |E|^2 raises the node's running maximum.  The node |E| is the one the
 * amplitude window uses: Yee components averaged to the node, positions
 * outside the box counted as zero, periodic axes wrapped; FP32.  Enabling
 * (again) clears the maximum; every = 0 stops sampling and keeps it.  Read with
 * PIC_DIAG_IMAX.  The maximum takes 4 bytes per padded grid point, allocated on
 * the first enable (through the configuration's allocator when it has one).
 * A batch does not sample: pic_batch_step returns PIC_E_STATE while a member
 * has sampling on.  Errors: PIC_E_INVAL (every < 0), PIC_E_NOMEM,
 * PIC_E_STATE (latched error). */
pic_status pic_set_imax(pic_ctx* c, int32_t every);

/* Energy histogram of the charged macroparticles (Sec. 5: histograms of the
 * electrons' energy in one layer at a given time, fitted with a chi^2 law).
 * The particles whose x cell lies in [x_lo_cell, x_hi_cell) (every cell when
 * x_hi_cell <= x_lo_cell) are counted per kind by kinetic energy
 * KE = m c^2 |u|^2 / (gamma + 1) [eV], gamma = sqrt(1 + |u|^2), evaluated in
 * FP64 from the FP32 u with every operation rounded on its own, in the order
 * written (|u|^2 summed x, y, z).  Bin edges are the caller's (strictly
 * increasing, finite, 2 .. 4097 of them). */
typedef struct {
  int32_t nedges;
  const double* edges_eV;    /* host array of nedges bin edges [eV] */
  int64_t x_lo_cell, x_hi_cell;
} pic_spectrum;

/* Synchronous.  out (host, out_count = 2 * nmat * (nedges + 1) entries): one
 * row per kind (2 m electron, 2 m + 1 positive carrier of material m); column 0
 * counts KE below the first edge, column j (1 .. nedges - 1) KE in
 * [edge j-1, edge j), column nedges KE at or above the last edge.  The counts
 * are exact (integers).  Edges and counts use a 0.5 MB device buffer allocated
 * on the first call (through the configuration's allocator when it has one).
 * Errors: PIC_E_INVAL (bad edges, range beyond int32 or out_count),
 * PIC_E_NOMEM, PIC_E_DEVICE. */
pic_status pic_spectrum_counts(pic_ctx* c, const pic_spectrum* s, uint64_t* out, size_t out_count);

/* The same energy histogram without any device allocation, for callers that
 * cannot allocate device memory mid-run (code inside HIP graph capture, tight
 * serving loops, hosts that forbid hipMalloc): the edges and counts are staged
 * in a fixed device array of the library (557 KB, one per GPU, held until the
 * process ends; its address is resolved once per GPU by pic_init).  Same
 * arguments, limits (at most 4097 edges, else PIC_E_INVAL) and results as
 * pic_spectrum_counts.  Every call on one GPU shares that array: calls that
 * overlap in time on one GPU (from several threads, or contexts on different
 * streams) race and must be serialised by the caller.  Errors: PIC_E_INVAL,
 * PIC_E_DEVICE. */
pic_status pic_spectrum_counts_noalloc(pic_ctx* c, const pic_spectrum* s, uint64_t* out, size_t out_count);

/* A recorded position of a sampled particle: id (the parent neutral's id,
 * cell index x ppc + k; particles placed by pic_set_state: cells x ppc + their
 * index), kind, the step index after which it was taken, and the position
 * (cell + offset, as in pic_particle; absent axes 0). */
typedef struct {
  uint32_t id;
  int32_t kind;
  int32_t step;
  int32_t cell[3];
  float off[3];
  int32_t reserved;
} pic_track;

/* Trajectory sampling (Sec. 5: tracks of a random 2 % of the electrons).  A
 * particle is sampled iff the first 32-bit word of the Philox-4x32-10 block
 * with key (seed) and counter (id, 0, 6) is below `threshold` (fraction x 2^32):
 * an electron and its positive carrier, which share the id, go together, and
 * the choice does not depend on where the particle sits.  every > 0: after
 * each step whose new step index is a multiple of `every`, every sampled live
 * particle appends one pic_track; records beyond max_records are dropped and
 * counted (PIC_SC_TRACKS_DROPPED).  Enabling clears the records; every = 0
 * stops recording and keeps them.  Read with PIC_DIAG_TRACKS.  The records take
 * 40 B each plus 256 B, allocated here (through the configuration's allocator
 * when it has one).  A batch does not record: pic_batch_step returns
 * PIC_E_STATE while a member records.  Errors: PIC_E_INVAL (negative
 * arguments, or ids that do not fit 32 bits: cells x ppc + capacity >= 2^32),
 * PIC_E_NOMEM, PIC_E_STATE (latched error). */
pic_status pic_set_tracks(pic_ctx* c, uint32_t threshold, int32_t every, int64_t max_records);

/* Far field tiles (default on): the push tracks on the device every x cell
 * that has held a charged particle at any step so far.  A field tile whose x
 * column lies farther than 6 cells from all of them and from the amplitude
 * window has carried no current at any step (a step's deposit stays within 3
 * cells of the particle's cell), so its update neither reads nor clears the
 * current: 48 instead of 72 bytes per cell.  A far tile whose staged x range
 * (tile plus 2 cells) also lies beyond the field front (the last x column of
 * a tile that has stored a nonzero E or b) has only zero inputs; it is not
 * updated at all, its outputs being zero already.  Results are identical
 * either way; on = 0 makes every tile read its current and be updated (for
 * comparison).  Batches always skip. */
pic_status pic_set_far_tiles(pic_ctx* c, int32_t on);

/* Tile sort of the charged particles (the resort of the particle loop): every
 * `period` steps (default 8; 0 = never) the device checks whether births
 * since the last sort exceed 1/32 of the slots in use, or the particles that
 * started a step outside their tile, summed over the steps since the sort,
 * exceed 1/16 of them (at least 256 either way), and if so counting-sorts
 * the charged particles by tile of the deposit (compacting dead slots).  The
 * order of the slots returned by PIC_DIAG_PARTICLES changes with each sort;
 * physics results do not (only the summation order of the current).  A batch
 * checks every 8 batch steps. */
pic_status pic_set_resort(pic_ctx* c, int32_t period);

void pic_destroy(pic_ctx* c);
const char* pic_status_str(pic_status s);

#ifdef __cplusplus
}
#endif

#endif /* PIC_H */
