/*
 * pic.h -- C ABI of the MI355X (gfx950) PIC-MCC library for a capacitively
 * coupled rf discharge in oxygen with electrons, O- and O2+ (Bronold,
 * Matyash, Tskhakaya, Schneider, Fehske, "Radio-frequency discharges in
 * Oxygen. Part 1: Modeling").
 *
 * The problem statement follows the paper's abstract and Sec. II: for a given
 * external voltage and pressure the model determines the potential in the gap
 * and the distribution functions of e, O- and O2+.  A planar gap 0 <= x <= L
 * (1d3v), one electrode at x = 0 driven by U(t) = U_rf sin(2 pi f t), the
 * other grounded, both perfectly absorbing, O2 at pressure p and temperature T.
 *
 * Every step of the particle path runs in the library's HIP kernels on the
 * GPU; the host code only sequences launches, owns memory and copies results.
 *
 * Conventions
 *   - Every function returns 0 (PIC_OK) or a negative PIC_E* code.  Errors are
 *     sticky per context (except the argument checks that say otherwise);
 *     pic_last_error() returns the message of the last one.
 *   - Pointers named *_host are host memory owned by the caller; the library
 *     never keeps them after the call returns and never frees them.  All device
 *     memory is allocated and freed by the library.
 *   - One context is used by one host thread at a time.
 *   - Species indices: 0 = electrons, 1 = O-, 2 = O2+.
 */
#ifndef PIC_H
#define PIC_H
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define PIC_OK 0
#define PIC_EINVAL (-1)    /* invalid argument */
#define PIC_ENOMEM (-2)    /* device allocation failed */
#define PIC_EDEVICE (-3)   /* HIP runtime error */
#define PIC_EGUARD (-4)    /* null-collision bound exceeded 1 or non-finite state */
#define PIC_EOVERFLOW (-5) /* particle, birth or request capacity exceeded */

#define PIC_FP32 0
#define PIC_FP64 1

#define PIC_NCHAN 19        /* collision channels, numbered as below */
#define PIC_XS_NPOINTS 897  /* energy nodes E_k = 2^(-14 + k/32) (1 + (k%32)/32) eV */

/*
 * Channel numbering (Table I of the paper; reaction number in brackets):
 *   0 e+O2 elastic (4)            1-4 e+O2 vibrational v=1..4 (7)
 *   5 e+O2 Rydberg (8)            6 e+O2 dissociation 6.4 eV (9)
 *   7 e+O2 dissociation 8.6 eV (10)  8 e+O2 a1Delta_g (11)  9 e+O2 b1Sigma_g (12)
 *  10 e+O2 dissociative attachment (15)   11 e+O2 impact ionisation (18)
 *  12 e+O2+ dissociative recombination (13)  13 e+O- impact detachment (19)
 *  14 O-+O2 elastic (5)  15 O-+O2 direct detachment (16)
 *  16 O-+O2(a) associative detachment (17)  17 O-+O2+ neutralisation (14)
 *  18 O2+ + O2 charge exchange (6)
 */

typedef struct pic_ctx pic_ctx;

/* Geometry, discretisation and initial load (Sec. II). */
typedef struct {
  double gap_m;               /* L */
  int32_t n_cells;            /* cells of width L/n_cells, 4 <= n_cells <= 8192 */
  double area_m2;             /* lateral area A (the paper takes lambda_De^2 of a reference system) */
  double weight;              /* real particles per macro particle, all species */
  int32_t steps_per_period;   /* dt = 1 / (f * steps_per_period) */
  int32_t ion_subcycle;       /* ions are moved every ion_subcycle steps with tau = ion_subcycle * dt */
  int32_t sort_every;         /* particles are re-sorted into cells every sort_every steps */
  int32_t drive_dc;           /* 0: sinusoidal drive; 1: constant U = voltage (test switch) */
  int64_t n_init[3];          /* initial macro particles per species, at most 2^30 - 65536 */
  double T_init_eV[3];        /* initial Maxwellian temperatures */
  uint64_t seed;              /* Philox key */
  int32_t precision;          /* PIC_FP32 or PIC_FP64 particle state */
  int64_t capacity[3];        /* store capacity per species (< 2^30); 0 -> 2 n_init + 65536 */
  int32_t eedf_bins;          /* electron energy histogram at x = L/2, 0 <= bins <= 256 */
  double eedf_emax_eV;
  int32_t fneg_xbins;         /* O- f(E,x), E = sign(v_x) M v_x^2 / 2; xbins*ebins <= 2048 */
  int32_t fneg_ebins;
  double fneg_emax_eV;
  int32_t coulomb_every;      /* intra-species Coulomb collisions (1)-(3) every coulomb_every steps
                                 (n2 = t_c2 / dt of Sec. II); 0 = off; a multiple of sort_every */
} pic_geometry;

/* Gas and cross sections (Sec. III). */
typedef struct {
  double T_gas_K;             /* reservoir temperature; n_O2 = p / (k T) */
  double metastable_frac;     /* C: n(O2(a1Delta_g)) = C n_O2 for associative detachment */
  const double* sigma_m2;     /* host [PIC_NCHAN][PIC_XS_NPOINTS], linear in E between nodes */
  const double* threshold_eV; /* host [PIC_NCHAN], channel closed below */
  const double* loss_eV;      /* host [PIC_NCHAN], excitation energy dE of Eq. (5) */
  double coulomb_log;         /* ln(Lambda) of Eq. (2); > 0 when coulomb_every > 0 */
  int32_t coulomb_inter;      /* 0 or 1: after the like-species pass, unlike pairs (e,O-), (e,O2+),
                                 (O-,O2+) collide in each cell (binary model of Takizuka and Abe,
                                 Eq. (2) with the reduced mass and the lower of the two densities;
                                 an extension: Sec. III names only like-species collisions) */
  int32_t dsmc;               /* 0: null-collision Monte Carlo of (4)-(19) in every push (tau = the
                                 species' push interval); 1: the per-cell collision list of Sec. II
                                 instead: every sort_every steps, after the sort, the particles of
                                 each cell go through the types (4)-(19) of Table I in order, each
                                 with P = n_j sigma_j u tau of Eq. (1), tau = sort_every dt; products
                                 of a type take part in the later ones; a partner type uses the
                                 populations at its start (one partner per test particle, chosen by
                                 a hash of the two ids; the smallest test id wins a partner).
                                 Requires sort_every to be a multiple of ion_subcycle and every gas
                                 type's tau n max(sigma g) <= 1 (else PIC_EINVAL); a partner type
                                 whose N_t(c) tau W max(sigma g) / (A dx) exceeds 1 in a cell with
                                 test particles raises the guard.  Not batched: pic_step_batch
                                 steps such a discharge alone */
} pic_gas;

/*
 * Create a discharge: allocate the particle stores on the current HIP device,
 * sample the initial load (uniform x, Maxwellian v), deposit, solve the field
 * at t = 0 and take the leapfrog half step back in velocity.  The call is
 * synchronous.  Returns PIC_EINVAL for inconsistent inputs, PIC_ENOMEM when
 * device memory runs out.
 */
int pic_create(const pic_geometry* geometry, const pic_gas* gas, double voltage_V, double frequency_Hz,
               double pressure_Pa, pic_ctx** out);

/* Use this HIP stream (hipStream_t passed as void*) for all later work; NULL = the context's own. */
int pic_set_stream(pic_ctx* ctx, void* hip_stream);

/*
 * Enqueue n_steps time steps (asynchronous).  One step: field solve, push and
 * collisions of every species moved in this step, partner reactions, births
 * and, every sort_every steps, the cell sort, followed every coulomb_every
 * steps by the intra-species Coulomb collisions of Sec. III (binary model of
 * Takizuka and Abe, variance of tan(chi/2) from Eq. (2); at most 16384
 * particles of one species per cell, else PIC_EOVERFLOW) and, when the gas
 * sets coulomb_inter, by the unlike-species pairs (same limit).  Guard conditions
 * raised on the device are reported by pic_sync.
 */
int pic_step(pic_ctx* ctx, int64_t n_steps);

/*
 * Wait for the context's stream.  Returns PIC_EGUARD when the device raised a
 * guard: the null-collision bound nu_max tau of a species exceeded 1 (the
 * per-channel probabilities of Eq. (1) must sum to at most one per step) or
 * a particle's state became non-finite; PIC_EOVERFLOW when a store, the
 * birth list or the partner-request list ran out of capacity.
 */
int pic_sync(pic_ctx* ctx);

/*
 * Moments and diagnostics (synchronising).  Arrays may be NULL when not
 * wanted; the caller owns them.  What the paper reports of a discharge: the
 * densities and the potential averaged over an rf cycle (the quantities whose
 * constancy defines the periodic steady state, Sec. II), the electron energy
 * distribution at the centre of the gap and the O- distribution f(E, x) with
 * E = sign(v_x) M v_x^2 / 2 (Sec. IV), the events of each reaction of
 * Table I and the particles lost to each electrode (Sec. II).
 */
typedef struct {
  int64_t step;               /* steps taken */
  int64_t cycles;             /* complete rf cycles */
  int64_t alive[3];           /* macro particles per species */
  int64_t events[PIC_NCHAN];  /* collision events per channel since creation */
  int64_t absorbed[2][3];     /* [electrode x=0, x=L][species] */
  int64_t particle_steps;     /* particles pushed since creation */
  int64_t births;             /* particles created since creation */
  int64_t next_id;
  double* density_m3;         /* host [3][n_cells+1]: last complete rf cycle average */
  double* phi_V;              /* host [n_cells+1]: last complete rf cycle average */
  int64_t* eedf;              /* host [eedf_bins+1] counts over the last complete cycle */
  int64_t* fneg;              /* host [fneg_xbins*fneg_ebins] counts over the last complete cycle */
} pic_moments_t;
int pic_moments(pic_ctx* ctx, pic_moments_t* out);

/*
 * Alive particles of one species (synchronising), in store order: the
 * phase-space state of the 1d3v model of Sec. II, position x = (cell + off) dx
 * and the three velocity components (v_x at the half step of the leapfrog),
 * with each particle's id.  cap is the capacity of the caller's arrays (v
 * holds 3*cap doubles); *n_out receives the number of alive particles even
 * when it exceeds cap.
 */
int pic_particles(pic_ctx* ctx, int species, int64_t cap, uint64_t* id_host, int32_t* cell_host,
                  double* off_host, double* v_host, int64_t* n_out);

/*
 * Potential and field at the nodes that the next step will use (Poisson's
 * equation with the driven and the grounded electrode, Sec. II), host
 * [n_cells+1] each (synchronising).
 */
int pic_field(pic_ctx* ctx, double* phi_host, double* E_host);

/*
 * Node charge of the current alive population by linear weighting (Sec. II,
 * charge assignment), per species, fixed point: 2^24 units per macro
 * particle; host [3][n_cells+1] (synchronising).
 */
int pic_charge(pic_ctx* ctx, int64_t* Q_host);

/*
 * Timing of the fused particle kernel: enable = k >= 1 starts recording HIP
 * events around every k-th launch of it on the context's stream (k = 1: every
 * launch; the two event records add a gap of a few microseconds to each step
 * they bracket, so a larger k keeps them out of most steps), enable = 0
 * stops; a negative value is PIC_EINVAL.  pic_kernel_time syncs and returns
 * the summed duration and the number of timed launches since the last enable.
 */
int pic_timing(pic_ctx* ctx, int enable);
int pic_kernel_time(pic_ctx* ctx, double* push_ms, int64_t* launches);

/*
 * Launch shape of the fused particle kernel: number of persistent
 * workgroups (0 restores the occupancy-derived default of the current
 * shape).  Results do not depend on it; the determinism tests vary it.
 */
int pic_set_grid(pic_ctx* ctx, int32_t push_workgroups);

/*
 * Tile shape of the fused particle kernel: threads per workgroup and
 * consecutive particles per thread (a tile is their product).  The shapes
 * built are 256 x 4 (the default), 512 x 4 and 256 x 8; others return
 * PIC_EINVAL (not sticky).  Setting a shape restores its default grid.
 * Results do not depend on the shape.
 */
int pic_set_shape(pic_ctx* ctx, int32_t threads_per_workgroup, int32_t particles_per_thread);
/* The shape and persistent grid the fused particle kernel launches with. */
int pic_launch_shape(pic_ctx* ctx, int32_t* threads_per_workgroup, int32_t* particles_per_thread,
                     int32_t* push_workgroups);

/*
 * Autotuning of the launch shape: times the fused particle kernel (HIP
 * events) over steps_per_trial steps on each tile shape and a few
 * persistent-grid sizes (for the default shape the occupancy default and 1,
 * 2, 4, 6, 8 workgroups per CU; for the others their occupancy default and
 * three quarters of it) and keeps the fastest; *chosen (may be NULL)
 * receives its workgroup count, pic_launch_shape the rest.  The trial steps
 * are real steps of the discharge (run eagerly); results depend on neither
 * the shape nor the grid, so nothing else changes.
 */
int pic_autotune(pic_ctx* ctx, int64_t steps_per_trial, int32_t* chosen);

/*
 * Autotuning of the batched launches of pic_step_batch for the batch
 * ctx[0..n): times steps_per_trial batched steps (real steps of every
 * discharge) on each tile shape with two totals of push workgroups, and
 * keeps the fastest for batches led by ctx[0].  The discharges must be
 * batchable (as for pic_step_batch's batched path; else PIC_EINVAL, not
 * sticky).  Outputs may be NULL.
 */
int pic_autotune_batch(pic_ctx* const* ctx, int n, int64_t steps_per_trial, int32_t* threads_per_workgroup,
                       int32_t* particles_per_thread, int32_t* push_workgroups);

/*
 * Graph replay (enable = 1) or eager launches (0, the default).  The launch
 * sequence of a step repeats, with identical arguments, every P steps, P
 * twice the least common multiple of sort_every and coulomb_every; with
 * replay on, pic_step captures one such sequence into a HIP graph the first
 * time it stands at a step count divisible by P, and from then on launches
 * that graph for every whole period (steps in between run eagerly).  Results
 * are identical either way.  Timing (pic_timing) uses eager launches.
 * pic_set_grid and enable = 0 drop the captured graph.
 */
int pic_set_graphs(pic_ctx* ctx, int enable);

/*
 * Advance n independent discharges by n_steps steps each (the batched use of
 * the model: many voltages, pressures, gaps and grids at once).  When the
 * contexts share precision and sort and Coulomb periods, stand at the same
 * phase of the step sequence (step counts equal modulo the period of
 * pic_set_graphs) and none is timing, every kernel of a step is launched once
 * for all of them, with per-discharge constants and state in device tables
 * (allocated for ctx[0] at its first batch, kept, and grown when a larger
 * batch needs more), on ctx[0]'s stream, ordered after each context's
 * earlier work and before its later work; this path synchronises before
 * returning.  Otherwise the contexts'
 * steps are enqueued round robin, one period at a time, each on its own
 * stream (asynchronous, like pic_step); when any of them has Coulomb
 * collisions on (coulomb_every > 0) the periods are chained by events so
 * that no two contexts' steps run at the same time.  Either way every
 * discharge ends exactly as if stepped alone.  ctx[0..n) must be distinct;
 * the first error stops the work and is returned (other contexts may then
 * stand at earlier steps).
 *
 * Known limitation: large discharges with Coulomb collisions on, stepped by
 * separate pic_step calls on different streams so that their Coulomb
 * kernels run at the same time, have ended in states that differ from their
 * lone runs; the cause is not found.  pic_step_batch does not overlap them;
 * callers who step contexts concurrently themselves should order them the
 * same way when they need bit-reproducible results.
 */
int pic_step_batch(pic_ctx* const* ctx, int n, int64_t n_steps);

/*
 * For callers that cannot allocate device memory (serving loops and
 * harnesses that forbid hipMalloc and hipFree while they run): the batched
 * launches of pic_step_batch, with the batch's tables (constants, device
 * state and grid offsets of each discharge) in a fixed device array of the
 * library instead of memory allocated for the leading context.  The call
 * allocates nothing.  Limits: 1 <= n <= PIC_BATCH_STATIC_MAX discharges that
 * share precision, sort and Coulomb periods, the phase of the step sequence
 * and the device, none timing; otherwise PIC_EINVAL with a message in
 * pic_last_error(ctx[0]), no work done and the contexts still usable (the
 * error is not sticky).  Synchronising, like the batched
 * path of pic_step_batch; results are identical to it.  Every call on a GPU
 * uses that GPU's one array: calls from several host threads that overlap
 * on one GPU race and must not be made.
 */
#define PIC_BATCH_STATIC_MAX 64
int pic_step_batch_static(pic_ctx* const* ctx, int n, int64_t n_steps);

int pic_destroy(pic_ctx* ctx);
const char* pic_last_error(const pic_ctx* ctx);

#ifdef __cplusplus
}
#endif
#endif
