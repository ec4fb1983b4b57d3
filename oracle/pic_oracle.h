/*
 * CPU oracle for one step of the 1d3v PIC-MCC oxygen rf discharge
 * (Bronold et al., "Radio-frequency discharges in Oxygen. Part 1: Modeling").
 *
 * TEST INFRASTRUCTURE ONLY.  This is the plain, slow, single-threaded
 * statement of what the hot path computes; it is used by the tests, by the
 * smoke check and by the benchmark's CPU baseline.  The product path never
 * links, loads or calls it.
 *
 * The same source is compiled twice: with real = float (liboracle32.so) and
 * with real = double (-DORACLE_FP64, liboracle64.so).
 */
#ifndef PIC_ORACLE_H
#define PIC_ORACLE_H
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define OR_NCH 19
#define OR_NPT 897

typedef struct {
  double gap_m;
  int32_t n_cells;
  double area_m2;
  double weight;
  int32_t steps_per_period;   /* dt = 1 / (f * steps_per_period) */
  int32_t ion_subcycle;
  int32_t sort_every;
  int32_t drive_dc;           /* 1: constant U = voltage (test switch) */
  int64_t n_init[3];          /* e, O-, O2+ */
  double T_init_eV[3];
  uint64_t seed;
  double voltage_V, frequency_Hz, pressure_Pa, T_gas_K, metastable_frac;
  int32_t eedf_bins;
  double eedf_emax_eV;
  int32_t fneg_xbins, fneg_ebins;
  double fneg_emax_eV;
  int32_t coulomb_every;      /* intra-species Coulomb collisions every n2 steps, 0 = off */
  double coulomb_log;         /* ln Lambda */
  int32_t coulomb_inter;      /* 1: inter-species Coulomb collisions after the intra-species ones */
  int32_t field_off;          /* test switch, 1: the particles' charge does not enter the field
                                 (rate pins at weights whose self field would swamp the step) */
  int32_t dsmc;               /* 1: collisions (4)-(19) as the per-cell list of Sec. II every sort_every
                                 steps (tau = sort_every dt) instead of null-collision Monte Carlo
                                 every step; sort_every a multiple of ion_subcycle */
} or_params;

typedef struct or_ctx or_ctx;

/* error codes (same meaning as the product library's) */
#define OR_OK 0
#define OR_EINVAL (-1)
#define OR_ENOMEM (-2)
#define OR_EGUARD (-4)
#define OR_EOVERFLOW (-5)

or_ctx* or_create(const or_params* p, const double* sigma /*[19][897] m^2*/,
                  const double* threshold_eV, const double* loss_eV, int* err);
void or_destroy(or_ctx* c);
int or_step(or_ctx* c, int64_t n_steps);

int64_t or_alive(const or_ctx* c, int sp);
/* alive particles of species sp in store order: id, cell, off, v (3 per particle) */
int64_t or_particles(const or_ctx* c, int sp, int64_t cap, uint64_t* id, int32_t* cell,
                     double* off, double* v);
/* the field the next step will use (solved from the current particles), n_cells+1 nodes */
void or_field(const or_ctx* c, double* phi, double* E);
/* Q (fixed point 2^-24) of the current alive population, [3][n_cells+1] */
void or_charge(const or_ctx* c, int64_t* Q);
/* counters: events[19], absorbed[2][3], misc[8] = {psteps, births, next_id, step,
   cycles, top_energy_hits, requests, accepted} */
void or_counters(const or_ctx* c, int64_t* events, int64_t* absorbed, int64_t* misc);
/* last complete rf-cycle sums: Q[3][Nc+1] (int64), phi[Nc+1], eedf[bins+1], fneg[xb*eb] */
void or_cycle_sums(const or_ctx* c, int64_t* Qsum, double* phisum, int64_t* eedf, int64_t* fneg);
/* derived constants: pmax[3] of the next step, Mgas[3], Mad, Mpart[3] (channels 12,13,17) */
void or_constants(const or_ctx* c, double* out /*[16]*/);

/* standalone pieces used by the pin tests */
void or_philox(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4]);
double or_sigma(const or_ctx* c, int chan, double E_eV);   /* table interpolation in `real` */
/* Poisson solve of the discrete Dirichlet problem from integer net charge q[0..N] */
void or_solve_field(int32_t N, double dx, double cphi, double cE, double U0, const int64_t* q,
                    double* phi, double* E);
/* the sampler's sin(2 pi u), cos(2 pi u) and ln u in the working precision, for n points u */
void or_math(const double* u, int64_t n, double* sn, double* cs, double* lg);
/* test hook: multiply velocity component d of every particle of species sp by f[d] */
void or_scale_velocities(or_ctx* c, int sp, const double f[3]);
/* test hook: replace the initial load (before the first step) by n[s] particles of each
   species, concatenated e, O-, O2+: cell, off in [0,1), v (3 per particle) */
int or_load(or_ctx* c, const int64_t n[3], const int32_t* cell, const double* off, const double* v);
/* event log: enable with capacity; entries of 16 doubles (see source) */
void or_log_enable(or_ctx* c, int64_t cap);
int64_t or_log_read(const or_ctx* c, double* out, int64_t cap);

#ifdef __cplusplus
}
#endif
#endif
