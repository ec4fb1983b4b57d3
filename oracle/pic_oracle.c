/*
 * CPU oracle for the per-step particle work of the 1d3v PIC-MCC model of a
 * capacitively coupled rf discharge in oxygen (Bronold et al., Sec. II-III).
 *
 * TEST INFRASTRUCTURE ONLY: the tests, the smoke check and the benchmark's CPU
 * baseline use it; the product library never does.  It is deliberately plain:
 * one thread, arrays of structs, loops in the order the step is defined, no
 * blocking, no incremental bookkeeping (charge and counts are recomputed from
 * the particles every step).
 *
 * What one step n computes (each piece cites the passage it follows):
 *   1. charge assignment by linear weighting (Sec. II, item (i)), as 24-bit
 *      fixed point per node;
 *   2. the potential from Poisson's equation with U(t) = U_rf sin(2 pi f t) on
 *      the electrode at x = 0 and ground at x = L (Sec. II), written as the
 *      exact discrete Green's function of the 3-point Dirichlet problem;
 *   3. for each species moved this step (electrons every step, ions every
 *      ion_subcycle steps): linear-interpolated field, leapfrog push along x,
 *      absorption at both electrodes (Sec. II);
 *   4. null-collision Monte Carlo whose per-channel probability is
 *      P_j = n_j sigma_j u_j tau_j, Eq. (1), over the reaction set of Table I;
 *      gas targets drawn from a Maxwellian at the gas temperature (Sec. III B);
 *      isotropic binary collisions (Sec. III A), inelastic ones with
 *      u' = sqrt(u^2 - 2 dE / m_ab), Eq. (5); production/loss rules of
 *      Sec. III C; associative detachment with n_Delta = C n_O2 (Sec. III C);
 *   5. partner reactions (13), (14), (19) with one particular partner from the
 *      same cell (Eq. (1) and the cell sorting of Sec. II), claims resolved so
 *      that each particle is consumed at most once;
 *   6. newborn particles appended with canonical ids; periodic re-sort into
 *      cells, which also defines the partner populations of the cells.
 *
 * Randomness: Philox4x32-10 (Salmon, Moraes, Dror, Shaw, SC'11), counter
 * (id_lo, id_hi, n, k), key = 64-bit seed.  The samplers' sin, cos and ln are
 * fixed-term series evaluated in `real` (see the elementary functions below).
 */
#include "pic_oracle.h"

#include <math.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#ifdef ORACLE_FP64
typedef double real;
#define RSQRT(x) sqrt(x)
#define RFLOOR(x) floor(x)
#else
typedef float real;
#define RSQRT(x) sqrtf(x)
#define RFLOOR(x) floorf(x)
#endif

#define NCH OR_NCH
#define NPT OR_NPT
#define ONE_FIX ((int64_t)1 << 24)
#define ID_MASK ((((uint64_t)1) << 40) - 1)

enum { SP_E = 0, SP_N = 1, SP_P = 2 };

/* SI constants (CODATA 2018) */
static const double QE = 1.602176634e-19;
static const double KB = 1.380649e-23;
static const double EPS0 = 8.8541878128e-12;
static const double ME = 9.1093837015e-31;
static const double AMU = 1.66053906660e-27;
static const double TWO_PI = 6.283185307179586;
static const double PI = 3.141592653589793;

/* ----------------------------------------------------------------------- */
/* Philox4x32-10                                                            */
/* ----------------------------------------------------------------------- */
void or_philox(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4]) {
  uint32_t x0 = ctr[0], x1 = ctr[1], x2 = ctr[2], x3 = ctr[3];
  uint32_t k0 = key[0], k1 = key[1];
  for (int r = 0; r < 10; r++) {
    uint64_t p0 = (uint64_t)0xD2511F53u * x0;
    uint64_t p1 = (uint64_t)0xCD9E8D57u * x2;
    uint32_t y0 = (uint32_t)(p1 >> 32) ^ x1 ^ k0;
    uint32_t y1 = (uint32_t)p1;
    uint32_t y2 = (uint32_t)(p0 >> 32) ^ x3 ^ k1;
    uint32_t y3 = (uint32_t)p0;
    x0 = y0; x1 = y1; x2 = y2; x3 = y3;
    k0 += 0x9E3779B9u;
    k1 += 0xBB67AE85u;
  }
  out[0] = x0; out[1] = x1; out[2] = x2; out[3] = x3;
}

static void rng(uint64_t seed, uint64_t id, uint32_t n, uint32_t k, uint32_t w[4]) {
  uint32_t ctr[4] = {(uint32_t)id, (uint32_t)(id >> 32), n, k};
  uint32_t key[2] = {(uint32_t)seed, (uint32_t)(seed >> 32)};
  or_philox(ctr, key, w);
}

/* uniform on (0,1) in the working precision, exact */
static real unif(uint32_t w) {
#ifdef ORACLE_FP64
  return ((double)w + 0.5) * 0x1p-32;
#else
  return ((float)(w >> 9) + 0.5f) * 0x1p-23f;
#endif
}

/* 52-bit uniform on (0,1) in double, exact; used for every collision decision */
static double unif52(uint32_t a, uint32_t b) {
  uint64_t m = ((uint64_t)a << 20) | (uint64_t)(b >> 12);
  return ((double)m + 0.5) * 0x1p-52;
}

/* ----------------------------------------------------------------------- */
/* elementary functions of the samplers, in the working precision           */
/*                                                                          */
/* sin and cos of 2 pi u: u = (k + f)/4 with |f| <= 1/2, Taylor series of   */
/* sin(pi f / 2) and cos(pi f / 2) in f (6/7 terms in float, 10/11 in       */
/* double), then the quadrant k.  ln u: u = m 2^e with m in [1/sqrt2,       */
/* sqrt2), ln m = 2 atanh(s) = 2 s (1 + s^2/3 + s^4/5 + ...), s = (m-1)/    */
/* (m+1) (6 terms in float, 12 in double).  Fixed term counts and Horner    */
/* order, so the result is a fixed sequence of IEEE operations.  The        */
/* coefficients are formed in double and rounded once.                      */
/* ----------------------------------------------------------------------- */
#ifdef ORACLE_FP64
#define NSIN 10
#define NCOS 11
#define NLOG 12
#else
#define NSIN 6
#define NCOS 7
#define NLOG 6
#endif
static real SINC[NSIN], COSC[NCOS], LOGC[NLOG], LN2R, SQRT2R;

static void init_series(void) {
  const double h = 1.5707963267948966; /* pi / 2 */
  const double t = h * h;
  double c = h, d = 1.0;
  for (int j = 0; j < NSIN; j++) {
    SINC[j] = (real)c;
    c = (c * -t) / (double)((2 * j + 2) * (2 * j + 3));
  }
  for (int j = 0; j < NCOS; j++) {
    COSC[j] = (real)d;
    d = (d * -t) / (double)((2 * j + 1) * (2 * j + 2));
  }
  for (int k = 0; k < NLOG; k++) LOGC[k] = (real)(1.0 / (double)(2 * k + 1));
  LN2R = (real)0.6931471805599453;
  SQRT2R = (real)1.4142135623730951;
}

static void sincos2pi(real u, real* sn, real* cs) {
  real x = u * (real)4;
  int k = (int)x;
  real f = x - (real)k;
  if (f > (real)0.5) {
    f = f - (real)1;
    k = k + 1;
  }
  real z = f * f;
  real ps = SINC[NSIN - 1];
  for (int j = NSIN - 2; j >= 0; j--) ps = ps * z + SINC[j];
  real s = f * ps;
  real pc = COSC[NCOS - 1];
  for (int j = NCOS - 2; j >= 0; j--) pc = pc * z + COSC[j];
  switch (k & 3) {
    case 0: *sn = s; *cs = pc; break;
    case 1: *sn = pc; *cs = -s; break;
    case 2: *sn = -s; *cs = -pc; break;
    default: *sn = -pc; *cs = s; break;
  }
}

static real plog(real u) {
  int e;
  real m;
#ifdef ORACLE_FP64
  uint64_t b;
  memcpy(&b, &u, 8);
  e = (int)((b >> 52) & 0x7FF) - 1023;
  b = (b & 0xFFFFFFFFFFFFFull) | 0x3FF0000000000000ull;
  memcpy(&m, &b, 8);
#else
  uint32_t b;
  memcpy(&b, &u, 4);
  e = (int)((b >> 23) & 0xFF) - 127;
  b = (b & 0x7FFFFFu) | 0x3F800000u;
  memcpy(&m, &b, 4);
#endif
  if (m > SQRT2R) {
    m = m * (real)0.5;
    e = e + 1;
  }
  real s = (m - (real)1) / (m + (real)1);
  real z = s * s;
  real p = LOGC[NLOG - 1];
  for (int k = NLOG - 2; k >= 0; k--) p = p * z + LOGC[k];
  return (real)e * LN2R + (s + s) * p;
}

static real bm_radius(real u) { return RSQRT((real)-2 * plog(u)); }
static real cos2pi(real u) {
  real s, c;
  sincos2pi(u, &s, &c);
  return c;
}
static real sin2pi(real u) {
  real s, c;
  sincos2pi(u, &s, &c);
  return s;
}

void or_math(const double* u, int64_t n, double* sn, double* cs, double* lg) {
  init_series();
  for (int64_t i = 0; i < n; i++) {
    real s, c;
    sincos2pi((real)u[i], &s, &c);
    sn[i] = (double)s;
    cs[i] = (double)c;
    lg[i] = (double)plog((real)u[i]);
  }
}

/* isotropic unit vector: cos(theta) = 1 - 2u, phi = 2 pi u' */
static void iso_dir(uint32_t wc, uint32_t wp, real n[3]) {
  real u = unif(wc);
  real ct = (real)1 - (real)2 * u;
  real st = RSQRT((real)1 - ct * ct);
  real up = unif(wp);
  n[0] = st * cos2pi(up);
  n[1] = st * sin2pi(up);
  n[2] = ct;
}

/* ----------------------------------------------------------------------- */
/* context                                                                  */
/* ----------------------------------------------------------------------- */
typedef struct {
  int32_t cell, sort_cell, alive;
  real off, v[3];
  uint64_t id;
} part;

typedef struct {
  part* a;
  int64_t n, cap;
} store;

typedef struct {
  int sp;
  int64_t idx;
  uint64_t id;
  int chan;
  int32_t cell;
  real u_acc;
  int64_t partner; /* index in the partner store, -1 none */
  int accepted;
} request;

typedef struct {
  int sp;
  uint64_t creator;
  int k;
  int32_t cell;
  real off, v[3];
} birth;

struct or_ctx {
  or_params P;
  int N;                 /* cells */
  double dx, dt, ngas;
  double tau[3], mass[3], charge[3];
  double MO2;
  /* working-precision constants */
  real qmdt[3], dtdx[3], hk[3], vth0[3], vthg;
  real a_g[3], b_g[3], hmu_g[3], c2e_g[3];      /* species + O2 gas */
  real a_c[NCH], b_c[NCH], hmu_c[NCH], c2e_c[NCH]; /* partner channels */
  real ddf, adf, hme, hmn;
  real sig[NCH][NPT];
  real thr[NCH], loss[NCH];
  double M_gas[3], M_ad, M_ch[NCH];
  real Mr_ch[NCH];
  double PG[NCH];        /* tau * n_target for gas channels */
  double PGtot[3];
  double KP[NCH];        /* tau * M_j * W / (A dx) for partner channels */
  /* per-cell collision list (dsmc): tau = sort_every dt for every type */
  double PGl[NCH];       /* tau * n_target for gas channels */
  double Bl[16];         /* bound of Eq. (1) for gas type (4 + t): PGl * max sigma g */
  double KPl;            /* tau * W / (A dx): Eq. (1) per partner particle of the cell and unit sigma g */
  double KMl[NCH];       /* KPl * M_j for partner channels */
  double cphi, cE;
  real cc_coul[3], cc_coul_half[3]; /* Eq. (2) prefactor per particle in the cell */
  real cc_inter[3];                  /* the same for the pairs (e, O-), (e, O2+), (O-, O2+) */
  real fr_inter[3][2];               /* mu / m of the pair's first and second species */
  double* Udrive;        /* [M] */
  /* state */
  store st[3];
  int64_t step;
  uint64_t next_id;
  int32_t* seglen[3];
  int32_t segmax[3];
  double* phi;
  double* E;
  real* Er;
  int64_t* Q;            /* [3][N+1] */
  /* counters */
  int64_t events[NCH], absorbed[2][3], psteps, births, cycles, tophits, nreq, nacc;
  int nanflag;
  /* diagnostics */
  int64_t *Qacc, *Qlast, *eedf_acc, *eedf_last, *fneg_acc, *fneg_last;
  double *phiacc, *philast;
  /* per-step scratch */
  request* req;
  int64_t nreq_step, capreq;
  birth* bir;
  int64_t nbir, capbir;
  /* event log */
  double* log;
  int64_t nlog, caplog;
};

static const int partner_of[NCH] = {-1, -1, -1, -1, -1, -1, -1, -1, -1, -1,
                                    -1, -1, SP_P, SP_N, -1, -1, -1, SP_P, -1};

/* channels of each species, in the order of the collision decision */
static const int part_ch[3][2] = {{12, 13}, {17, -1}, {-1, -1}};
static const int n_part_ch[3] = {2, 1, 0};
static const int gas_ch_e[] = {0, 1, 2, 3, 4, 5, 6, 7, 8, 9, 10, 11};
static const int gas_ch_n[] = {14, 15, 16};
static const int gas_ch_p[] = {18};

/* the collision list of Table I in order, type (4 + t) of the per-cell scheme */
typedef struct {
  int sp, n, ch[4];  /* test species, gas channels (n = 0: partner type with channel ch[0]) */
} ltype;

static const ltype LIST[16] = {
    {SP_E, 1, {0}},  {SP_N, 1, {14}}, {SP_P, 1, {18}}, {SP_E, 4, {1, 2, 3, 4}}, {SP_E, 1, {5}},
    {SP_E, 1, {6}},  {SP_E, 1, {7}},  {SP_E, 1, {8}},  {SP_E, 1, {9}},          {SP_E, 0, {12}},
    {SP_N, 0, {17}}, {SP_E, 1, {10}}, {SP_N, 1, {15}}, {SP_N, 1, {16}},         {SP_E, 1, {11}},
    {SP_E, 0, {13}}};

/* random streams of type (4 + t): decision, gas molecule, scattering angles */
#define LK_DEC(t) (32u + 3u * (uint32_t)(t))
#define LK_GAS(t) (33u + 3u * (uint32_t)(t))
#define LK_ANG(t) (34u + 3u * (uint32_t)(t))

static void gas_channels(int s, const int** list, int* n) {
  if (s == SP_E) { *list = gas_ch_e; *n = 12; }
  else if (s == SP_N) { *list = gas_ch_n; *n = 3; }
  else { *list = gas_ch_p; *n = 1; }
}

static int st_grow(store* s, int64_t need) {
  if (need <= s->cap) return 0;
  int64_t nc = s->cap ? s->cap : 1024;
  while (nc < need) nc *= 2;
  part* a = (part*)realloc(s->a, (size_t)nc * sizeof(part));
  if (!a) return -1;
  s->a = a;
  s->cap = nc;
  return 0;
}

/* ----------------------------------------------------------------------- */
/* cross-section tables                                                     */
/* ----------------------------------------------------------------------- */
static double grid_E(int k) { return ldexp(1.0 + (double)(k % 32) / 32.0, -14 + k / 32); }

/* linear interpolation on the binade grid; index and weight from the bits */
static real sigma_at(const or_ctx* c, int j, real E) {
  const real* s = c->sig[j];
#ifdef ORACLE_FP64
  uint64_t b;
  memcpy(&b, &E, 8);
  if (b < 0x3F10000000000000ull) return s[0];
  if (b >= 0x40D0000000000000ull) return s[NPT - 1];
  int k = (int)((b >> 47) - (0x3F10000000000000ull >> 47));
  double t = (double)(b & ((1ull << 47) - 1)) * 0x1p-47;
#else
  uint32_t b;
  memcpy(&b, &E, 4);
  if (b < 0x38800000u) return s[0];
  if (b >= 0x46800000u) return s[NPT - 1];
  int k = (int)((b >> 18) - (0x38800000u >> 18));
  float t = (float)(b & 0x3FFFFu) * 0x1p-18f;
#endif
  real d = s[k + 1] - s[k];
  real p = t * d;
  return s[k] + p;
}

double or_sigma(const or_ctx* c, int chan, double E) { return (double)sigma_at(c, chan, (real)E); }

/* upper bound of sum_j sigma_j(E) g(E) over the tabulated range for the
   channel list, with g(E) = sqrt(E * 2e/mu): on each segment the bound is
   the larger end value times g at the upper end; below the first node sigma
   is constant and g < g(E_0). */
static double bound_M(const double* sig /*[NCH][NPT]*/, const int* chans, int nch, double mu) {
  double c2 = (2.0 * QE) / mu;
  double M = 0.0;
  {
    double s = 0.0;
    for (int q = 0; q < nch; q++) s = s + sig[chans[q] * NPT + 0];
    double v = s * sqrt(grid_E(0) * c2);
    if (v > M) M = v;
  }
  for (int k = 0; k < NPT - 1; k++) {
    double s = 0.0;
    for (int q = 0; q < nch; q++) {
      double a = sig[chans[q] * NPT + k], b = sig[chans[q] * NPT + k + 1];
      s = s + (a > b ? a : b);
    }
    double v = s * sqrt(grid_E(k + 1) * c2);
    if (v > M) M = v;
  }
  return M * (1.0 + 1.0 / 65536.0);
}

/* ----------------------------------------------------------------------- */
/* field: exact Green's function of the Dirichlet problem                   */
/* -(phi_{i-1} - 2 phi_i + phi_{i+1}) = cphi * q_i, phi_0 = U0, phi_N = 0   */
/* phi_i = U0 (N-i)/N + cphi * sum_j G_ij q_j,  G_ij = min(i,j)(N-max(i,j))/N */
/* ----------------------------------------------------------------------- */
void or_solve_field(int32_t N, double dx, double cphi, double cE, double U0, const int64_t* q,
                    double* phi, double* E) {
  __int128* S1 = (__int128*)calloc((size_t)N + 1, sizeof(__int128));
  __int128* S2 = (__int128*)calloc((size_t)N + 1, sizeof(__int128));
  /* S1_i = sum_{j=1..i} j q_j ;  S2_i = sum_{j=i+1..N-1} (N-j) q_j */
  for (int i = 1; i <= N; i++) S1[i] = S1[i - 1] + (i < N ? (__int128)i * q[i] : 0);
  S2[N] = 0;
  for (int i = N - 1; i >= 0; i--) S2[i] = S2[i + 1] + (i + 1 <= N - 1 ? (__int128)(N - (i + 1)) * q[i + 1] : 0);
  phi[0] = U0;
  phi[N] = 0.0;
  for (int i = 1; i < N; i++) {
    __int128 T = (__int128)(N - i) * S1[i] + (__int128)i * S2[i];
    double a = U0 * (double)(N - i);
    double b = cphi * (double)T;
    phi[i] = (a + b) / (double)N;
  }
  double invdx = 1.0 / dx, inv2dx = 0.5 / dx;
  for (int i = 1; i < N; i++) E[i] = (phi[i - 1] - phi[i + 1]) * inv2dx;
  E[0] = (phi[0] - phi[1]) * invdx - cE * (double)q[0];
  E[N] = (phi[N - 1] - phi[N]) * invdx + cE * (double)q[N];
  free(S1);
  free(S2);
}

/* ----------------------------------------------------------------------- */
/* creation                                                                 */
/* ----------------------------------------------------------------------- */
static void deposit_all(or_ctx* c) {
  int N = c->N;
  memset(c->Q, 0, sizeof(int64_t) * 3 * (size_t)(N + 1));
  for (int s = 0; s < 3; s++) {
    int64_t* Q = c->Q + (size_t)s * (N + 1);
    for (int64_t i = 0; i < c->st[s].n; i++) {
      part* p = &c->st[s].a[i];
      if (!p->alive) continue;
      int64_t f = (int64_t)(p->off * (real)16777216.0);
      Q[p->cell] += ONE_FIX - f;
      Q[p->cell + 1] += f;
    }
  }
}

static void solve(or_ctx* c, double U) {
  int N = c->N;
  int64_t* q = (int64_t*)calloc((size_t)N + 1, sizeof(int64_t));
  for (int i = 0; i <= N; i++) q[i] = c->Q[2 * (N + 1) + i] - c->Q[i] - c->Q[(N + 1) + i];
  or_solve_field(N, c->dx, c->cphi, c->cE, U, q, c->phi, c->E);
  for (int i = 0; i <= N; i++) c->Er[i] = (real)c->E[i];
  free(q);
}

static real gather(const or_ctx* c, int cell, real off) {
  real E0 = c->Er[cell], E1 = c->Er[cell + 1];
  real d = E1 - E0;
  real t = off * d;
  return E0 + t;
}

static void do_sort(or_ctx* c) {
  /* at a sort step dead particles leave the store and every alive particle's
     current cell becomes its partner cell until the next sort */
  for (int s = 0; s < 3; s++) {
    store* S = &c->st[s];
    int64_t w = 0;
    for (int64_t i = 0; i < S->n; i++)
      if (S->a[i].alive) S->a[w++] = S->a[i];
    S->n = w;
    memset(c->seglen[s], 0, sizeof(int32_t) * (size_t)c->N);
    for (int64_t i = 0; i < S->n; i++) {
      S->a[i].sort_cell = S->a[i].cell;
      c->seglen[s][S->a[i].cell]++;
    }
    int32_t mx = 0;
    for (int i = 0; i < c->N; i++) mx = c->seglen[s][i] > mx ? c->seglen[s][i] : mx;
    c->segmax[s] = mx;
  }
}

static double pmax_of(const or_ctx* c, int s) {
  double P = c->PGtot[s];
  for (int q = 0; q < n_part_ch[s]; q++) {
    int j = part_ch[s][q];
    P = P + (double)c->segmax[partner_of[j]] * c->KP[j];
  }
  return P;
}

or_ctx* or_create(const or_params* p, const double* sigma, const double* thr, const double* loss, int* err) {
  init_series();
  *err = OR_OK;
  if (p->n_cells < 4 || p->gap_m <= 0 || p->area_m2 <= 0 || p->weight <= 0 || p->steps_per_period < 1 ||
      p->ion_subcycle < 1 || p->sort_every < 1 || p->frequency_Hz <= 0 || p->coulomb_every < 0 ||
      (p->coulomb_every > 0 && (p->coulomb_every % p->sort_every != 0 || !(p->coulomb_log > 0))) ||
      p->dsmc < 0 || p->dsmc > 1 || (p->dsmc && p->sort_every % p->ion_subcycle != 0)) {
    *err = OR_EINVAL;
    return NULL;
  }
  or_ctx* c = (or_ctx*)calloc(1, sizeof(or_ctx));
  c->P = *p;
  int N = c->N = p->n_cells;
  c->dx = p->gap_m / (double)N;
  c->dt = 1.0 / (p->frequency_Hz * (double)p->steps_per_period);
  c->ngas = p->pressure_Pa / (KB * p->T_gas_K);
  c->MO2 = 31.998 * AMU;
  c->mass[SP_E] = ME;
  c->mass[SP_N] = 15.999 * AMU + ME;
  c->mass[SP_P] = c->MO2 - ME;
  c->charge[SP_E] = -QE;
  c->charge[SP_N] = -QE;
  c->charge[SP_P] = QE;
  c->tau[SP_E] = c->dt;
  c->tau[SP_N] = c->dt * (double)p->ion_subcycle;
  c->tau[SP_P] = c->dt * (double)p->ion_subcycle;
  for (int s = 0; s < 3; s++) {
    double qm = c->charge[s] / c->mass[s];
    c->qmdt[s] = (real)(qm * c->tau[s]);
    c->dtdx[s] = (real)(c->tau[s] / c->dx);
    c->hk[s] = (real)(qm * (0.5 * c->tau[s]));
    c->vth0[s] = (real)sqrt((p->T_init_eV[s] * QE) / c->mass[s]);
    double mu = (c->mass[s] * c->MO2) / (c->mass[s] + c->MO2);
    c->a_g[s] = (real)(c->MO2 / (c->mass[s] + c->MO2));
    c->b_g[s] = (real)(c->mass[s] / (c->mass[s] + c->MO2));
    c->hmu_g[s] = (real)((0.5 * mu) / QE);
    c->c2e_g[s] = (real)((2.0 * QE) / mu);
  }
  c->vthg = (real)sqrt((KB * p->T_gas_K) / c->MO2);
  for (int j = 0; j < NCH; j++) {
    int t = partner_of[j];
    if (t < 0) continue;
    int s = (j == 17) ? SP_N : SP_E;
    double ms = c->mass[s], mt = c->mass[t];
    double mu = (ms * mt) / (ms + mt);
    c->a_c[j] = (real)(mt / (ms + mt));
    c->b_c[j] = (real)(ms / (ms + mt));
    c->hmu_c[j] = (real)((0.5 * mu) / QE);
    c->c2e_c[j] = (real)((2.0 * QE) / mu);
  }
  {
    double mu_n = (c->mass[SP_N] * c->MO2) / (c->mass[SP_N] + c->MO2);
    c->ddf = (real)sqrt((0.1 * c->mass[SP_N]) / ME);
    c->adf = (real)sqrt(mu_n / ME);
    c->hme = (real)((0.5 * ME) / QE);
    c->hmn = (real)((0.5 * c->mass[SP_N]) / QE);
  }
  for (int j = 0; j < NCH; j++) {
    for (int k = 0; k < NPT; k++) c->sig[j][k] = (real)sigma[j * NPT + k];
    c->thr[j] = (real)thr[j];
    c->loss[j] = (real)loss[j];
  }
  /* null-collision bounds */
  {
    static const int ge[] = {0, 1, 2, 3, 4, 5, 6, 7, 8, 9, 10, 11};
    static const int gn[] = {14, 15};
    static const int gp[] = {18};
    static const int gad[] = {16};
    double mu[3];
    for (int s = 0; s < 3; s++) mu[s] = (c->mass[s] * c->MO2) / (c->mass[s] + c->MO2);
    c->M_gas[SP_E] = bound_M(sigma, ge, 12, mu[SP_E]);
    c->M_gas[SP_N] = bound_M(sigma, gn, 2, mu[SP_N]);
    c->M_gas[SP_P] = bound_M(sigma, gp, 1, mu[SP_P]);
    c->M_ad = bound_M(sigma, gad, 1, mu[SP_N]);
    for (int j = 0; j < NCH; j++) {
      int t = partner_of[j];
      if (t < 0) continue;
      int s = (j == 17) ? SP_N : SP_E;
      double mum = (c->mass[s] * c->mass[t]) / (c->mass[s] + c->mass[t]);
      int one[1] = {j};
      c->M_ch[j] = bound_M(sigma, one, 1, mum);
      c->Mr_ch[j] = (real)c->M_ch[j];
      c->KP[j] = ((c->tau[s] * c->M_ch[j]) * p->weight) / (p->area_m2 * c->dx);
    }
    for (int j = 0; j < NCH; j++) {
      if (partner_of[j] >= 0) continue;
      int s = j <= 11 ? SP_E : (j <= 16 ? SP_N : SP_P);
      c->PG[j] = (j == 16) ? (c->tau[s] * p->metastable_frac) * c->ngas : c->tau[s] * c->ngas;
    }
    c->PGtot[SP_E] = c->PG[0] * c->M_gas[SP_E];
    c->PGtot[SP_N] = c->PG[14] * c->M_gas[SP_N] + c->PG[16] * c->M_ad;
    c->PGtot[SP_P] = c->PG[18] * c->M_gas[SP_P];
    if (p->dsmc) {
      double tl = c->dt * (double)p->sort_every;
      for (int j = 0; j < NCH; j++) {
        if (partner_of[j] >= 0) continue;
        c->PGl[j] = (j == 16) ? (tl * p->metastable_frac) * c->ngas : tl * c->ngas;
      }
      c->KPl = (tl * p->weight) / (p->area_m2 * c->dx);
      for (int j = 0; j < NCH; j++)
        if (partner_of[j] >= 0) c->KMl[j] = c->KPl * c->M_ch[j];
      for (int t = 0; t < 16; t++) {
        if (LIST[t].n == 0) continue;
        c->Bl[t] = c->PGl[LIST[t].ch[0]] * bound_M(sigma, LIST[t].ch, LIST[t].n, mu[LIST[t].sp]);
        if (c->Bl[t] > 1.0) { *err = OR_EINVAL; or_destroy(c); return NULL; }
      }
    }
  }
  /* Eq. (2) with eps0^2 (Takizuka-Abe): <tan^2(chi/2)> = q^4 n lnL t_c2 / (8 pi eps0^2 mu^2 u^3),
     mu = m/2, n = W N_cell / (A dx), t_c2 = coulomb_every dt */
  for (int s = 0; s < 3; s++) {
    double mu = 0.5 * c->mass[s];
    double tc2 = c->dt * (double)(p->coulomb_every > 0 ? p->coulomb_every : 1);
    double num = ((((QE * QE) * (QE * QE)) * p->coulomb_log) * tc2) * p->weight;
    double den = (((8.0 * PI) * (EPS0 * EPS0)) * (mu * mu)) * (p->area_m2 * c->dx);
    c->cc_coul[s] = (real)(num / den);
    c->cc_coul_half[s] = (real)((0.5 * num) / den);
  }
  /* unlike species a, b (all singly charged): the reduced mass of the pair and
     the lower of the two densities (W N_min / (A dx)) */
  {
    static const int pa[3] = {0, 0, 1}, pb[3] = {1, 2, 2};
    for (int q = 0; q < 3; q++) {
      double ma = c->mass[pa[q]], mb = c->mass[pb[q]];
      double mu = (ma * mb) / (ma + mb);
      double tc2 = c->dt * (double)(p->coulomb_every > 0 ? p->coulomb_every : 1);
      double num = ((((QE * QE) * (QE * QE)) * p->coulomb_log) * tc2) * p->weight;
      double den = (((8.0 * PI) * (EPS0 * EPS0)) * (mu * mu)) * (p->area_m2 * c->dx);
      c->cc_inter[q] = (real)(num / den);
      c->fr_inter[q][0] = (real)(mu / ma);
      c->fr_inter[q][1] = (real)(mu / mb);
    }
  }
  c->cphi = ((c->dx * QE) * p->weight) / ((EPS0 * 16777216.0) * p->area_m2);
  c->cE = (QE * p->weight) / ((EPS0 * 16777216.0) * p->area_m2);
  if (p->field_off) c->cphi = c->cE = 0.0; /* test switch: the charge does not enter the field */
  int M = p->steps_per_period;
  c->Udrive = (double*)malloc(sizeof(double) * (size_t)M);
  for (int k = 0; k < M; k++) {
    if (p->drive_dc) c->Udrive[k] = p->voltage_V;
    else c->Udrive[k] = p->voltage_V * sin((TWO_PI * (double)k) / (double)M);
  }
  c->phi = (double*)calloc((size_t)N + 1, sizeof(double));
  c->E = (double*)calloc((size_t)N + 1, sizeof(double));
  c->Er = (real*)calloc((size_t)N + 1, sizeof(real));
  c->Q = (int64_t*)calloc(3 * ((size_t)N + 1), sizeof(int64_t));
  c->Qacc = (int64_t*)calloc(3 * ((size_t)N + 1), sizeof(int64_t));
  c->Qlast = (int64_t*)calloc(3 * ((size_t)N + 1), sizeof(int64_t));
  c->phiacc = (double*)calloc((size_t)N + 1, sizeof(double));
  c->philast = (double*)calloc((size_t)N + 1, sizeof(double));
  int nb = p->eedf_bins > 0 ? p->eedf_bins : 1;
  c->eedf_acc = (int64_t*)calloc((size_t)nb + 1, sizeof(int64_t));
  c->eedf_last = (int64_t*)calloc((size_t)nb + 1, sizeof(int64_t));
  int nf = (p->fneg_xbins > 0 ? p->fneg_xbins : 1) * (p->fneg_ebins > 0 ? p->fneg_ebins : 1);
  c->fneg_acc = (int64_t*)calloc((size_t)nf, sizeof(int64_t));
  c->fneg_last = (int64_t*)calloc((size_t)nf, sizeof(int64_t));
  for (int s = 0; s < 3; s++) c->seglen[s] = (int32_t*)calloc((size_t)N, sizeof(int32_t));

  /* initial load (Sec. II): uniform in x, Maxwellian in v; ids e, O-, O2+ */
  uint64_t id = 0;
  for (int s = 0; s < 3; s++) {
    if (st_grow(&c->st[s], p->n_init[s] + 16)) { *err = OR_ENOMEM; or_destroy(c); return NULL; }
    for (int64_t i = 0; i < p->n_init[s]; i++, id++) {
      uint32_t w[4], u[4];
      rng(p->seed, id, 0xFFFFFFFFu, 0, w);
      rng(p->seed, id, 0xFFFFFFFFu, 1, u);
      part q;
      q.id = id;
      q.alive = 1;
      q.cell = (int32_t)(((uint64_t)w[0] * (uint64_t)N) >> 32);
      q.sort_cell = q.cell;
      q.off = unif(w[1]);
      real r1 = bm_radius(unif(u[0])), a1 = unif(u[1]);
      real r2 = bm_radius(unif(u[2])), a2 = unif(u[3]);
      q.v[0] = c->vth0[s] * (r1 * cos2pi(a1));
      q.v[1] = c->vth0[s] * (r1 * sin2pi(a1));
      q.v[2] = c->vth0[s] * (r2 * cos2pi(a2));
      c->st[s].a[c->st[s].n++] = q;
    }
  }
  c->next_id = id;
  /* field at t = 0 and the half step back of the leapfrog velocities */
  deposit_all(c);
  solve(c, c->Udrive[0]);
  for (int s = 0; s < 3; s++)
    for (int64_t i = 0; i < c->st[s].n; i++) {
      part* q = &c->st[s].a[i];
      real Ep = gather(c, q->cell, q->off);
      real dv = c->hk[s] * Ep;
      q->v[0] = q->v[0] - dv;
    }
  do_sort(c);
  c->step = 0;
  return c;
}

/* test hook: replace the initial load by the given particles (species in the
   order e, O-, O2+, n[s] each; ids 0.. in that order) and take the creation
   steps again: deposit, field at t = 0, half step back, sort.  Only before the
   first step. */
int or_load(or_ctx* c, const int64_t n[3], const int32_t* cell, const double* off, const double* v) {
  if (c->step != 0) return OR_EINVAL;
  uint64_t id = 0;
  int64_t k = 0;
  for (int s = 0; s < 3; s++) {
    c->st[s].n = 0;
    if (st_grow(&c->st[s], n[s] + 16)) return OR_ENOMEM;
    for (int64_t i = 0; i < n[s]; i++, id++, k++) {
      if (cell[k] < 0 || cell[k] >= c->N || !(off[k] >= 0.0) || !(off[k] < 1.0)) return OR_EINVAL;
      part q;
      q.id = id;
      q.alive = 1;
      q.cell = cell[k];
      q.sort_cell = q.cell;
      q.off = (real)off[k];
      for (int d = 0; d < 3; d++) q.v[d] = (real)v[3 * k + d];
      c->st[s].a[c->st[s].n++] = q;
    }
  }
  c->next_id = id;
  deposit_all(c);
  solve(c, c->Udrive[0]);
  for (int s = 0; s < 3; s++)
    for (int64_t i = 0; i < c->st[s].n; i++) {
      part* q = &c->st[s].a[i];
      real Ep = gather(c, q->cell, q->off);
      real dv = c->hk[s] * Ep;
      q->v[0] = q->v[0] - dv;
    }
  do_sort(c);
  return OR_OK;
}

void or_destroy(or_ctx* c) {
  if (!c) return;
  for (int s = 0; s < 3; s++) { free(c->st[s].a); free(c->seglen[s]); }
  free(c->Udrive); free(c->phi); free(c->E); free(c->Er); free(c->Q);
  free(c->Qacc); free(c->Qlast); free(c->phiacc); free(c->philast);
  free(c->eedf_acc); free(c->eedf_last); free(c->fneg_acc); free(c->fneg_last);
  free(c->req); free(c->bir); free(c->log);
  free(c);
}

/* ----------------------------------------------------------------------- */
/* step helpers                                                             */
/* ----------------------------------------------------------------------- */
static void add_birth(or_ctx* c, int sp, uint64_t creator, int k, int32_t cell, real off, const real v[3]) {
  if (c->nbir == c->capbir) {
    c->capbir = c->capbir ? 2 * c->capbir : 1024;
    c->bir = (birth*)realloc(c->bir, sizeof(birth) * (size_t)c->capbir);
  }
  birth* b = &c->bir[c->nbir++];
  b->sp = sp; b->creator = creator; b->k = k; b->cell = cell; b->off = off;
  b->v[0] = v[0]; b->v[1] = v[1]; b->v[2] = v[2];
}

static void add_request(or_ctx* c, int sp, int64_t idx, const part* p, int chan, real u_acc) {
  if (c->nreq_step == c->capreq) {
    c->capreq = c->capreq ? 2 * c->capreq : 256;
    c->req = (request*)realloc(c->req, sizeof(request) * (size_t)c->capreq);
  }
  request* r = &c->req[c->nreq_step++];
  r->sp = sp; r->idx = idx; r->id = p->id; r->chan = chan; r->cell = p->cell; r->u_acc = u_acc;
  r->partner = -1; r->accepted = 0;
}

static double ke(double m, const real v[3]) {
  return 0.5 * m * ((double)v[0] * v[0] + (double)v[1] * v[1] + (double)v[2] * v[2]);
}

/* event log entry (16 doubles): chan, species, kinetic energy before/after, momentum
   before[3]/after[3], loss, aux0, aux1.  Coulomb collisions log chan = 100 and
   per unit mass: e[2..9] as above, e[11] the Eq. (2) variance, e[12] the realised
   tan^2(chi/2), e[13] u, e[14] the cell's particle count, e[15] 1 in a triangle */
static void log_event(or_ctx* c, int chan, int sp, double keb, double kea, const double pb[3],
                      const double pa[3], double aux0, double aux1) {
  if (!c->log || c->nlog >= c->caplog) return;
  double* e = c->log + 16 * c->nlog++;
  memset(e, 0, 16 * sizeof(double));
  e[0] = chan; e[1] = sp; e[2] = keb; e[3] = kea;
  for (int d = 0; d < 3; d++) { e[4 + d] = pb[d]; e[7 + d] = pa[d]; }
  e[10] = c->loss[chan]; e[11] = aux0; e[12] = aux1;
}

/* equal-mass isotropic elastic collision of two electrons */
static void ee_elastic(real va[3], real vb[3], const real n[3]) {
  real V[3], g[3];
  for (int d = 0; d < 3; d++) { V[d] = (va[d] + vb[d]) * (real)0.5; g[d] = va[d] - vb[d]; }
  real g2 = (g[0] * g[0] + g[1] * g[1]) + g[2] * g[2];
  real h = (real)0.5 * RSQRT(g2);
  for (int d = 0; d < 3; d++) { va[d] = V[d] + h * n[d]; vb[d] = V[d] - h * n[d]; }
}

/* collision with a gas molecule drawn from the Maxwellian (Sec. III A/B/C) */
static void gas_event(or_ctx* c, int s, int j, part* p, const real vt[3], real g, real Erel, uint32_t n,
                      uint32_t kr) {
  uint32_t w[4];
  rng(c->P.seed, p->id, n, kr, w);
  real n1[3], n2[3];
  iso_dir(w[0], w[1], n1);
  iso_dir(w[2], w[3], n2);
  real a = c->a_g[s], b = c->b_g[s];
  real vc[3];
  for (int d = 0; d < 3; d++) vc[d] = b * p->v[d] + a * vt[d];
  double m = c->mass[s], M = c->MO2;
  double pb[3], pa[3], keb = ke(m, p->v) + ke(M, vt), kea = 0;
  for (int d = 0; d < 3; d++) pb[d] = m * (double)p->v[d] + M * (double)vt[d];
  c->events[j]++;
  if (j == 10) { /* (15) dissociative attachment: the electron becomes O- at v_cm */
    p->alive = 0;
    add_birth(c, SP_N, p->id, 0, p->cell, p->off, vc);
    log_event(c, j, s, keb, 0, pb, pb, 0, 0);
    return;
  }
  if (j == 15 || j == 16) { /* (16) direct / (17) associative detachment */
    real f = (j == 15) ? c->ddf : c->adf;
    real sp = f * g;
    real ve[3];
    for (int d = 0; d < 3; d++) ve[d] = vc[d] + sp * n1[d];
    p->alive = 0;
    add_birth(c, SP_E, p->id, 0, p->cell, p->off, ve);
    double ee = 0.5 * ME * ((double)sp * sp);
    double prim = (j == 15) ? 0.5 * m * ((double)g * g) : (double)Erel * QE;
    log_event(c, j, s, keb, 0, pb, pb, ee, prim);
    return;
  }
  real gp = g;
  if (c->loss[j] > (real)0 || j == 11) {
    real Ep = Erel - c->loss[j];
    gp = RSQRT(Ep * c->c2e_g[s]);
  }
  real ag = a * gp, bg = b * gp;
  if (j == 11) { /* (18) impact ionisation: inelastic, split O2 -> e + O2+, e-e elastic */
    real ve[3], vo[3], vn[3];
    for (int d = 0; d < 3; d++) { ve[d] = vc[d] + ag * n1[d]; vo[d] = vc[d] - bg * n1[d]; vn[d] = vo[d]; }
    ee_elastic(ve, vn, n2);
    for (int d = 0; d < 3; d++) p->v[d] = ve[d];
    add_birth(c, SP_E, p->id, 0, p->cell, p->off, vn);
    add_birth(c, SP_P, p->id, 1, p->cell, p->off, vo);
    kea = ke(ME, ve) + ke(ME, vn) + ke(c->mass[SP_P], vo);
    for (int d = 0; d < 3; d++) pa[d] = ME * (double)ve[d] + ME * (double)vn[d] + c->mass[SP_P] * (double)vo[d];
    log_event(c, j, s, keb, kea, pb, pa, 0, 0);
    return;
  }
  /* elastic (4),(5),(6) and excitation (7)-(12) */
  real vtp[3];
  for (int d = 0; d < 3; d++) { p->v[d] = vc[d] + ag * n1[d]; vtp[d] = vc[d] - bg * n1[d]; }
  kea = ke(m, p->v) + ke(M, vtp);
  for (int d = 0; d < 3; d++) pa[d] = m * (double)p->v[d] + M * (double)vtp[d];
  log_event(c, j, s, keb, kea, pb, pa, 0, 0);
}

/* candidate test and channel decision for one pushed particle (Eq. (1)) */
static void mcc(or_ctx* c, int s, int64_t idx, part* p, uint32_t n, double pmax) {
  uint32_t w[4];
  rng(c->P.seed, p->id, n, 0, w);
  double U = unif52(w[0], w[1]);
  if (!(U < pmax)) return;
  double cum = 0.0;
  for (int q = 0; q < n_part_ch[s]; q++) {
    int j = part_ch[s][q];
    double L = (double)c->seglen[partner_of[j]][p->cell];
    cum = cum + L * c->KP[j];
    if (U < cum) { add_request(c, s, idx, p, j, unif(w[2])); return; }
  }
  uint32_t u[4];
  rng(c->P.seed, p->id, n, 1, u);
  real r1 = bm_radius(unif(u[0])), a1 = unif(u[1]);
  real r2 = bm_radius(unif(u[2])), a2 = unif(u[3]);
  real vt[3];
  vt[0] = c->vthg * (r1 * cos2pi(a1));
  vt[1] = c->vthg * (r1 * sin2pi(a1));
  vt[2] = c->vthg * (r2 * cos2pi(a2));
  real gx = p->v[0] - vt[0], gy = p->v[1] - vt[1], gz = p->v[2] - vt[2];
  real g2 = (gx * gx + gy * gy) + gz * gz;
  real g = RSQRT(g2);
  real Erel = c->hmu_g[s] * g2;
  if (Erel >= (real)16384) c->tophits++;
  const int* list;
  int nl;
  gas_channels(s, &list, &nl);
  for (int q = 0; q < nl; q++) {
    int j = list[q];
    real sg = 0;
    if (Erel >= c->thr[j]) sg = sigma_at(c, j, Erel) * g;
    cum = cum + c->PG[j] * (double)sg;
    if (U < cum) { gas_event(c, s, j, p, vt, g, Erel, n, 2); return; }
  }
}

static void push_species(or_ctx* c, int s, uint32_t n) {
  double pmax = pmax_of(c, s);
  store* S = &c->st[s];
  int N = c->N;
  int cmid = N / 2;
  for (int64_t i = 0; i < S->n; i++) {
    part* p = &S->a[i];
    if (!p->alive) continue;
    c->psteps++;
    real Ep = gather(c, p->cell, p->off);
    real dv = c->qmdt[s] * Ep;
    p->v[0] = p->v[0] + dv;
    real dxp = p->v[0] * c->dtdx[s];
    real off = p->off + dxp;
    real fl = RFLOOR(off);
    if (!(fl == fl) || fl > (real)1e9 || fl < (real)-1e9) { p->alive = 0; c->nanflag = 1; continue; }
    int32_t cell = p->cell + (int32_t)fl;
    off = off - fl;
    if (off >= (real)1) { off = 0; cell += 1; }
    p->off = off;
    p->cell = cell;
    if (cell < 0) { c->absorbed[0][s]++; p->alive = 0; continue; }
    if (cell >= N) { c->absorbed[1][s]++; p->alive = 0; continue; }
    if (!c->P.dsmc) {
      mcc(c, s, i, p, n, pmax);
      if (!p->alive) continue;
    }
    if (s == SP_E && cell == cmid && c->P.eedf_bins > 0) {
      real e2 = (p->v[0] * p->v[0] + p->v[1] * p->v[1]) + p->v[2] * p->v[2];
      real Ek = c->hme * e2;
      real sc = (real)((double)c->P.eedf_bins / c->P.eedf_emax_eV);
      real bf = Ek * sc;
      int64_t bin = (bf >= (real)c->P.eedf_bins) ? c->P.eedf_bins : (int64_t)bf;
      c->eedf_acc[bin]++;
    }
    if (s == SP_N && c->P.fneg_xbins > 0 && c->P.fneg_ebins > 0) {
      real Ex = c->hmn * (p->v[0] * p->v[0]);
      if (p->v[0] < (real)0) Ex = -Ex;
      real sc = (real)((double)c->P.fneg_ebins / (2.0 * c->P.fneg_emax_eV));
      real em = (real)c->P.fneg_emax_eV;
      real bf = (Ex + em) * sc;
      int64_t eb = bf < (real)0 ? 0 : (bf >= (real)c->P.fneg_ebins ? c->P.fneg_ebins - 1 : (int64_t)bf);
      int64_t xb = ((int64_t)cell * c->P.fneg_xbins) / N;
      c->fneg_acc[xb * c->P.fneg_ebins + eb]++;
    }
  }
}

static uint64_t pick_key(uint64_t seed, uint64_t id_p, uint64_t id_t, uint32_t n) {
  uint32_t ctr[4] = {(uint32_t)id_p, (uint32_t)(id_p >> 32), (uint32_t)id_t, (uint32_t)(id_t >> 32)};
  uint32_t key[2] = {(uint32_t)seed ^ n, (uint32_t)(seed >> 32) ^ 0x5BD1E995u};
  uint32_t w[4];
  or_philox(ctr, key, w);
  return ((uint64_t)(w[0] >> 8) << 40) | (id_p & ID_MASK);
}

/* (19): inelastic e-O- collision of test electron T and partner O- P: the O-
   splits into O + e (loss dE of Eq. (5)), the two electrons scatter
   elastically; directions from stream kr of T */
static void impact_detach(or_ctx* c, part* T, part* P, uint32_t n, uint32_t kr) {
  const int j = 13;
  real a = c->a_c[j], b = c->b_c[j];
  real gx = T->v[0] - P->v[0], gy = T->v[1] - P->v[1], gz = T->v[2] - P->v[2];
  real g2 = (gx * gx + gy * gy) + gz * gz;
  real Erel = c->hmu_c[j] * g2;
  uint32_t w[4];
  rng(c->P.seed, T->id, n, kr, w);
  real n1[3], n2[3];
  iso_dir(w[0], w[1], n1);
  iso_dir(w[2], w[3], n2);
  real vc[3], ve[3], vn[3], vo[3];
  for (int d = 0; d < 3; d++) vc[d] = b * T->v[d] + a * P->v[d];
  real Ep = Erel - c->loss[j];
  real gp = RSQRT(Ep * c->c2e_c[j]);
  real ag = a * gp, bg = b * gp;
  double pb[3], pa[3];
  double keb = ke(ME, T->v) + ke(c->mass[SP_N], P->v);
  for (int d = 0; d < 3; d++) {
    pb[d] = ME * (double)T->v[d] + c->mass[SP_N] * (double)P->v[d];
    ve[d] = vc[d] + ag * n1[d];
    vo[d] = vc[d] - bg * n1[d];
    vn[d] = vo[d];
  }
  ee_elastic(ve, vn, n2);
  for (int d = 0; d < 3; d++) T->v[d] = ve[d];
  P->alive = 0;
  add_birth(c, SP_E, T->id, 0, P->cell, P->off, vn);
  double kea = ke(ME, ve) + ke(ME, vn) + ke(c->mass[SP_N] - ME, vo);
  for (int d = 0; d < 3; d++) pa[d] = ME * (double)ve[d] + ME * (double)vn[d] + (c->mass[SP_N] - ME) * (double)vo[d];
  log_event(c, j, SP_E, keb, kea, pb, pa, 0, 0);
}

/* partner reactions: pick, acceptance, claims (Sec. III C, Eq. (1)) */
static void claims(or_ctx* c, uint32_t n) {
  int64_t R = c->nreq_step;
  c->nreq += R;
  for (int64_t r = 0; r < R; r++) {
    request* q = &c->req[r];
    int t = partner_of[q->chan];
    store* S = &c->st[t];
    uint64_t best = UINT64_MAX;
    int64_t bi = -1;
    for (int64_t i = 0; i < S->n; i++) {
      if (S->a[i].sort_cell != q->cell) continue;
      uint64_t k = pick_key(c->P.seed, S->a[i].id, q->id, n);
      if (k < best) { best = k; bi = i; }
    }
    q->partner = bi;
    q->accepted = 0;
    if (bi < 0 || !S->a[bi].alive) continue;
    part* T = &c->st[q->sp].a[q->idx];
    part* P = &S->a[bi];
    int j = q->chan;
    real gx = T->v[0] - P->v[0], gy = T->v[1] - P->v[1], gz = T->v[2] - P->v[2];
    real g2 = (gx * gx + gy * gy) + gz * gz;
    real g = RSQRT(g2);
    real Erel = c->hmu_c[j] * g2;
    real sg = 0;
    if (Erel >= c->thr[j]) sg = sigma_at(c, j, Erel) * g;
    q->accepted = (q->u_acc * c->Mr_ch[j] < sg);
  }
  /* stage 1: electron test particles (13), (19); stage 2: O- test particles (14) */
  for (int stage = 1; stage <= 2; stage++) {
    for (int64_t r = 0; r < R; r++) {
      request* q = &c->req[r];
      int is_e = (q->chan == 12 || q->chan == 13);
      if (stage == 1 && !is_e) continue;
      if (stage == 2 && is_e) continue;
      if (!q->accepted) continue;
      int t = partner_of[q->chan];
      part* T = &c->st[q->sp].a[q->idx];
      part* P = &c->st[t].a[q->partner];
      if (!T->alive || !P->alive) continue;
      int win = 1;
      for (int64_t r2 = 0; r2 < R && win; r2++) {
        request* o = &c->req[r2];
        if (r2 == r || !o->accepted) continue;
        int o_e = (o->chan == 12 || o->chan == 13);
        if (o_e != is_e) continue;
        if (partner_of[o->chan] != t || o->partner != q->partner) continue;
        if (!c->st[o->sp].a[o->idx].alive) continue;
        if (o->id < q->id) win = 0;
      }
      q->accepted = win ? 2 : 0;
    }
    for (int64_t r = 0; r < R; r++) {
      request* q = &c->req[r];
      if (q->accepted != 2) continue;
      q->accepted = 1;
      int j = q->chan, t = partner_of[j];
      part* T = &c->st[q->sp].a[q->idx];
      part* P = &c->st[t].a[q->partner];
      c->nacc++;
      c->events[j]++;
      if (j == 12 || j == 17) { T->alive = 0; P->alive = 0; continue; }
      impact_detach(c, T, P, n, 2);
    }
  }
}

/* ----------------------------------------------------------------------- */
/* the per-cell collision list of Sec. II (test switch dsmc = 1): after the */
/* sort every sort_every steps, the particles of each cell go through the   */
/* collision types (4)-(19) of Table I in the table's order, type (4 + t)   */
/* with the probability of Eq. (1), P = n_j sigma_j u tau, and tau =        */
/* sort_every dt for all of them.  The products of a type are placed, with  */
/* canonical ids, before the next type starts and take part in the later    */
/* ones; the partner densities n_j of a type are those at its start.        */
/* Readings: one decision per particle and type (the four vibrational       */
/* levels of (7) form one type, the level chosen with the same uniform); a  */
/* gas molecule is drawn for each decision; a simulated partner is one      */
/* particle of the cell chosen by a hash of the two ids; when several test  */
/* particles accept the same partner, the one with the smallest id collides.*/
/* A uniform at or above the type's largest probability cannot collide, so  */
/* no target is drawn for it (the draws are counter-based: this changes no  */
/* other draw).                                                             */
/* ----------------------------------------------------------------------- */
static int commit_births(or_ctx* c);

static void list_gas_type(or_ctx* c, int t, uint32_t n) {
  const ltype* L = &LIST[t];
  int s = L->sp;
  store* S = &c->st[s];
  for (int64_t i = 0; i < S->n; i++) {
    part* p = &S->a[i];
    if (!p->alive) continue;
    uint32_t w[4];
    rng(c->P.seed, p->id, n, LK_DEC(t), w);
    double U = unif52(w[0], w[1]);
    if (!(U < c->Bl[t])) continue;
    uint32_t u[4];
    rng(c->P.seed, p->id, n, LK_GAS(t), u);
    real r1 = bm_radius(unif(u[0])), a1 = unif(u[1]);
    real r2 = bm_radius(unif(u[2])), a2 = unif(u[3]);
    real vt[3];
    vt[0] = c->vthg * (r1 * cos2pi(a1));
    vt[1] = c->vthg * (r1 * sin2pi(a1));
    vt[2] = c->vthg * (r2 * cos2pi(a2));
    real gx = p->v[0] - vt[0], gy = p->v[1] - vt[1], gz = p->v[2] - vt[2];
    real g2 = (gx * gx + gy * gy) + gz * gz;
    real g = RSQRT(g2);
    real Erel = c->hmu_g[s] * g2;
    if (Erel >= (real)16384) c->tophits++;
    double cum = 0.0;
    for (int q = 0; q < L->n; q++) {
      int j = L->ch[q];
      real sg = 0;
      if (Erel >= c->thr[j]) sg = sigma_at(c, j, Erel) * g;
      cum = cum + c->PGl[j] * (double)sg;
      if (U < cum) { gas_event(c, s, j, p, vt, g, Erel, n, LK_ANG(t)); break; }
    }
  }
}

static int list_partner_type(or_ctx* c, int t, uint32_t n) {
  int j = LIST[t].ch[0];
  int s = LIST[t].sp, tg = partner_of[j];
  store* S = &c->st[s];
  store* P = &c->st[tg];
  int64_t* cnt = (int64_t*)calloc((size_t)c->N, sizeof(int64_t));
  for (int64_t i = 0; i < P->n; i++)
    if (P->a[i].alive) cnt[P->a[i].cell]++;
  c->nreq_step = 0;
  int rc = OR_OK;
  for (int64_t i = 0; i < S->n; i++) {
    part* T = &S->a[i];
    if (!T->alive) continue;
    double Nt = (double)cnt[T->cell];
    if (Nt * c->KMl[j] > 1.0) { rc = OR_EGUARD; break; }
    uint32_t w[4];
    rng(c->P.seed, T->id, n, LK_DEC(t), w);
    double U = unif52(w[0], w[1]);
    if (!(U < Nt * c->KMl[j])) continue;
    uint64_t best = UINT64_MAX;
    int64_t bi = -1;
    for (int64_t k = 0; k < P->n; k++) {
      if (!P->a[k].alive || P->a[k].cell != T->cell) continue;
      uint64_t key = pick_key(c->P.seed, P->a[k].id, T->id, n);
      if (key < best) { best = key; bi = k; }
    }
    c->nreq++;
    part* Q = &P->a[bi];
    real gx = T->v[0] - Q->v[0], gy = T->v[1] - Q->v[1], gz = T->v[2] - Q->v[2];
    real g2 = (gx * gx + gy * gy) + gz * gz;
    real g = RSQRT(g2);
    real Erel = c->hmu_c[j] * g2;
    real sg = 0;
    if (Erel >= c->thr[j]) sg = sigma_at(c, j, Erel) * g;
    if (!(U < (Nt * c->KPl) * (double)sg)) continue;
    add_request(c, s, i, T, j, 0);
    c->req[c->nreq_step - 1].partner = bi;
  }
  free(cnt);
  if (rc) return rc;
  /* a partner accepted by several test particles collides with the smallest id */
  int64_t R = c->nreq_step;
  for (int64_t r = 0; r < R; r++) {
    request* q = &c->req[r];
    q->accepted = 1;
    for (int64_t r2 = 0; r2 < R; r2++)
      if (c->req[r2].partner == q->partner && c->req[r2].id < q->id) q->accepted = 0;
  }
  for (int64_t r = 0; r < R; r++) {
    request* q = &c->req[r];
    if (!q->accepted) continue;
    part* T = &S->a[q->idx];
    part* Q = &P->a[q->partner];
    c->nacc++;
    c->events[j]++;
    if (j == 13) impact_detach(c, T, Q, n, LK_ANG(t));
    else { T->alive = 0; Q->alive = 0; }
  }
  c->nreq_step = 0;
  return OR_OK;
}

static int list_pass(or_ctx* c, uint32_t n) {
  for (int t = 0; t < 16; t++) {
    if (LIST[t].n > 0) list_gas_type(c, t, n);
    else {
      int rc = list_partner_type(c, t, n);
      if (rc) return rc;
    }
    if (c->nbir > 0) {
      int rc = commit_births(c);
      if (rc) return rc;
    }
  }
  return OR_OK;
}

/* ----------------------------------------------------------------------- */
/* intra-species Coulomb collisions (1)-(3): binary model of Takizuka and  */
/* Abe with a Gaussian tan(chi/2) of variance Eq. (2) and uniform azimuth  */
/* ----------------------------------------------------------------------- */
typedef struct {
  uint32_t h;
  uint64_t id;
  int64_t idx;
} ckey;

static void ta_collide_m(or_ctx* c, part* A, part* B, real cc, uint64_t rid, uint32_t n, uint32_t k,
                         int sp, int64_t m, int half, real fa, real fb, double ma, double mb);

/* like particles: each takes half of the change of the relative velocity */
static void ta_collide(or_ctx* c, part* A, part* B, real cc, uint64_t rid, uint32_t n, uint32_t k, int sp,
                       int64_t m, int half) {
  ta_collide_m(c, A, B, cc, rid, n, k, sp, m, half, (real)0.5, (real)0.5, 1.0, 1.0);
}

static int ckey_cmp(const void* x, const void* y) {
  const ckey* a = (const ckey*)x;
  const ckey* b = (const ckey*)y;
  if (a->h != b->h) return a->h < b->h ? -1 : 1;
  if (a->id != b->id) return a->id < b->id ? -1 : 1;
  return 0;
}

/* one binary collision of A and B (equal masses); cc = Eq. (2) prefactor times the
   particle count m of the cell; randoms from Philox with counter (rid_lo, rid_hi, n, k),
   where rid = (s N + cell) 2^32 + rank of A in the cell's pairing order */
static void ta_collide_m(or_ctx* c, part* A, part* B, real cc, uint64_t rid, uint32_t n, uint32_t k,
                         int sp, int64_t m, int half, real fa, real fb, double ma, double mb) {
  real ux = A->v[0] - B->v[0], uy = A->v[1] - B->v[1], uz = A->v[2] - B->v[2];
  real up2 = ux * ux + uy * uy;
  real u2 = up2 + uz * uz;
  if (!(u2 > (real)0)) return;
  real u = RSQRT(u2);
  real var = cc / (u2 * u);
  uint32_t w[4];
  rng(c->P.seed, rid, n, k, w);
  real st, omc;
  if (var > (real)1) { /* deflection too large for the small-angle model: isotropic */
    real ct = (real)1 - (real)2 * unif(w[3]);
    st = RSQRT((real)1 - ct * ct);
    omc = (real)1 - ct;
  } else {
    real nrm = bm_radius(unif(w[0])) * cos2pi(unif(w[1]));
    real d = RSQRT(var) * nrm;
    real d2 = d * d;
    real inv = (real)1 / ((real)1 + d2);
    st = (d + d) * inv;
    omc = (d2 + d2) * inv;
  }
  real ph = unif(w[2]);
  real s1 = st * cos2pi(ph), s2 = st * sin2pi(ph);
  real du[3];
  if (up2 > (real)0) {
    real up = RSQRT(up2);
    real iup = (real)1 / up;
    real r = uz * s1, t = u * s2;
    du[0] = (ux * r - uy * t) * iup - ux * omc;
    du[1] = (uy * r + ux * t) * iup - uy * omc;
    du[2] = -(up * s1) - uz * omc;
  } else {
    du[0] = u * s1;
    du[1] = u * s2;
    du[2] = -(u * omc);
  }
  double pb[3], pa[3], keb = 0, kea = 0;
  if (c->log) {
    for (int d = 0; d < 3; d++) pb[d] = ma * (double)A->v[d] + mb * (double)B->v[d];
    keb = ke(ma, A->v) + ke(mb, B->v);
  }
  /* the relative velocity changes by du; each particle takes its share mu/m */
  for (int d = 0; d < 3; d++) {
    A->v[d] = A->v[d] + fa * du[d];
    B->v[d] = B->v[d] - fb * du[d];
  }
  if (c->log && c->nlog < c->caplog) {
    for (int d = 0; d < 3; d++) pa[d] = ma * (double)A->v[d] + mb * (double)B->v[d];
    kea = ke(ma, A->v) + ke(mb, B->v);
    double vx = (double)A->v[0] - B->v[0], vy = (double)A->v[1] - B->v[1], vz = (double)A->v[2] - B->v[2];
    double cosx = ((double)ux * vx + (double)uy * vy + (double)uz * vz) /
                  (sqrt((double)u2) * sqrt(vx * vx + vy * vy + vz * vz));
    double t2 = (1.0 - cosx) / (1.0 + cosx);
    double* e = c->log + 16 * c->nlog++;
    memset(e, 0, 16 * sizeof(double));
    e[0] = 100; e[1] = sp; e[2] = keb; e[3] = kea;
    for (int d = 0; d < 3; d++) { e[4 + d] = pb[d]; e[7 + d] = pa[d]; }
    e[11] = (double)var; e[12] = t2; e[13] = sqrt((double)u2); e[14] = (double)m; e[15] = half;
  }
}

static void coulomb(or_ctx* c, uint32_t n) {
  int N = c->N;
  for (int s = 0; s < 3; s++) {
    store* S = &c->st[s];
    int64_t* start = (int64_t*)calloc((size_t)N + 1, sizeof(int64_t));
    int64_t nal = 0;
    for (int64_t i = 0; i < S->n; i++)
      if (S->a[i].alive) { start[S->a[i].cell + 1]++; nal++; }
    for (int cc = 0; cc < N; cc++) start[cc + 1] += start[cc];
    ckey* keys = (ckey*)malloc(sizeof(ckey) * (size_t)(nal > 0 ? nal : 1));
    int64_t* fill = (int64_t*)calloc((size_t)N, sizeof(int64_t));
    for (int64_t i = 0; i < S->n; i++) {
      part* p = &S->a[i];
      if (!p->alive) continue;
      uint32_t w[4];
      rng(c->P.seed, p->id, n, 16, w);
      ckey* k = &keys[start[p->cell] + fill[p->cell]++];
      k->h = w[0];
      k->id = p->id;
      k->idx = i;
    }
    for (int cc = 0; cc < N; cc++) {
      int64_t m = start[cc + 1] - start[cc];
      if (m < 2) continue;
      ckey* K = keys + start[cc];
      qsort(K, (size_t)m, sizeof(ckey), ckey_cmp);
      const uint64_t key = (uint64_t)(s * N + cc) << 32;
      int64_t first = 0;
      if (m % 2 == 1) {  /* odd: the first three collide pairwise with half the interval */
        real ch = c->cc_coul_half[s] * (real)m;
        part *a = &S->a[K[0].idx], *b = &S->a[K[1].idx], *d = &S->a[K[2].idx];
        ta_collide(c, a, b, ch, key | 0, n, 17, s, m, 1);
        ta_collide(c, b, d, ch, key | 1, n, 18, s, m, 1);
        ta_collide(c, d, a, ch, key | 2, n, 19, s, m, 1);
        first = 3;
      }
      real cf = c->cc_coul[s] * (real)m;
      for (int64_t q = first; q + 1 < m; q += 2)
        ta_collide(c, &S->a[K[q].idx], &S->a[K[q + 1].idx], cf, key | (uint64_t)q, n, 17, s, m, 0);
    }
    free(start);
    free(keys);
    free(fill);
  }
}

/* the alive particles of species s grouped by cell, each cell in pairing
   order: Philox counter (id, n, k) word 0, ties by id; start[N + 1] */
static ckey* cell_order(or_ctx* c, int s, uint32_t n, uint32_t k, int64_t** start_out) {
  int N = c->N;
  store* S = &c->st[s];
  int64_t* start = (int64_t*)calloc((size_t)N + 1, sizeof(int64_t));
  int64_t nal = 0;
  for (int64_t i = 0; i < S->n; i++)
    if (S->a[i].alive) { start[S->a[i].cell + 1]++; nal++; }
  for (int cc = 0; cc < N; cc++) start[cc + 1] += start[cc];
  ckey* keys = (ckey*)malloc(sizeof(ckey) * (size_t)(nal > 0 ? nal : 1));
  int64_t* fill = (int64_t*)calloc((size_t)N, sizeof(int64_t));
  for (int64_t i = 0; i < S->n; i++) {
    part* p = &S->a[i];
    if (!p->alive) continue;
    uint32_t w[4];
    rng(c->P.seed, p->id, n, k, w);
    ckey* q = &keys[start[p->cell] + fill[p->cell]++];
    q->h = w[0];
    q->id = p->id;
    q->idx = i;
  }
  for (int cc = 0; cc < N; cc++)
    if (start[cc + 1] - start[cc] > 1) qsort(keys + start[cc], (size_t)(start[cc + 1] - start[cc]), sizeof(ckey), ckey_cmp);
  free(fill);
  *start_out = start;
  return keys;
}

/* Inter-species Coulomb collisions (the unlike-particle rule of the binary
   model of Takizuka and Abe): for the pairs (e, O-), (e, O2+), (O-, O2+) in
   turn, in each cell holding N_a and N_b particles of the two species, every
   particle of the more numerous species (the first species on a tie)
   collides once: the one of rank i with the particle of rank i mod N_min of
   the other species, in increasing i, so that a particle of the less
   numerous species collides about N_max / N_min times in a row.  Ranks in
   each species' own pairing order (Philox k = 20); the variance of
   tan(chi/2) is that of Eq. (2) with the reduced mass of the pair and the
   lower density W N_min / (A dx); the velocities change by mu/m of the
   change of the relative velocity.  Randoms: counter
   ((q N + cell) 2^32 + i, n, 21), q the pair. */
static void coulomb_inter(or_ctx* c, uint32_t n) {
  static const int pa[3] = {0, 0, 1}, pb[3] = {1, 2, 2};
  int N = c->N;
  int64_t* st[3];
  ckey* K[3];
  for (int s = 0; s < 3; s++) K[s] = cell_order(c, s, n, 20, &st[s]);
  for (int q = 0; q < 3; q++) {
    int a = pa[q], b = pb[q];
    for (int cc = 0; cc < N; cc++) {
      int64_t na = st[a][cc + 1] - st[a][cc], nb = st[b][cc + 1] - st[b][cc];
      if (na == 0 || nb == 0) continue;
      int big = na >= nb ? a : b, sml = na >= nb ? b : a;
      int64_t nbig = na >= nb ? na : nb, nsml = na >= nb ? nb : na;
      real fbig = c->fr_inter[q][big == a ? 0 : 1], fsml = c->fr_inter[q][big == a ? 1 : 0];
      real cf = c->cc_inter[q] * (real)nsml;
      const uint64_t key = (uint64_t)(q * N + cc) << 32;
      const ckey* KB = K[big] + st[big][cc];
      const ckey* KS = K[sml] + st[sml][cc];
      for (int64_t i = 0; i < nbig; i++) {
        part* A = &c->st[big].a[KB[i].idx];
        part* B = &c->st[sml].a[KS[i % nsml].idx];
        ta_collide_m(c, A, B, cf, key | (uint64_t)i, n, 21, 3 + q, nsml, big, fbig, fsml, c->mass[big],
                     c->mass[sml]);
      }
    }
  }
  for (int s = 0; s < 3; s++) {
    free(st[s]);
    free(K[s]);
  }
}

static int birth_cmp(const void* x, const void* y) {
  const birth* a = (const birth*)x;
  const birth* b = (const birth*)y;
  if (a->creator != b->creator) return a->creator < b->creator ? -1 : 1;
  return a->k - b->k;
}

static int commit_births(or_ctx* c) {
  qsort(c->bir, (size_t)c->nbir, sizeof(birth), birth_cmp);
  for (int64_t i = 0; i < c->nbir; i++) {
    birth* b = &c->bir[i];
    store* S = &c->st[b->sp];
    if (st_grow(S, S->n + 1)) return OR_ENOMEM;
    part q;
    q.id = c->next_id + (uint64_t)i;
    q.alive = 1;
    q.cell = b->cell;
    q.sort_cell = -1;
    q.off = b->off;
    q.v[0] = b->v[0]; q.v[1] = b->v[1]; q.v[2] = b->v[2];
    S->a[S->n++] = q;
  }
  c->next_id += (uint64_t)c->nbir;
  c->births += c->nbir;
  c->nbir = 0;
  if (c->next_id > ID_MASK) return OR_EOVERFLOW;
  return OR_OK;
}

static int one_step(or_ctx* c) {
  int N = c->N;
  uint32_t n = (uint32_t)c->step;
  int M = c->P.steps_per_period;
  int ion = (c->step % c->P.ion_subcycle) == 0;
  deposit_all(c);
  solve(c, c->Udrive[c->step % M]);
  for (int i = 0; i < 3 * (N + 1); i++) c->Qacc[i] += c->Q[i];
  for (int i = 0; i <= N; i++) c->phiacc[i] += c->phi[i];
  for (int s = 0; s < 3; s++) {
    if (s != SP_E && !ion) continue;
    if (!c->P.dsmc && pmax_of(c, s) > 1.0) return OR_EGUARD;
  }
  c->nreq_step = 0;
  c->nbir = 0;
  push_species(c, SP_E, n);
  if (ion) {
    push_species(c, SP_N, n);
    push_species(c, SP_P, n);
  }
  claims(c, n);
  if (c->nanflag) return OR_EGUARD;
  int rc = commit_births(c);
  if (rc) return rc;
  if ((c->step + 1) % c->P.sort_every == 0) {
    do_sort(c);
    if (c->P.dsmc) {
      rc = list_pass(c, n);
      if (rc) return rc;
      do_sort(c);
    }
  }
  if (c->P.coulomb_every > 0 && (c->step + 1) % c->P.coulomb_every == 0) {
    coulomb(c, n);
    if (c->P.coulomb_inter) coulomb_inter(c, n);
  }
  if ((c->step + 1) % M == 0) {
    memcpy(c->Qlast, c->Qacc, sizeof(int64_t) * 3 * (size_t)(N + 1));
    memcpy(c->philast, c->phiacc, sizeof(double) * (size_t)(N + 1));
    int nb = c->P.eedf_bins > 0 ? c->P.eedf_bins : 1;
    memcpy(c->eedf_last, c->eedf_acc, sizeof(int64_t) * (size_t)(nb + 1));
    int nf = (c->P.fneg_xbins > 0 ? c->P.fneg_xbins : 1) * (c->P.fneg_ebins > 0 ? c->P.fneg_ebins : 1);
    memcpy(c->fneg_last, c->fneg_acc, sizeof(int64_t) * (size_t)nf);
    memset(c->Qacc, 0, sizeof(int64_t) * 3 * (size_t)(N + 1));
    memset(c->phiacc, 0, sizeof(double) * (size_t)(N + 1));
    memset(c->eedf_acc, 0, sizeof(int64_t) * (size_t)(nb + 1));
    memset(c->fneg_acc, 0, sizeof(int64_t) * (size_t)nf);
    c->cycles++;
  }
  c->step++;
  return OR_OK;
}

int or_step(or_ctx* c, int64_t n_steps) {
  for (int64_t k = 0; k < n_steps; k++) {
    int rc = one_step(c);
    if (rc) return rc;
  }
  return OR_OK;
}

/* ----------------------------------------------------------------------- */
/* queries                                                                  */
/* ----------------------------------------------------------------------- */
int64_t or_alive(const or_ctx* c, int sp) {
  int64_t k = 0;
  for (int64_t i = 0; i < c->st[sp].n; i++) k += c->st[sp].a[i].alive;
  return k;
}

int64_t or_particles(const or_ctx* c, int sp, int64_t cap, uint64_t* id, int32_t* cell, double* off, double* v) {
  int64_t k = 0;
  for (int64_t i = 0; i < c->st[sp].n; i++) {
    const part* p = &c->st[sp].a[i];
    if (!p->alive) continue;
    if (k < cap) {
      id[k] = p->id;
      cell[k] = p->cell;
      off[k] = (double)p->off;
      for (int d = 0; d < 3; d++) v[3 * k + d] = (double)p->v[d];
    }
    k++;
  }
  return k;
}

/* the field the next step will use: solved from the current particles */
void or_field(const or_ctx* c, double* phi, double* E) {
  or_ctx* m = (or_ctx*)c;
  deposit_all(m);
  solve(m, m->Udrive[m->step % m->P.steps_per_period]);
  memcpy(phi, c->phi, sizeof(double) * (size_t)(c->N + 1));
  memcpy(E, c->E, sizeof(double) * (size_t)(c->N + 1));
}

void or_charge(const or_ctx* c, int64_t* Q) {
  deposit_all((or_ctx*)c);
  memcpy(Q, c->Q, sizeof(int64_t) * 3 * (size_t)(c->N + 1));
}

void or_counters(const or_ctx* c, int64_t* events, int64_t* absorbed, int64_t* misc) {
  memcpy(events, c->events, sizeof(c->events));
  memcpy(absorbed, c->absorbed, sizeof(c->absorbed));
  misc[0] = c->psteps;
  misc[1] = c->births;
  misc[2] = (int64_t)c->next_id;
  misc[3] = c->step;
  misc[4] = c->cycles;
  misc[5] = c->tophits;
  misc[6] = c->nreq;
  misc[7] = c->nacc;
}

void or_cycle_sums(const or_ctx* c, int64_t* Qsum, double* phisum, int64_t* eedf, int64_t* fneg) {
  int N = c->N;
  memcpy(Qsum, c->Qlast, sizeof(int64_t) * 3 * (size_t)(N + 1));
  memcpy(phisum, c->philast, sizeof(double) * (size_t)(N + 1));
  int nb = c->P.eedf_bins > 0 ? c->P.eedf_bins : 1;
  memcpy(eedf, c->eedf_last, sizeof(int64_t) * (size_t)(nb + 1));
  int nf = (c->P.fneg_xbins > 0 ? c->P.fneg_xbins : 1) * (c->P.fneg_ebins > 0 ? c->P.fneg_ebins : 1);
  memcpy(fneg, c->fneg_last, sizeof(int64_t) * (size_t)nf);
}

void or_constants(const or_ctx* c, double* out) {
  for (int s = 0; s < 3; s++) out[s] = pmax_of(c, s);
  for (int s = 0; s < 3; s++) out[3 + s] = c->M_gas[s];
  out[6] = c->M_ad;
  out[7] = c->M_ch[12];
  out[8] = c->M_ch[13];
  out[9] = c->M_ch[17];
  out[10] = c->dx;
  out[11] = c->dt;
  out[12] = c->ngas;
  out[13] = c->cphi;
  out[14] = c->cE;
  out[15] = (double)c->segmax[SP_P];
}

void or_scale_velocities(or_ctx* c, int sp, const double f[3]) {
  store* S = &c->st[sp];
  for (int64_t i = 0; i < S->n; i++)
    for (int d = 0; d < 3; d++) S->a[i].v[d] = (real)((double)S->a[i].v[d] * f[d]);
}

void or_log_enable(or_ctx* c, int64_t cap) {
  free(c->log);
  c->log = cap > 0 ? (double*)calloc((size_t)cap * 16, sizeof(double)) : NULL;
  c->caplog = cap;
  c->nlog = 0;
}

int64_t or_log_read(const or_ctx* c, double* out, int64_t cap) {
  int64_t k = c->nlog < cap ? c->nlog : cap;
  if (k > 0) memcpy(out, c->log, sizeof(double) * 16 * (size_t)k);
  return c->nlog;
}
