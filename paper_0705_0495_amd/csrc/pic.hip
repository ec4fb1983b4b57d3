// Host runtime and C ABI of the gfx950 PIC-MCC library (declared in pic.h).
//
// The host computes the constants of a discharge once (in double, rounded
// once to the particle precision), owns the device memory and enqueues the
// kernels of each step on one HIP stream:
//   k_push     fused gather/push/absorb/null test/deposit, then the
//              collisions of each workgroup's candidates (persistent grid)
//   k_serial   partner reactions, births, closing the step and the field
//              solve of the next step (1 workgroup)
//   k_sort_*   every sort_every steps, followed by k_coulomb (every
//              coulomb_every steps) and k_field
// Nothing in a step waits for the host.
#include "pic.h"

#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <string>
#include <vector>

#include "pic_kernels.hpp"
#include "pic_list.hpp"

using namespace pic;

namespace {

const double QE = 1.602176634e-19;
const double KB = 1.380649e-23;
const double EPS0 = 8.8541878128e-12;
const double ME = 9.1093837015e-31;
const double AMU = 1.66053906660e-27;
const double TWO_PI_H = 6.283185307179586;

double node_energy(int k) { return std::ldexp(1.0 + (double)(k % 32) / 32.0, -14 + k / 32); }

// upper bound of sum_j sigma_j(E) g(E) on the tabulated range: larger end
// value of each segment times g at its upper end; constant below the first node
double bound_sum(const double* sig, const int* ch, int nch, double mu) {
  const double c2 = (2.0 * QE) / mu;
  double M = 0.0;
  double s0 = 0.0;
  for (int q = 0; q < nch; q++) s0 = s0 + sig[ch[q] * NPT + 0];
  M = std::max(M, s0 * std::sqrt(node_energy(0) * c2));
  for (int k = 0; k < NPT - 1; k++) {
    double s = 0.0;
    for (int q = 0; q < nch; q++) {
      double a = sig[ch[q] * NPT + k], b = sig[ch[q] * NPT + k + 1];
      s = s + (a > b ? a : b);
    }
    double v = s * std::sqrt(node_energy(k + 1) * c2);
    if (v > M) M = v;
  }
  return M * (1.0 + 1.0 / 65536.0);
}

struct Base {
  virtual ~Base() {}
  virtual int create() = 0;
  virtual int step(int64_t n) = 0;
  virtual int particles(int sp, int64_t cap, uint64_t* id, int32_t* cell, double* off, double* v, int64_t* n) = 0;
  virtual int field(double* phi, double* E) = 0;
  virtual int charge(int64_t* Q) = 0;
  virtual int moments(pic_moments_t* m) = 0;
  virtual int read_err(int32_t* err) = 0;
  virtual void set_grid(int g) = 0;
  virtual int set_graphs(int on) = 0;
  virtual int64_t chunk() const = 0;
  virtual int64_t steps_done() const = 0;
  virtual int64_t chunk_period() const = 0;
  virtual int autotune(int64_t steps, int32_t* chosen) = 0;
  virtual bool graphs_on() const = 0;
  virtual int set_shape(int shape) = 0;
  virtual void launch_shape(int32_t* shape, int32_t* grid) const = 0;
  virtual int grid_default_of(int shape) const = 0;
};

}  // namespace

struct pic_ctx {
  pic_geometry G;
  pic_gas gas;
  std::vector<double> sigma, thr, loss;
  double U_rf, freq, pres;
  int dev = 0;                   // HIP device of the context's memory
  hipStream_t stream = nullptr;
  hipStream_t own = nullptr;
  hipEvent_t order_ev = nullptr;  // orders this context's stream before batched launches
  char* btab = nullptr;           // device tables of batches led by this context (grown, kept)
  size_t btab_bytes = 0;
  int bshape = 0, bgrid = 0;         // push launch shape and grid of batches led by this context (0: default)
  hipGraphExec_t bgraph = nullptr;  // one captured period of the batch led by this context
  std::vector<char> bsig;           // what that capture depends on: tables, their address, steps
  std::string msg;
  int err = 0;
  bool timing = false;
  int time_every = 1;        // record the events around every time_every-th launch
  int64_t time_count = 0;    // launches of the fused kernel since timing was enabled
  std::vector<std::pair<hipEvent_t, hipEvent_t>> events;
  size_t ev_used = 0;
  double timed_ms = 0;
  int64_t timed_launches = 0;
  Base* impl = nullptr;
};

static int fail(pic_ctx* c, int code, const std::string& m) {
  if (c) {
    if (!c->err) {
      c->err = code;
      c->msg = m;
    }
  }
  return code;
}

// an argument error that leaves the context usable: message only, not sticky
static int reject(pic_ctx* c, const std::string& m) {
  if (c && !c->err) c->msg = m;
  return PIC_EINVAL;
}

#define HIPCHK(ctx, call)                                                                     \
  do {                                                                                        \
    hipError_t e_ = (call);                                                                   \
    if (e_ != hipSuccess)                                                                     \
      return fail((ctx), e_ == hipErrorOutOfMemory ? PIC_ENOMEM : PIC_EDEVICE,                \
                  std::string(#call) + ": " + hipGetErrorString(e_));                         \
  } while (0)

namespace {

template <class R>
struct Impl : Base {
  pic_ctx* c;
  Consts<R> C;
  Dev<R> D;
  std::vector<void*> allocs;
  int grid_push = 0, grid_push_default = 0, grid_births = 64, grid_scatter = 0, ncu = 1;
  int shape = 0;                    // launch shape of the push kernel (SHAPE_TPB/SHAPE_PPT index)
  int grid_def[SHAPES] = {0, 0, 0};  // occupancy-derived persistent grid of each shape
  int64_t nstep = 0;  // steps enqueued
  bool elds = false;  // k_push stages the node field in LDS
  Dev<R> hD[2];             // host source of the device copies (kept until the copies are done)
  Consts<R>* dC = nullptr;  // device copies of C and of D at both buffer parities (read by k_push)
  Dev<R>* dD = nullptr;
  const int32_t* dev_parity0_cell = nullptr;  // D.st[0].cell at parity 0
  int tab_total = 0;  // values of the compact gas-channel copies (Dev::sigc)
  bool graphs = false;                // replay captured step sequences
  hipGraphExec_t gexec = nullptr;     // period() steps from a step count divisible by period()
  bool list = false;                  // collisions (4)-(19) as the per-cell list (pic_gas::dsmc)
  ListK LK;

  explicit Impl(pic_ctx* ctx) : c(ctx) { memset(&D, 0, sizeof(D)); memset(&C, 0, sizeof(C)); }
  ~Impl() override {
    if (gexec) (void)hipGraphExecDestroy(gexec);
    for (void* p : allocs) (void)hipFree(p);
  }

  // steps after which the launch sequence repeats with the same arguments:
  // the sort and Coulomb periods, doubled so that the sorts' exchanges of the
  // two particle buffers return them to where they were
  int64_t period() const {
    const int64_t a = c->G.sort_every, b = c->G.coulomb_every > 0 ? c->G.coulomb_every : 1;
    int64_t x = a, y = b;
    while (y) {
      const int64_t t = x % y;
      x = y;
      y = t;
    }
    return 2 * (a / x) * b;
  }
  int64_t chunk() const override { return graphs ? period() : (int64_t)c->G.sort_every; }
  int64_t steps_done() const override { return nstep; }
  int64_t chunk_period() const override { return period(); }
  bool graphs_on() const override { return graphs; }

  void launch_shape(int32_t* sh, int32_t* g) const override {
    if (sh) *sh = shape;
    if (g) *g = grid_push;
  }
  int grid_default_of(int sh) const override { return grid_def[sh]; }
  int set_shape(int sh) override {
    if (sh < 0 || sh >= SHAPES) return PIC_EINVAL;
    shape = sh;
    grid_push = grid_push_default = grid_def[sh];
    drop_graph();
    return 0;
  }

  // times the push kernel on a few launch shapes (threads per workgroup and
  // particles per thread) and persistent-grid sizes, steps_per_trial real
  // steps each (results depend on neither), and keeps the fastest
  int autotune(int64_t steps, int32_t* chosen) override {
    const bool was = c->timing;
    const int was_every = c->time_every;
    std::vector<std::pair<int, int>> cand;
    cand.push_back({0, grid_def[0]});
    for (int k : {1, 2, 4, 6, 8})
      if (k * ncu != grid_def[0]) cand.push_back({0, k * ncu});
    for (int sh = 1; sh < SHAPES; sh++) {
      cand.push_back({sh, grid_def[sh]});
      cand.push_back({sh, std::max(1, (3 * grid_def[sh]) / 4)});
    }
    std::pair<int, int> best = cand[0];
    double tbest = 1e300;
    for (const auto& sg : cand) {
      set_shape(sg.first);
      set_grid(sg.second);
      c->timing = true;
      c->time_every = 1;
      c->time_count = 0;
      c->timed_ms = 0;
      c->timed_launches = 0;
      c->ev_used = 0;
      int rc = step_eager(steps);
      if (!rc) rc = drain_events();
      if (rc) return rc;
      const double t = c->timed_ms / (double)std::max<int64_t>(1, c->timed_launches);
      if (t < tbest) {
        tbest = t;
        best = sg;
      }
    }
    c->timing = was;
    c->time_every = was_every;
    c->time_count = 0;
    c->timed_ms = 0;
    c->timed_launches = 0;
    c->ev_used = 0;
    set_shape(best.first);
    set_grid(best.second);
    if (chosen) *chosen = best.second;
    return 0;
  }

  template <class T>
  int alloc(T** p, size_t n) {
    void* q = nullptr;
    size_t bytes = std::max<size_t>(n, 1) * sizeof(T);
    hipError_t e = hipMalloc(&q, bytes);
    if (e != hipSuccess) return fail(c, PIC_ENOMEM, "hipMalloc of " + std::to_string(bytes) + " bytes failed");
    allocs.push_back(q);
    e = hipMemsetAsync(q, 0, bytes, c->stream);
    if (e != hipSuccess) return fail(c, PIC_EDEVICE, "hipMemsetAsync failed");
    *p = (T*)q;
    return 0;
  }

  int alloc_store(Store<R>& s, int64_t cap) {
    int rc;
    if ((rc = alloc(&s.cell, cap + 4))) return rc;
    if ((rc = alloc(&s.off, cap + 4))) return rc;
    if ((rc = alloc(&s.vx, cap + 4))) return rc;
    if ((rc = alloc(&s.vyz, 2 * (cap + 4)))) return rc;
    if ((rc = alloc(&s.id, cap + 4))) return rc;
    return 0;
  }

  void constants() {
    const pic_geometry& G = c->G;
    const int N = G.n_cells;
    const double dx = G.gap_m / (double)N;
    const double dt = 1.0 / (c->freq * (double)G.steps_per_period);
    const double ngas = c->pres / (KB * c->gas.T_gas_K);
    const double MO2 = 31.998 * AMU;
    const double mass[3] = {ME, 15.999 * AMU + ME, MO2 - ME};
    const double charge[3] = {-QE, -QE, QE};
    const double tau[3] = {dt, dt * (double)G.ion_subcycle, dt * (double)G.ion_subcycle};
    C.N = N;
    C.cmid = N / 2;
    C.M = G.steps_per_period;
    C.nsub = G.ion_subcycle;
    C.seed_lo = (uint32_t)G.seed;
    C.seed_hi = (uint32_t)(G.seed >> 32);
    double mu_g[3];
    for (int s = 0; s < 3; s++) {
      const double qm = charge[s] / mass[s];
      C.qmdt[s] = (R)(qm * tau[s]);
      C.dtdx[s] = (R)(tau[s] / dx);
      C.hk[s] = (R)(qm * (0.5 * tau[s]));
      C.vth0[s] = (R)std::sqrt((G.T_init_eV[s] * QE) / mass[s]);
      mu_g[s] = (mass[s] * MO2) / (mass[s] + MO2);
      C.a_g[s] = (R)(MO2 / (mass[s] + MO2));
      C.b_g[s] = (R)(mass[s] / (mass[s] + MO2));
      C.hmu_g[s] = (R)((0.5 * mu_g[s]) / QE);
      C.c2e_g[s] = (R)((2.0 * QE) / mu_g[s]);
    }
    C.vthg = (R)std::sqrt((KB * c->gas.T_gas_K) / MO2);
    // partner channels 12 (e, O2+), 13 (e, O-), 17 (O-, O2+): the slot of Eq. (1)
    // per partner particle of the cell is tau M_j W / (A dx), W real particles each
    const int pch[3] = {12, 13, 17}, ps[3] = {0, 0, 1}, pt[3] = {2, 1, 2};
    double Mpart[3];
    const double* sig = c->sigma.data();
    for (int q = 0; q < 3; q++) {
      const double ms = mass[ps[q]], mt = mass[pt[q]];
      const double mu = (ms * mt) / (ms + mt);
      C.a_c[q] = (R)(mt / (ms + mt));
      C.b_c[q] = (R)(ms / (ms + mt));
      C.hmu_c[q] = (R)((0.5 * mu) / QE);
      C.c2e_c[q] = (R)((2.0 * QE) / mu);
      const int one[1] = {pch[q]};
      const double Mj = bound_sum(sig, one, 1, mu);
      C.Mr_c[q] = (R)Mj;
      C.KP[q] = ((tau[ps[q]] * Mj) * G.weight) / (G.area_m2 * dx);
      Mpart[q] = Mj;
    }
    C.ddf = (R)std::sqrt((0.1 * mass[1]) / ME);
    C.adf = (R)std::sqrt(mu_g[1] / ME);
    C.hme = (R)((0.5 * ME) / QE);
    C.hmn = (R)((0.5 * mass[1]) / QE);
    for (int j = 0; j < NCH; j++) {
      C.thr[j] = (R)c->thr[j];
      C.loss[j] = (R)c->loss[j];
      C.PG[j] = 0.0;
    }
    for (int j = 0; j < NCH; j++) {
      if (j == 12 || j == 13 || j == 17) continue;
      const int s = j <= 11 ? 0 : (j <= 16 ? 1 : 2);
      C.PG[j] = (j == 16) ? (tau[s] * c->gas.metastable_frac) * ngas : tau[s] * ngas;
    }
    const int ge[12] = {0, 1, 2, 3, 4, 5, 6, 7, 8, 9, 10, 11}, gn[2] = {14, 15}, gp[1] = {18}, gad[1] = {16};
    const double Me = bound_sum(sig, ge, 12, mu_g[0]);
    const double Mn = bound_sum(sig, gn, 2, mu_g[1]);
    const double Mp = bound_sum(sig, gp, 1, mu_g[2]);
    const double Mad = bound_sum(sig, gad, 1, mu_g[1]);
    // compact copies of each species' gas channels for the collisions' LDS:
    // channel j from node tab_k0[j] (the last zero node below its first
    // nonzero one) up; species s's copy at tab_base[s] of Dev::sigc
    {
      const int g0[3] = {0, 14, 18}, gn[3] = {12, 3, 1};
      for (int j = 0; j < NCH; j++) C.tab_k0[j] = C.tab_off[j] = 0;
      int base = 0;
      for (int s = 0; s < 3; s++) {
        int off = 0;
        for (int j = g0[s]; j < g0[s] + gn[s]; j++) {
          int f = 0;
          while (f < NPT && sig[(size_t)j * NPT + f] == 0.0) f++;
          const int k0 = f >= NPT ? NPT : std::max(f - 1, 0);
          C.tab_k0[j] = k0;
          C.tab_off[j] = off;
          off += NPT - k0;
        }
        const int padded = (off + 3) & ~3;
        C.tab_n[s] = (size_t)padded * sizeof(R) <= (size_t)TAB_LDS_BYTES ? off : 0;
        C.tab_base[s] = base;
        base += padded;
      }
      tab_total = base;
    }
    C.PGtot[0] = C.PG[0] * Me;
    C.PGtot[1] = C.PG[14] * Mn + C.PG[16] * Mad;
    C.PGtot[2] = C.PG[18] * Mp;
    // the per-cell collision list of Sec. II: every type (4)-(19) with tau =
    // sort_every dt, once per sort; the null-collision test of the push is off
    list = c->gas.dsmc != 0;
    memset(&LK, 0, sizeof(LK));
    if (list) {
      const double tl = dt * (double)G.sort_every;
      for (int j = 0; j < NCH; j++) {
        if (j == 12 || j == 13 || j == 17) continue;
        LK.PGl[j] = (j == 16) ? (tl * c->gas.metastable_frac) * ngas : tl * ngas;
      }
      LK.KPl = (tl * G.weight) / (G.area_m2 * dx);
      for (int q = 0; q < 3; q++) LK.KM[q] = LK.KPl * Mpart[q];
      for (int t = 0; t < LIST_N; t++) {
        if (LIST_NCH[t] == 0) continue;
        int ch[4];
        for (int q = 0; q < LIST_NCH[t]; q++) ch[q] = LIST_CH0[t] + q;
        LK.B[t] = LK.PGl[LIST_CH0[t]] * bound_sum(sig, ch, LIST_NCH[t], mu_g[LIST_SP[t]]);
      }
      for (int s = 0; s < 3; s++) C.PGtot[s] = 0.0;
      for (int q = 0; q < 3; q++) C.KP[q] = 0.0;
    }
    C.cphi = ((dx * QE) * G.weight) / ((EPS0 * 16777216.0) * G.area_m2);
    C.cE = (QE * G.weight) / ((EPS0 * 16777216.0) * G.area_m2);
    C.invdx = 1.0 / dx;
    C.inv2dx = 0.5 / dx;
    C.eedf_bins = G.eedf_bins;
    C.fneg_xbins = G.fneg_xbins;
    C.fneg_ebins = G.fneg_ebins;
    C.eedf_sc = (R)(G.eedf_bins > 0 ? (double)G.eedf_bins / G.eedf_emax_eV : 0.0);
    C.fneg_sc = (R)(G.fneg_ebins > 0 ? (double)G.fneg_ebins / (2.0 * G.fneg_emax_eV) : 0.0);
    C.fneg_em = (R)G.fneg_emax_eV;
    // series of the samplers' sin, cos and ln: coefficients in double, rounded once
    {
      const double h = 1.5707963267948966;  // pi / 2
      const double t = h * h;
      double cs = h, cc = 1.0;
      for (int j = 0; j < Series<R>::NS; j++) {
        C.sinc[j] = (R)cs;
        cs = (cs * -t) / (double)((2 * j + 2) * (2 * j + 3));
      }
      for (int j = 0; j < Series<R>::NC; j++) {
        C.cosc[j] = (R)cc;
        cc = (cc * -t) / (double)((2 * j + 1) * (2 * j + 2));
      }
      for (int k = 0; k < Series<R>::NL; k++) C.logc[k] = (R)(1.0 / (double)(2 * k + 1));
      C.ln2 = (R)0.6931471805599453;
      C.sqrt2 = (R)1.4142135623730951;
    }
    // Eq. (2) with eps0^2 and the reduced mass mu = m/2 of like particles; the
    // density is W * (particles in the cell) / (A dx), t_c2 = coulomb_every dt
    const double PI_H = 3.141592653589793;
    for (int s = 0; s < 3; s++) {
      const double mu = 0.5 * mass[s];
      const double tc2 = dt * (double)(G.coulomb_every > 0 ? G.coulomb_every : 1);
      const double num = ((((QE * QE) * (QE * QE)) * c->gas.coulomb_log) * tc2) * G.weight;
      const double den = (((8.0 * PI_H) * (EPS0 * EPS0)) * (mu * mu)) * (G.area_m2 * dx);
      C.ccoul[s] = (R)(num / den);
      C.ccoul_h[s] = (R)((0.5 * num) / den);
    }
    // unlike pairs (e, O-), (e, O2+), (O-, O2+), all singly charged: the
    // reduced mass of the pair; the density is that of the less numerous one
    {
      const int pa[3] = {0, 0, 1}, pb[3] = {1, 2, 2};
      for (int q = 0; q < 3; q++) {
        const double ma = mass[pa[q]], mb = mass[pb[q]];
        const double mu = (ma * mb) / (ma + mb);
        const double tc2 = dt * (double)(G.coulomb_every > 0 ? G.coulomb_every : 1);
        const double num = ((((QE * QE) * (QE * QE)) * c->gas.coulomb_log) * tc2) * G.weight;
        const double den = (((8.0 * PI_H) * (EPS0 * EPS0)) * (mu * mu)) * (G.area_m2 * dx);
        C.cinter[q] = (R)(num / den);
        C.finter[q][0] = (R)(mu / ma);
        C.finter[q][1] = (R)(mu / mb);
      }
    }
    C.inter = (G.coulomb_every > 0 && c->gas.coulomb_inter) ? 1 : 0;
  }

  int create() override {
    const pic_geometry& G = c->G;
    const int N = G.n_cells;
    constants();
    int rc;
    for (int s = 0; s < 3; s++) {
      int64_t cap = G.capacity[s] > 0 ? G.capacity[s] : 2 * G.n_init[s] + 65536;
      cap = (cap + 3) & ~(int64_t)3;
      if (cap < G.n_init[s] || cap >= ((int64_t)1 << 30) - 8)
        return fail(c, PIC_EINVAL, "capacity must hold the initial load and stay below 2^30");
      D.cap[s] = cap;
      if ((rc = alloc_store(D.st[s], cap))) return rc;
      if ((rc = alloc_store(D.alt[s], cap))) return rc;
    }
    if ((rc = alloc(&D.N, 3))) return rc;
    if ((rc = alloc(&D.Nnew, 3))) return rc;
    if ((rc = alloc(&D.cnt, 3 * (size_t)N))) return rc;
    if ((rc = alloc(&D.F, 3 * (size_t)N))) return rc;
    if ((rc = alloc(&D.seg, 3 * (size_t)(N + 1)))) return rc;
    if ((rc = alloc(&D.cursor, 3 * (size_t)N))) return rc;
    if ((rc = alloc(&D.segmax, 3))) return rc;
    if ((rc = alloc(&D.E2, 2 * (size_t)N))) return rc;
    if ((rc = alloc(&D.phi, (size_t)N + 1))) return rc;
    if ((rc = alloc(&D.E, (size_t)N + 1))) return rc;
    double* Ud;
    if ((rc = alloc(&Ud, (size_t)G.steps_per_period))) return rc;
    D.U = Ud;
    R* sg;
    if ((rc = alloc(&sg, (size_t)NPT * TS))) return rc;
    D.sig = sg;
    int64_t totcap = D.cap[0] + D.cap[1] + D.cap[2];
    D.nb_cap = (int32_t)std::min<int64_t>(std::max<int64_t>(65536, totcap / 32), 1 << 24);
    if ((rc = alloc(&D.nb, (size_t)D.nb_cap))) return rc;
    if ((rc = alloc(&D.nbc, 4))) return rc;
    if ((rc = alloc(&D.bhist, (size_t)NBUCKET))) return rc;
    if ((rc = alloc(&D.perm, (size_t)D.nb_cap))) return rc;
    for (int s = 0; s < 3; s++) {
      if ((rc = alloc(&D.cand[s], (size_t)D.cap[s] + TILE_MAX))) return rc;
      if ((rc = alloc(&D.tcnt[s], (size_t)(D.cap[s] / WTILE_MIN + 8)))) return rc;
    }
    if ((rc = alloc(&D.ncand, 3))) return rc;
    D.req_cap = REQ_CAP;
    if ((rc = alloc(&D.req, (size_t)D.req_cap))) return rc;
    if (list) {
      for (int t = 0; t < LIST_N; t++)
        if (LIST_NCH[t] > 0 && LK.B[t] > 1.0)
          return fail(c, PIC_EINVAL, "collision list: tau n sigma g of type (" + std::to_string(4 + t) +
                                         ") can exceed 1; sort every fewer steps");
      D.lreq_cap = (int32_t)std::min<int64_t>(std::max<int64_t>(REQ_CAP, totcap / 64), 1 << 24);
      if ((rc = alloc(&D.lreq, (size_t)D.lreq_cap))) return rc;
    }
    if ((rc = alloc(&D.nreq, 1))) return rc;
    if ((rc = alloc(&D.ctr, 1))) return rc;
    if ((rc = alloc(&D.Qcur, 3 * (size_t)(N + 1)))) return rc;
    if ((rc = alloc(&D.qnet, (size_t)(N + 1)))) return rc;
    if ((rc = alloc(&D.Qacc, 3 * (size_t)(N + 1)))) return rc;
    if ((rc = alloc(&D.Qlast, 3 * (size_t)(N + 1)))) return rc;
    if ((rc = alloc(&D.phiacc, (size_t)N + 1))) return rc;
    if ((rc = alloc(&D.philast, (size_t)N + 1))) return rc;
    if ((rc = alloc(&D.eedf_acc, (size_t)EEDF_MAX + 1))) return rc;
    if ((rc = alloc(&D.eedf_last, (size_t)EEDF_MAX + 1))) return rc;
    if ((rc = alloc(&D.fneg_acc, (size_t)FNEG_MAX))) return rc;
    if ((rc = alloc(&D.fneg_last, (size_t)FNEG_MAX))) return rc;
    if ((rc = alloc(&D.done, 4))) return rc;
    if ((rc = alloc(&D.ncoul, 1))) return rc;
    if ((rc = alloc(&D.coul_big, 3 * (size_t)N))) return rc;
    if ((rc = alloc(&D.ncl, 1))) return rc;
    if ((rc = alloc(&D.clist, 3 * (size_t)N))) return rc;

    // drive table and cross-section table (host math, uploaded once)
    std::vector<double> U(G.steps_per_period);
    for (int k = 0; k < G.steps_per_period; k++)
      U[k] = G.drive_dc ? c->U_rf : c->U_rf * std::sin((TWO_PI_H * (double)k) / (double)G.steps_per_period);
    std::vector<R> tab((size_t)NPT * TS, (R)0);
    for (int j = 0; j < NCH; j++)
      for (int k = 0; k < NPT; k++) tab[(size_t)k * TS + j] = (R)c->sigma[(size_t)j * NPT + k];
    HIPCHK(c, hipMemcpyAsync(Ud, U.data(), sizeof(double) * U.size(), hipMemcpyHostToDevice, c->stream));
    HIPCHK(c, hipMemcpyAsync(sg, tab.data(), sizeof(R) * tab.size(), hipMemcpyHostToDevice, c->stream));
    // (host buffers of the asynchronous copies live until the synchronisation at the end)
    std::vector<R> cmp((size_t)std::max(tab_total, 4), (R)0);
    {
      const int g0[3] = {0, 14, 18}, gn[3] = {12, 3, 1};
      for (int s = 0; s < 3; s++)
        for (int j = g0[s]; j < g0[s] + gn[s]; j++)
          for (int k = C.tab_k0[j]; k < NPT; k++)
            cmp[(size_t)C.tab_base[s] + C.tab_off[j] + (k - C.tab_k0[j])] = (R)c->sigma[(size_t)j * NPT + k];
      R* sc;
      if ((rc = alloc(&sc, cmp.size()))) return rc;
      D.sigc = sc;
      HIPCHK(c, hipMemcpyAsync(sc, cmp.data(), sizeof(R) * cmp.size(), hipMemcpyHostToDevice, c->stream));
    }
    Counters h;
    memset(&h, 0, sizeof(h));
    h.next_id = G.n_init[0] + G.n_init[1] + G.n_init[2];
    HIPCHK(c, hipMemcpyAsync(D.ctr, &h, sizeof(h), hipMemcpyHostToDevice, c->stream));
    HIPCHK(c, hipMemcpyAsync(D.N, G.n_init, sizeof(int64_t) * 3, hipMemcpyHostToDevice, c->stream));

    // the kernel constants and the device state at both buffer parities, for
    // the kernels that read them from device memory
    {
      if ((rc = alloc(&dC, 1))) return rc;
      if ((rc = alloc(&dD, 2))) return rc;
      dev_parity0_cell = D.st[0].cell;
      hD[0] = D;
      hD[1] = D;
      for (int s = 0; s < 3; s++) std::swap(hD[1].st[s], hD[1].alt[s]);
      HIPCHK(c, hipMemcpyAsync(dC, &C, sizeof(C), hipMemcpyHostToDevice, c->stream));
      HIPCHK(c, hipMemcpyAsync(dD, hD, sizeof(hD), hipMemcpyHostToDevice, c->stream));
    }
    // launch shapes
    int dev = 0, occ = 0;
    HIPCHK(c, hipGetDevice(&dev));
    HIPCHK(c, hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev));
    elds = N <= PushE<R>::MAXN;
    {
      const void* kf[SHAPES] = {
          elds ? (const void*)k_push<R, true, Shape0> : (const void*)k_push<R, false, Shape0>,
          elds ? (const void*)k_push<R, true, Shape1> : (const void*)k_push<R, false, Shape1>,
          elds ? (const void*)k_push<R, true, Shape2> : (const void*)k_push<R, false, Shape2>};
      for (int sh = 0; sh < SHAPES; sh++) {
        HIPCHK(c, hipOccupancyMaxActiveBlocksPerMultiprocessor(&occ, kf[sh], SHAPE_TPB[sh], 0));
        grid_def[sh] = std::max(1, ncu * std::max(1, occ));
      }
    }
    grid_push = grid_push_default = grid_def[shape];
    grid_scatter = std::max(1, ncu * 2);


    // initial load, deposit, field at t = 0, half step back, first sort
    const int64_t tot = G.n_init[0] + G.n_init[1] + G.n_init[2];
    if (tot > 0) {
      const int b = 256;
      const int g = (int)((tot + b - 1) / b);
      hipLaunchKernelGGL(k_load<R>, dim3(g), dim3(b), 0, c->stream, C, D, G.n_init[0], G.n_init[1], G.n_init[2]);
      hipLaunchKernelGGL(k_deposit_all<R>, dim3(g), dim3(b), 0, c->stream, C, D);
    }
    HIPCHK(c, launch_field(C, D, 0, c->stream));
    if (tot > 0) {
      const int b = 256;
      const int g = (int)((tot + b - 1) / b);
      hipLaunchKernelGGL(k_halfkick<R>, dim3(g), dim3(b), 0, c->stream, C, D);
    }
    HIPCHK(c, hipGetLastError());
    if ((rc = sort())) return rc;
    // field, diagnostics and accumulator clearing of step 0
    HIPCHK(c, launch_field(C, D, 1, c->stream));
    HIPCHK(c, hipStreamSynchronize(c->stream));
    int32_t e;
    if ((rc = read_err(&e))) return rc;
    return 0;
  }

  void set_grid(int g) override {
    grid_push = g > 0 ? g : grid_push_default;
    drop_graph();
  }

  void drop_graph() {
    if (gexec) (void)hipGraphExecDestroy(gexec);
    gexec = nullptr;
  }

  int set_graphs(int on) override {
    graphs = on != 0;
    if (!graphs) drop_graph();
    return 0;
  }

  // capture period() steps from the current state (the stream must be idle of
  // other captures); the host's step count and buffers are restored after
  int capture() {
    const int64_t P = period();
    const int64_t n0 = nstep;
    Store<R> st0[3];
    memcpy(st0, D.st, sizeof(st0));
    hipGraph_t g = nullptr;
    HIPCHK(c, hipStreamBeginCapture(c->stream, hipStreamCaptureModeThreadLocal));
    const int rc = step_eager(P);
    const hipError_t e = hipStreamEndCapture(c->stream, &g);
    nstep = n0;
    if (rc) {
      if (g) (void)hipGraphDestroy(g);
      return rc;
    }
    if (e != hipSuccess) return fail(c, PIC_EDEVICE, std::string("hipStreamEndCapture: ") + hipGetErrorString(e));
    if (memcmp(st0, D.st, sizeof(st0)) != 0) {
      (void)hipGraphDestroy(g);
      return fail(c, PIC_EDEVICE, "captured steps did not return the particle buffers");
    }
    const hipError_t ei = hipGraphInstantiate(&gexec, g, nullptr, nullptr, 0);
    (void)hipGraphDestroy(g);
    if (ei != hipSuccess) {
      gexec = nullptr;
      return fail(c, PIC_EDEVICE, std::string("hipGraphInstantiate: ") + hipGetErrorString(ei));
    }
    return 0;
  }

  int step(int64_t nsteps) override {
    if (!graphs || c->timing) return step_eager(nsteps);
    const int64_t P = period();
    while (nsteps > 0) {
      const int64_t ph = nstep % P;
      if (ph == 0 && nsteps >= P) {
        if (!gexec) {
          const int rc = capture();
          if (rc) return rc;
        }
        HIPCHK(c, hipGraphLaunch(gexec, c->stream));
        nstep += P;
        nsteps -= P;
      } else {
        const int64_t k = ph == 0 ? nsteps : std::min(nsteps, P - ph);
        const int rc = step_eager(k);
        if (rc) return rc;
        nsteps -= k;
      }
    }
    return 0;
  }

  int sort() {
    hipLaunchKernelGGL(k_sort_scan<R>, dim3(3), dim3(SCAN_TPB), 0, c->stream, C, D);
    hipLaunchKernelGGL(k_sort_scatter<R>, dim3(grid_scatter), dim3(SORT_TPB), 0, c->stream, C, D);
    HIPCHK(c, hipGetLastError());
    for (int s = 0; s < 3; s++) std::swap(D.st[s], D.alt[s]);
    return 0;
  }

  // the device copy of D at the current buffer parity
  const Dev<R>* dpar() const { return dD + (D.st[0].cell == dev_parity0_cell ? 0 : 1); }

  // the per-cell collision list after the sort of this step's end: the types
  // in the order of Table I, births placed after each type that makes them
  // (at the end of their stores, where the partner choice of impact
  // detachment (19) finds the O- born in (15)), the sort repeated at the end
  void list_partner_kernels(int t, int grid) {
    const Dev<R>* dp = dpar();
    const int gc = 64;
    if (t == 9) {
      hipLaunchKernelGGL((k_list_pick<R, 9>), dim3(grid), dim3(LIST_TPB), 0, c->stream, dC, dp, LK);
      hipLaunchKernelGGL((k_list_claim<R, 9>), dim3(gc), dim3(LIST_TPB), 0, c->stream, dp);
      hipLaunchKernelGGL((k_list_apply<R, 9>), dim3(gc), dim3(LIST_TPB), 0, c->stream, dC, dp);
    } else if (t == 10) {
      hipLaunchKernelGGL((k_list_pick<R, 10>), dim3(grid), dim3(LIST_TPB), 0, c->stream, dC, dp, LK);
      hipLaunchKernelGGL((k_list_claim<R, 10>), dim3(gc), dim3(LIST_TPB), 0, c->stream, dp);
      hipLaunchKernelGGL((k_list_apply<R, 10>), dim3(gc), dim3(LIST_TPB), 0, c->stream, dC, dp);
    } else {
      hipLaunchKernelGGL((k_list_pick<R, 15>), dim3(grid), dim3(LIST_TPB), 0, c->stream, dC, dp, LK);
      hipLaunchKernelGGL((k_list_claim<R, 15>), dim3(gc), dim3(LIST_TPB), 0, c->stream, dp);
      hipLaunchKernelGGL((k_list_apply<R, 15>), dim3(gc), dim3(LIST_TPB), 0, c->stream, dC, dp);
    }
    hipLaunchKernelGGL(k_list_commit<R>, dim3(1), dim3(TAIL_TPB), 0, c->stream, dC, dp);
  }

  int list_pass() {
    const int grid = std::max(1, ncu * 8);
    const Dev<R>* dp = dpar();
    hipLaunchKernelGGL(k_list_scatter<R>, dim3(grid), dim3(LIST_TPB), 0, c->stream, dC, dp, LK);
    list_partner_kernels(9, grid);
    list_partner_kernels(10, grid);
    hipLaunchKernelGGL((k_list_gas<R, 11>), dim3(grid), dim3(LIST_TPB), 0, c->stream, dC, dp, LK);
    hipLaunchKernelGGL(k_list_commit<R>, dim3(1), dim3(TAIL_TPB), 0, c->stream, dC, dp);
    hipLaunchKernelGGL((k_list_gas<R, 12>), dim3(grid), dim3(LIST_TPB), 0, c->stream, dC, dp, LK);
    hipLaunchKernelGGL(k_list_commit<R>, dim3(1), dim3(TAIL_TPB), 0, c->stream, dC, dp);
    hipLaunchKernelGGL((k_list_gas<R, 13>), dim3(grid), dim3(LIST_TPB), 0, c->stream, dC, dp, LK);
    hipLaunchKernelGGL(k_list_commit<R>, dim3(1), dim3(TAIL_TPB), 0, c->stream, dC, dp);
    hipLaunchKernelGGL((k_list_gas<R, 14>), dim3(grid), dim3(LIST_TPB), 0, c->stream, dC, dp, LK);
    hipLaunchKernelGGL(k_list_commit<R>, dim3(1), dim3(TAIL_TPB), 0, c->stream, dC, dp);
    list_partner_kernels(15, grid);
    HIPCHK(c, hipGetLastError());
    return sort();
  }

  template <class SH>
  void launch_push_sh(const Dev<R>* dpar) {
    if (elds) hipLaunchKernelGGL((k_push<R, true, SH>), dim3(grid_push), dim3(SH::TPB), 0, c->stream, dC, dpar);
    else hipLaunchKernelGGL((k_push<R, false, SH>), dim3(grid_push), dim3(SH::TPB), 0, c->stream, dC, dpar);
  }
  void launch_push(const Dev<R>* dpar) {
    if (shape == 1) launch_push_sh<Shape1>(dpar);
    else if (shape == 2) launch_push_sh<Shape2>(dpar);
    else launch_push_sh<Shape0>(dpar);
  }

  int step_eager(int64_t nsteps) {
    const int sort_every = c->G.sort_every;
    for (int64_t k = 0; k < nsteps; k++) {
      hipEvent_t e0 = nullptr, e1 = nullptr;
      const bool timed = c->timing && (c->time_count++ % c->time_every) == 0;
      if (timed) {
        if (c->ev_used == c->events.size()) {
          hipEvent_t a, b;
          HIPCHK(c, hipEventCreate(&a));
          HIPCHK(c, hipEventCreate(&b));
          c->events.push_back({a, b});
        }
        e0 = c->events[c->ev_used].first;
        e1 = c->events[c->ev_used].second;
        c->ev_used++;
        HIPCHK(c, hipEventRecord(e0, c->stream));
      }
      const Dev<R>* dpar = dD + (D.st[0].cell == dev_parity0_cell ? 0 : 1);
      launch_push(dpar);
      if (timed) HIPCHK(c, hipEventRecord(e1, c->stream));
      HIPCHK(c, hipGetLastError());
      nstep++;
      const bool sort_now = (nstep % sort_every) == 0;
      // without a sort the node charge is formed by many workgroups first
      if (!sort_now) HIPCHK(c, launch_charge(C, D, c->stream));
      HIPCHK(c, launch_serial(C, D, sort_now ? 0 : 2, c->stream));
      if (sort_now) {
        int rc = sort();
        if (rc) return rc;
        if (list && (rc = list_pass())) return rc;
        const int ce = c->G.coulomb_every;
        if (ce > 0 && nstep % ce == 0) {
          HIPCHK(c, launch_coulomb(C, D, ncu, c->stream));
        }
        HIPCHK(c, launch_field(C, D, 1, c->stream));
      }
      if (c->timing && c->ev_used >= 16384) {
        int rc = drain_events();
        if (rc) return rc;
      }
    }
    return 0;
  }

  int drain_events() {
    HIPCHK(c, hipStreamSynchronize(c->stream));
    for (size_t i = 0; i < c->ev_used; i++) {
      float ms = 0;
      HIPCHK(c, hipEventElapsedTime(&ms, c->events[i].first, c->events[i].second));
      c->timed_ms += ms;
      c->timed_launches++;
    }
    c->ev_used = 0;
    return 0;
  }

  int read_err(int32_t* e) override {
    Counters h;
    HIPCHK(c, hipMemcpyAsync(&h, D.ctr, sizeof(h), hipMemcpyDeviceToHost, c->stream));
    HIPCHK(c, hipStreamSynchronize(c->stream));
    *e = h.err;
    if (h.err & (ERR_CAP | ERR_NB | ERR_REQ | ERR_ID | ERR_SORT | ERR_COUL))
      return fail(c, PIC_EOVERFLOW, "device reported capacity overflow (flags " + std::to_string(h.err) + ")");
    if (h.err & (ERR_PMAX | ERR_NAN))
      return fail(c, PIC_EGUARD, "device guard raised (flags " + std::to_string(h.err) + ")");
    return 0;
  }

  int particles(int sp, int64_t cap, uint64_t* id, int32_t* cell, double* off, double* v, int64_t* nout) override {
    int64_t Nh[3];
    HIPCHK(c, hipMemcpyAsync(Nh, D.N, sizeof(Nh), hipMemcpyDeviceToHost, c->stream));
    HIPCHK(c, hipStreamSynchronize(c->stream));
    const int64_t n = Nh[sp];
    std::vector<int32_t> hc(n);
    std::vector<R> ho(n), hx(n), hyz(2 * n);
    std::vector<uint64_t> hi(n);
    const Store<R>& s = D.st[sp];
    if (n > 0) {
      HIPCHK(c, hipMemcpyAsync(hc.data(), s.cell, n * sizeof(int32_t), hipMemcpyDeviceToHost, c->stream));
      HIPCHK(c, hipMemcpyAsync(ho.data(), s.off, n * sizeof(R), hipMemcpyDeviceToHost, c->stream));
      HIPCHK(c, hipMemcpyAsync(hx.data(), s.vx, n * sizeof(R), hipMemcpyDeviceToHost, c->stream));
      HIPCHK(c, hipMemcpyAsync(hyz.data(), s.vyz, 2 * n * sizeof(R), hipMemcpyDeviceToHost, c->stream));
      HIPCHK(c, hipMemcpyAsync(hi.data(), s.id, n * sizeof(uint64_t), hipMemcpyDeviceToHost, c->stream));
      HIPCHK(c, hipStreamSynchronize(c->stream));
    }
    int64_t k = 0;
    for (int64_t i = 0; i < n; i++) {
      if (hc[i] == DEAD) continue;
      if (k < cap) {
        if (id) id[k] = hi[i];
        if (cell) cell[k] = hc[i];
        if (off) off[k] = (double)ho[i];
        if (v) {
          v[3 * k] = (double)hx[i];
          v[3 * k + 1] = (double)hyz[2 * i];
          v[3 * k + 2] = (double)hyz[2 * i + 1];
        }
      }
      k++;
    }
    *nout = k;
    return 0;
  }

  int field(double* phi, double* E) override {
    const int N = C.N;
    if (phi) HIPCHK(c, hipMemcpyAsync(phi, D.phi, sizeof(double) * (N + 1), hipMemcpyDeviceToHost, c->stream));
    if (E) HIPCHK(c, hipMemcpyAsync(E, D.E, sizeof(double) * (N + 1), hipMemcpyDeviceToHost, c->stream));
    HIPCHK(c, hipStreamSynchronize(c->stream));
    return 0;
  }

  int charge(int64_t* Q) override {
    const int N = C.N;
    HIPCHK(c, hipMemcpyAsync(Q, D.Qcur, sizeof(int64_t) * 3 * (N + 1), hipMemcpyDeviceToHost, c->stream));
    HIPCHK(c, hipStreamSynchronize(c->stream));
    return 0;
  }

  int moments(pic_moments_t* m) override {
    const int N = C.N;
    Counters h;
    int64_t Nh[3];
    HIPCHK(c, hipMemcpyAsync(&h, D.ctr, sizeof(h), hipMemcpyDeviceToHost, c->stream));
    HIPCHK(c, hipMemcpyAsync(Nh, D.N, sizeof(Nh), hipMemcpyDeviceToHost, c->stream));
    std::vector<int64_t> Q(3 * (size_t)(N + 1));
    std::vector<double> ph(N + 1);
    HIPCHK(c, hipMemcpyAsync(Q.data(), D.Qlast, sizeof(int64_t) * Q.size(), hipMemcpyDeviceToHost, c->stream));
    HIPCHK(c, hipMemcpyAsync(ph.data(), D.philast, sizeof(double) * ph.size(), hipMemcpyDeviceToHost, c->stream));
    if (m->eedf && c->G.eedf_bins > 0)
      HIPCHK(c, hipMemcpyAsync(m->eedf, D.eedf_last, sizeof(int64_t) * (c->G.eedf_bins + 1), hipMemcpyDeviceToHost,
                               c->stream));
    if (m->fneg && c->G.fneg_xbins * c->G.fneg_ebins > 0)
      HIPCHK(c, hipMemcpyAsync(m->fneg, D.fneg_last, sizeof(int64_t) * c->G.fneg_xbins * c->G.fneg_ebins,
                               hipMemcpyDeviceToHost, c->stream));
    HIPCHK(c, hipStreamSynchronize(c->stream));
    m->step = h.step;
    m->cycles = h.cycles;
    for (int j = 0; j < NCH; j++) m->events[j] = h.events[j];
    for (int k = 0; k < 6; k++) m->absorbed[k / 3][k % 3] = h.absorbed[k];
    m->particle_steps = h.psteps;
    m->births = h.births;
    m->next_id = h.next_id;
    // alive counts: every alive particle carries 2^24 units of node charge
    {
      std::vector<int64_t> Qc(3 * (size_t)(N + 1));
      int rc = charge(Qc.data());
      if (rc) return rc;
      for (int s = 0; s < 3; s++) {
        int64_t tot = 0;
        for (int i = 0; i <= N; i++) tot += Qc[(size_t)s * (N + 1) + i];
        m->alive[s] = tot >> 24;
      }
    }
    const double Mst = (double)c->G.steps_per_period;
    const double dx = c->G.gap_m / (double)N;
    if (m->density_m3)
      for (int s = 0; s < 3; s++)
        for (int i = 0; i <= N; i++) {
          const double vol = c->G.area_m2 * dx * ((i == 0 || i == N) ? 0.5 : 1.0);
          m->density_m3[s * (N + 1) + i] = c->G.weight * ((double)Q[s * (N + 1) + i] / 16777216.0) / vol / Mst;
        }
    if (m->phi_V)
      for (int i = 0; i <= N; i++) m->phi_V[i] = ph[i] / Mst;
    return 0;
  }
};

// workgroup offsets of a 1-D batched grid: total workgroups split over the
// discharges in proportion to their weights, at least one each
void split_grid(const std::vector<double>& w, int total, int32_t* off) {
  double sum = 0;
  for (double x : w) sum += x;
  off[0] = 0;
  for (size_t i = 0; i < w.size(); i++) {
    const int g = std::max(1, (int)std::lround(total * (w[i] / std::max(sum, 1.0))));
    off[i + 1] = off[i] + g;
  }
}

// device bytes of the tables of a batch of n discharges: constants, the
// device state at both parities of the particle buffers, four offset arrays
template <class R>
constexpr size_t batch_table_bytes(int n) {
  return sizeof(Consts<R>) * (size_t)n + sizeof(Dev<R>) * 2 * (size_t)n + sizeof(int32_t) * 4 * (size_t)(n + 1);
}

// Steps of n discharges of one precision, same sort and Coulomb periods and
// same phase, as batched launches (one per kernel for all of them) on
// ctx[0]'s stream, ordered after every context's earlier work and before its
// later work.  The launches read their tables from buf (tab_cap bytes of
// device memory that no other work uses meanwhile).  Synchronising: returns
// when the steps are done, so that the next call may rewrite the tables.
template <class R>
int batch_run(pic_ctx* const* ctx, int n, int64_t steps, char* buf, size_t tab_cap, bool allow_graph) {
  pic_ctx* c0 = ctx[0];
  hipStream_t st = c0->stream;
  if (batch_table_bytes<R>(n) > tab_cap) return fail(c0, PIC_EINVAL, "batch tables exceed their buffer");
  std::vector<Impl<R>*> im((size_t)n);
  for (int i = 0; i < n; i++) im[i] = static_cast<Impl<R>*>(ctx[i]->impl);
  for (int i = 1; i < n; i++) {
    if (ctx[i]->stream == st) continue;
    HIPCHK(c0, hipEventRecord(ctx[i]->order_ev, ctx[i]->stream));
    HIPCHK(c0, hipStreamWaitEvent(st, ctx[i]->order_ev, 0));
  }
  // constants, the device state as it is now and with the two particle
  // buffers exchanged (after an odd number of sorts), grid offsets
  std::vector<Consts<R>> hc((size_t)n);
  std::vector<Dev<R>> hd(2 * (size_t)n);
  std::vector<double> w((size_t)n);
  std::vector<int32_t> off(4 * (size_t)(n + 1));
  int maxN = 0, inter_cells = 0;
  bool elds = true;
  for (int i = 0; i < n; i++) {
    hc[i] = im[i]->C;
    if (im[i]->C.inter) inter_cells = std::max(inter_cells, im[i]->C.N);
    hd[i] = im[i]->D;
    hd[n + i] = im[i]->D;
    for (int s = 0; s < 3; s++) std::swap(hd[n + i].st[s], hd[n + i].alt[s]);
    maxN = std::max(maxN, im[i]->C.N);
    elds = elds && im[i]->elds;
    const pic_geometry& G = ctx[i]->G;
    w[i] = (double)(G.n_init[0] + G.n_init[1] + G.n_init[2]) + 1.0;
  }
  const int bshape = c0->bshape;
  split_grid(w, c0->bgrid > 0 ? c0->bgrid : im[0]->grid_default_of(bshape), &off[0]);
  split_grid(w, im[0]->grid_scatter, &off[n + 1]);
  off[2 * (n + 1)] = 0;
  for (int i = 0; i < n; i++) off[2 * (n + 1) + i + 1] = off[2 * (n + 1) + i] + 3 * im[i]->C.N;
  // persistent grid over the listed Coulomb cells of all discharges: one
  // workgroup per CU (their LDS fills one)
  off[3 * (n + 1)] = 0;
  for (int i = 0; i < n; i++) off[3 * (n + 1) + i + 1] = (int32_t)(((int64_t)(i + 1) * im[0]->ncu) / n);
  const size_t bc = sizeof(Consts<R>) * n, bd = sizeof(Dev<R>) * 2 * n, bo = sizeof(int32_t) * off.size();
  HIPCHK(c0, hipMemcpyAsync(buf, hc.data(), bc, hipMemcpyHostToDevice, st));
  HIPCHK(c0, hipMemcpyAsync(buf + bc, hd.data(), bd, hipMemcpyHostToDevice, st));
  HIPCHK(c0, hipMemcpyAsync(buf + bc + bd, off.data(), bo, hipMemcpyHostToDevice, st));
  const Consts<R>* dC = (const Consts<R>*)buf;
  const Dev<R>* dD[2] = {(const Dev<R>*)(buf + bc), (const Dev<R>*)(buf + bc) + n};
  const int32_t* doff = (const int32_t*)(buf + bc + bd);
  BatchGrids g;
  g.push = doff;
  g.scat = doff + (n + 1);
  g.coul = doff + 2 * (n + 1);
  g.big = doff + 3 * (n + 1);
  g.n_push = off[n];
  g.n_scat = off[(n + 1) + n];
  g.n_coul = off[2 * (n + 1) + n];
  g.n_big = off[3 * (n + 1) + n];
  const int per = (maxN + 1 + FIELD_TPB - 1) / FIELD_TPB;
  const int sort_every = c0->G.sort_every, ce = c0->G.coulomb_every;
  // every context stands at the same phase of the launch sequence: the first
  // one's step count decides the sorts and Coulomb passes for all
  int64_t nstep = im[0]->nstep;
  int par = 0;
  int rc = 0;
  auto one_step = [&]() -> hipError_t {
    hipError_t e = launch_push_b<R>(dC, dD[par], n, g, elds, bshape, st);
    nstep++;
    const bool sort_now = nstep % sort_every == 0;
    // without a sort the node charge is formed by many workgroups first
    if (e == hipSuccess && !sort_now) e = launch_charge_b<R>(dC, dD[par], n, maxN, st);
    if (e == hipSuccess) e = launch_tail_b<R>(dC, dD[par], n, per, true, sort_now ? 0 : 2, st);
    if (sort_now && e == hipSuccess) {
      e = launch_sort_b<R>(dC, dD[par], n, g, st);
      par ^= 1;
      if (e == hipSuccess && ce > 0 && nstep % ce == 0) e = launch_coulomb_b<R>(dC, dD[par], n, g, inter_cells, st);
      if (e == hipSuccess) e = launch_tail_b<R>(dC, dD[par], n, per, false, 1, st);
    }
    return e;
  };
  // With graph replay on for the leading context, whole periods of the launch
  // sequence (it repeats every P steps with the same arguments, and an even
  // number of sorts returns the buffers) run as one captured graph.  The
  // capture is kept with what it depends on (the tables' bytes and address)
  // and reused by later calls for the same batch.
  const int64_t P = im[0]->chunk_period();
  const bool use_graph = allow_graph && im[0]->graphs_on();
  std::vector<char> sig;
  if (use_graph) {
    auto put = [&](const void* p, size_t b) { sig.insert(sig.end(), (const char*)p, (const char*)p + b); };
    put(&buf, sizeof(buf));
    put(&n, sizeof(n));
    put(&bshape, sizeof(bshape));
    put(hc.data(), bc);
    put(hd.data(), bd);
    put(off.data(), bo);
  }
  for (int64_t k = 0; k < steps && !rc;) {
    if (use_graph && nstep % P == 0 && steps - k >= P) {
      // the capture also depends on which of the two device-state tables the
      // period starts from
      sig.push_back((char)par);
      const bool same = c0->bgraph && c0->bsig == sig;
      sig.pop_back();
      if (!same) {
        if (c0->bgraph) (void)hipGraphExecDestroy(c0->bgraph);
        c0->bgraph = nullptr;
        c0->bsig.clear();
        hipGraph_t gr = nullptr;
        const int64_t n0 = nstep;
        const int par0 = par;
        HIPCHK(c0, hipStreamBeginCapture(st, hipStreamCaptureModeThreadLocal));
        hipError_t e = hipSuccess;
        for (int64_t q = 0; q < P && e == hipSuccess; q++) e = one_step();
        const hipError_t ee = hipStreamEndCapture(st, &gr);
        nstep = n0;
        if (e != hipSuccess || ee != hipSuccess || par != par0) {
          if (gr) (void)hipGraphDestroy(gr);
          rc = fail(c0, PIC_EDEVICE, std::string("batched capture: ") + hipGetErrorString(e != hipSuccess ? e : ee));
          break;
        }
        const hipError_t ei = hipGraphInstantiate(&c0->bgraph, gr, nullptr, nullptr, 0);
        (void)hipGraphDestroy(gr);
        if (ei != hipSuccess) {
          c0->bgraph = nullptr;
          rc = fail(c0, PIC_EDEVICE, std::string("hipGraphInstantiate: ") + hipGetErrorString(ei));
          break;
        }
        c0->bsig = sig;
        c0->bsig.push_back((char)par);
      }
      const hipError_t e = hipGraphLaunch(c0->bgraph, st);
      if (e != hipSuccess) rc = fail(c0, PIC_EDEVICE, std::string("batched graph: ") + hipGetErrorString(e));
      nstep += P;
      k += P;
      continue;
    }
    const hipError_t e = one_step();
    if (e != hipSuccess) rc = fail(c0, PIC_EDEVICE, std::string("batched launch: ") + hipGetErrorString(e));
    k++;
  }
  // every context stands where its own steps would have left it
  for (int i = 0; i < n; i++) {
    im[i]->nstep += steps;
    if (par)
      for (int s = 0; s < 3; s++) std::swap(im[i]->D.st[s], im[i]->D.alt[s]);
  }
  const hipError_t es = hipStreamSynchronize(st);
  if (rc) return rc;
  if (es != hipSuccess) return fail(c0, PIC_EDEVICE, std::string("batch: ") + hipGetErrorString(es));
  return 0;
}

// the batched launches apply when every context has the same precision and
// periods, stands at the same phase of the step sequence, lives on the same
// device and is not timing
bool batch_compatible(pic_ctx* const* ctx, int n) {
  if (n < 1 || n > BATCH_MAX) return false;
  const pic_geometry& G0 = ctx[0]->G;
  for (int i = 0; i < n; i++) {
    const pic_geometry& G = ctx[i]->G;
    if (G.precision != G0.precision || G.sort_every != G0.sort_every || G.coulomb_every != G0.coulomb_every)
      return false;
    // the per-cell collision list runs per discharge
    if (ctx[i]->gas.dsmc) return false;
    // the launch sequence is decided once for the batch: every context must
    // stand at the same phase of it (the steps themselves may differ)
    const int64_t P = ctx[0]->impl->chunk_period();
    if (ctx[i]->timing || ctx[i]->impl->steps_done() % P != ctx[0]->impl->steps_done() % P) return false;
    if (ctx[i]->dev != ctx[0]->dev) return false;
    for (int j = 0; j < i; j++)
      if (ctx[j] == ctx[i]) return false;
  }
  return true;
}

// more than one discharge: one launch per kernel pays off
bool batchable(pic_ctx* const* ctx, int n) { return n >= 2 && batch_compatible(ctx, n); }

// the resident table buffer of the batches led by c, grown to at least bytes
int batch_tables(pic_ctx* c, size_t bytes, char** out) {
  if (c->btab_bytes < bytes) {
    HIPCHK(c, hipStreamSynchronize(c->stream));
    if (c->btab) (void)hipFree(c->btab);
    c->btab = nullptr;
    c->btab_bytes = 0;
    const size_t want = std::max<size_t>(bytes + bytes / 2, 64 * 1024);
    void* p = nullptr;
    const hipError_t e = hipMalloc(&p, want);
    if (e != hipSuccess) return fail(c, PIC_ENOMEM, "hipMalloc of the batch tables failed");
    c->btab = (char*)p;
    c->btab_bytes = want;
  }
  *out = c->btab;
  return 0;
}

// ---------------------------------------------------------------------------
// Tables of pic_step_batch_static: a fixed device array instead of library
// allocations.  In host code `scratch` names a host-side stand-in; its device
// address on each GPU comes from hipGetSymbolAddress, taken once per device
// when the first context is created there, and only that address is used.
// ---------------------------------------------------------------------------
constexpr size_t SCRATCH_BYTES = std::max(batch_table_bytes<float>(PIC_BATCH_STATIC_MAX),
                                          batch_table_bytes<double>(PIC_BATCH_STATIC_MAX));
static __device__ __align__(256) char scratch[SCRATCH_BYTES];

std::mutex scratch_mu;
std::vector<char*> scratch_dev;  // device address of scratch per HIP device (null: not taken yet)

// with device dev current
hipError_t scratch_setup(int dev) {
  std::lock_guard<std::mutex> lock(scratch_mu);
  if ((int)scratch_dev.size() <= dev) scratch_dev.resize((size_t)dev + 1, nullptr);
  if (scratch_dev[dev]) return hipSuccess;
  void* p = nullptr;
  const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
  if (e == hipSuccess) scratch_dev[dev] = (char*)p;
  return e;
}

char* scratch_of(int dev) {
  std::lock_guard<std::mutex> lock(scratch_mu);
  return dev < (int)scratch_dev.size() ? scratch_dev[dev] : nullptr;
}

}  // namespace

extern "C" {

int pic_create(const pic_geometry* g, const pic_gas* gas, double voltage_V, double frequency_Hz, double pressure_Pa,
               pic_ctx** out) {
  if (!out) return PIC_EINVAL;
  *out = nullptr;
  if (!g || !gas || !gas->sigma_m2 || !gas->threshold_eV || !gas->loss_eV) return PIC_EINVAL;
  if (g->n_cells < 4 || g->n_cells > NMAX_CELLS || !(g->gap_m > 0) || !(g->area_m2 > 0) || !(g->weight > 0) ||
      g->steps_per_period < 1 || g->ion_subcycle < 1 || g->sort_every < 1 || !(frequency_Hz > 0) ||
      !(pressure_Pa >= 0) || !(gas->T_gas_K > 0) || g->precision < 0 || g->precision > 1 || g->eedf_bins < 0 ||
      g->eedf_bins > EEDF_MAX || g->fneg_xbins < 0 || g->fneg_ebins < 0 ||
      (int64_t)g->fneg_xbins * g->fneg_ebins > FNEG_MAX || (g->eedf_bins > 0 && !(g->eedf_emax_eV > 0)) ||
      (g->fneg_ebins > 0 && !(g->fneg_emax_eV > 0)) || g->coulomb_every < 0 ||
      (g->coulomb_every > 0 && (g->coulomb_every % g->sort_every != 0 || !(gas->coulomb_log > 0))) ||
      gas->coulomb_inter < 0 || gas->coulomb_inter > 1 || gas->dsmc < 0 || gas->dsmc > 1 ||
      (gas->dsmc && g->sort_every % g->ion_subcycle != 0))
    return PIC_EINVAL;
  for (int s = 0; s < 3; s++)
    if (g->n_init[s] < 0 || g->n_init[s] > ((int64_t)1 << 30) - 65536 || g->T_init_eV[s] < 0) return PIC_EINVAL;
  if (g->n_init[0] + g->n_init[1] + g->n_init[2] > (int64_t)(ID_MASK)) return PIC_EINVAL;
  pic_ctx* c = new pic_ctx();
  c->G = *g;
  c->gas = *gas;
  c->sigma.assign(gas->sigma_m2, gas->sigma_m2 + (size_t)NCH * NPT);
  c->thr.assign(gas->threshold_eV, gas->threshold_eV + NCH);
  c->loss.assign(gas->loss_eV, gas->loss_eV + NCH);
  c->gas.sigma_m2 = c->sigma.data();
  c->gas.threshold_eV = c->thr.data();
  c->gas.loss_eV = c->loss.data();
  c->U_rf = voltage_V;
  c->freq = frequency_Hz;
  c->pres = pressure_Pa;
  for (int j = 0; j < NCH; j++)
    if (c->thr[j] < c->loss[j]) {
      delete c;
      return PIC_EINVAL;
    }
  hipError_t e = hipGetDevice(&c->dev);
  if (e == hipSuccess) e = scratch_setup(c->dev);
  if (e == hipSuccess) e = hipEventCreateWithFlags(&c->order_ev, hipEventDisableTiming);
  if (e != hipSuccess) {
    delete c;
    return PIC_EDEVICE;
  }
  e = hipStreamCreate(&c->own);
  if (e != hipSuccess) {
    (void)hipEventDestroy(c->order_ev);
    delete c;
    return PIC_EDEVICE;
  }
  c->stream = c->own;
  if (g->precision == PIC_FP64) c->impl = new Impl<double>(c);
  else c->impl = new Impl<float>(c);
  int rc = c->impl->create();
  if (rc) {
    delete c->impl;
    (void)hipStreamDestroy(c->own);
    (void)hipEventDestroy(c->order_ev);
    delete c;
    return rc;
  }
  *out = c;
  return PIC_OK;
}

int pic_set_stream(pic_ctx* c, void* s) {
  if (!c) return PIC_EINVAL;
  c->stream = s ? (hipStream_t)s : c->own;
  return PIC_OK;
}

int pic_step(pic_ctx* c, int64_t n) {
  if (!c || n < 0) return PIC_EINVAL;
  if (c->err) return c->err;
  return c->impl->step(n);
}

int pic_sync(pic_ctx* c) {
  if (!c) return PIC_EINVAL;
  if (c->err) return c->err;
  int32_t e;
  return c->impl->read_err(&e);
}

int pic_moments(pic_ctx* c, pic_moments_t* m) {
  if (!c || !m) return PIC_EINVAL;
  if (c->err) return c->err;
  int rc = c->impl->moments(m);
  if (rc) return rc;
  return pic_sync(c);
}

int pic_particles(pic_ctx* c, int sp, int64_t cap, uint64_t* id, int32_t* cell, double* off, double* v,
                  int64_t* n_out) {
  if (!c || sp < 0 || sp > 2 || cap < 0 || !n_out) return PIC_EINVAL;
  if (c->err) return c->err;
  return c->impl->particles(sp, cap, id, cell, off, v, n_out);
}

int pic_field(pic_ctx* c, double* phi, double* E) {
  if (!c) return PIC_EINVAL;
  if (c->err) return c->err;
  return c->impl->field(phi, E);
}

int pic_charge(pic_ctx* c, int64_t* Q) {
  if (!c || !Q) return PIC_EINVAL;
  if (c->err) return c->err;
  return c->impl->charge(Q);
}

int pic_timing(pic_ctx* c, int enable) {
  if (!c) return PIC_EINVAL;
  if (enable < 0) return reject(c, "pic_timing: enable must be 0 (off) or a stride >= 1");
  if (enable) {
    c->timed_ms = 0;
    c->timed_launches = 0;
    c->ev_used = 0;
    c->time_every = enable;
    c->time_count = 0;
  }
  c->timing = enable != 0;
  return PIC_OK;
}

int pic_kernel_time(pic_ctx* c, double* ms, int64_t* launches) {
  if (!c || !ms || !launches) return PIC_EINVAL;
  hipError_t e = hipStreamSynchronize(c->stream);
  if (e != hipSuccess) return fail(c, PIC_EDEVICE, hipGetErrorString(e));
  for (size_t i = 0; i < c->ev_used; i++) {
    float t = 0;
    e = hipEventElapsedTime(&t, c->events[i].first, c->events[i].second);
    if (e != hipSuccess) return fail(c, PIC_EDEVICE, hipGetErrorString(e));
    c->timed_ms += t;
    c->timed_launches++;
  }
  c->ev_used = 0;
  *ms = c->timed_ms;
  *launches = c->timed_launches;
  return PIC_OK;
}

int pic_set_graphs(pic_ctx* c, int enable) {
  if (!c) return PIC_EINVAL;
  if (c->err) return c->err;
  return c->impl->set_graphs(enable);
}

int pic_step_batch(pic_ctx* const* ctx, int n, int64_t steps) {
  if (!ctx || n < 0 || steps < 0) return PIC_EINVAL;
  for (int i = 0; i < n; i++) {
    if (!ctx[i]) return PIC_EINVAL;
    if (ctx[i]->err) return ctx[i]->err;
  }
  if (steps > 0 && batchable(ctx, n)) {
    const bool f64 = ctx[0]->G.precision == PIC_FP64;
    const size_t bytes = f64 ? batch_table_bytes<double>(n) : batch_table_bytes<float>(n);
    char* buf = nullptr;
    const int rc = batch_tables(ctx[0], bytes, &buf);
    if (rc) return rc;
    return f64 ? batch_run<double>(ctx, n, steps, buf, ctx[0]->btab_bytes, true)
               : batch_run<float>(ctx, n, steps, buf, ctx[0]->btab_bytes, true);
  }
  // otherwise round robin in chunks of each context's period, so that every
  // stream holds queued work while the others run.  With Coulomb collisions
  // on in any of them the chunks are chained by events into one sequence:
  // large discharges whose Coulomb kernels ran at the same time on two
  // streams have ended in different states, for a reason not found, so their
  // steps are not allowed to overlap.
  bool chain = false;
  for (int i = 0; i < n; i++) chain = chain || ctx[i]->G.coulomb_every > 0;
  hipEvent_t ev = nullptr;
  if (chain && steps > 0 && n > 1) {
    const hipError_t e = hipEventCreateWithFlags(&ev, hipEventDisableTiming);
    if (e != hipSuccess) return fail(ctx[0], PIC_EDEVICE, std::string("hipEventCreate: ") + hipGetErrorString(e));
  }
  hipStream_t prev = nullptr;
  int rc = PIC_OK;
  std::vector<int64_t> left((size_t)n, steps);
  for (bool more = steps > 0; more && !rc;) {
    more = false;
    for (int i = 0; i < n && !rc; i++) {
      if (left[i] == 0) continue;
      if (ev && prev && prev != ctx[i]->stream) {
        hipError_t e = hipEventRecord(ev, prev);
        if (e == hipSuccess) e = hipStreamWaitEvent(ctx[i]->stream, ev, 0);
        if (e != hipSuccess) {
          rc = fail(ctx[i], PIC_EDEVICE, std::string("stream ordering: ") + hipGetErrorString(e));
          break;
        }
      }
      const int64_t k = std::min(left[i], ctx[i]->impl->chunk());
      rc = ctx[i]->impl->step(k);
      prev = ctx[i]->stream;
      left[i] -= k;
      more = more || left[i] > 0;
    }
  }
  if (ev) (void)hipEventDestroy(ev);
  return rc;
}

int pic_step_batch_static(pic_ctx* const* ctx, int n, int64_t steps) {
  if (!ctx || n < 1 || steps < 0) return PIC_EINVAL;
  for (int i = 0; i < n; i++) {
    if (!ctx[i]) return PIC_EINVAL;
    if (ctx[i]->err) return ctx[i]->err;
  }
  if (n > PIC_BATCH_STATIC_MAX)
    return reject(ctx[0], "pic_step_batch_static: " + std::to_string(n) + " discharges, at most " +
                              std::to_string(PIC_BATCH_STATIC_MAX));
  if (!batch_compatible(ctx, n))
    return reject(ctx[0],
                  "pic_step_batch_static: the discharges differ in precision, periods, phase or device, repeat, "
                  "or one is timing");
  if (steps == 0) return PIC_OK;
  char* buf = scratch_of(ctx[0]->dev);
  if (!buf) return fail(ctx[0], PIC_EDEVICE, "pic_step_batch_static: no device address of the static tables");
  return ctx[0]->G.precision == PIC_FP64 ? batch_run<double>(ctx, n, steps, buf, SCRATCH_BYTES, false)
                                         : batch_run<float>(ctx, n, steps, buf, SCRATCH_BYTES, false);
}

int pic_autotune(pic_ctx* c, int64_t steps_per_trial, int32_t* chosen) {
  if (!c || steps_per_trial <= 0) return PIC_EINVAL;
  if (c->err) return c->err;
  return c->impl->autotune(steps_per_trial, chosen);
}

int pic_set_shape(pic_ctx* c, int32_t tpb, int32_t ppt) {
  if (!c) return PIC_EINVAL;
  for (int sh = 0; sh < SHAPES; sh++)
    if (SHAPE_TPB[sh] == tpb && SHAPE_PPT[sh] == ppt) return c->impl->set_shape(sh);
  return reject(c, "pic_set_shape: " + std::to_string(tpb) + " x " + std::to_string(ppt) + " is not a shape built");
}

int pic_launch_shape(pic_ctx* c, int32_t* tpb, int32_t* ppt, int32_t* workgroups) {
  if (!c) return PIC_EINVAL;
  int32_t sh = 0, g = 0;
  c->impl->launch_shape(&sh, &g);
  if (tpb) *tpb = SHAPE_TPB[sh];
  if (ppt) *ppt = SHAPE_PPT[sh];
  if (workgroups) *workgroups = g;
  return PIC_OK;
}

int pic_autotune_batch(pic_ctx* const* ctx, int n, int64_t steps_per_trial, int32_t* tpb, int32_t* ppt,
                       int32_t* workgroups) {
  if (!ctx || n < 1 || steps_per_trial <= 0) return PIC_EINVAL;
  for (int i = 0; i < n; i++) {
    if (!ctx[i]) return PIC_EINVAL;
    if (ctx[i]->err) return ctx[i]->err;
  }
  if (!batch_compatible(ctx, n)) return reject(ctx[0], "pic_autotune_batch: the discharges cannot be batched");
  pic_ctx* c0 = ctx[0];
  const bool f64 = c0->G.precision == PIC_FP64;
  char* buf = nullptr;
  int rc = batch_tables(c0, f64 ? batch_table_bytes<double>(n) : batch_table_bytes<float>(n), &buf);
  if (rc) return rc;
  std::vector<std::pair<int, int>> cand;
  for (int sh = 0; sh < SHAPES; sh++) {
    const int d = c0->impl->grid_default_of(sh);
    cand.push_back({sh, d});
    cand.push_back({sh, std::max(1, (3 * d) / 4)});
  }
  hipEvent_t e0, e1;
  HIPCHK(c0, hipEventCreate(&e0));
  HIPCHK(c0, hipEventCreate(&e1));
  std::pair<int, int> best = cand[0];
  float tbest = 3e38f;
  for (const auto& sg : cand) {
    c0->bshape = sg.first;
    c0->bgrid = sg.second;
    (void)hipEventRecord(e0, c0->stream);
    rc = f64 ? batch_run<double>(ctx, n, steps_per_trial, buf, c0->btab_bytes, false)
             : batch_run<float>(ctx, n, steps_per_trial, buf, c0->btab_bytes, false);
    if (rc) break;
    (void)hipEventRecord(e1, c0->stream);
    (void)hipEventSynchronize(e1);
    float ms = 0;
    (void)hipEventElapsedTime(&ms, e0, e1);
    if (ms < tbest) {
      tbest = ms;
      best = sg;
    }
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  if (rc) return rc;
  c0->bshape = best.first;
  c0->bgrid = best.second;
  if (tpb) *tpb = SHAPE_TPB[best.first];
  if (ppt) *ppt = SHAPE_PPT[best.first];
  if (workgroups) *workgroups = best.second;
  return PIC_OK;
}

int pic_set_grid(pic_ctx* c, int32_t g) {
  if (!c || g < 0) return PIC_EINVAL;
  c->impl->set_grid(g);
  return PIC_OK;
}

int pic_destroy(pic_ctx* c) {
  if (!c) return PIC_EINVAL;
  (void)hipStreamSynchronize(c->stream);
  if (c->bgraph) (void)hipGraphExecDestroy(c->bgraph);
  if (c->btab) (void)hipFree(c->btab);
  if (c->order_ev) (void)hipEventDestroy(c->order_ev);
  delete c->impl;
  for (auto& p : c->events) {
    (void)hipEventDestroy(p.first);
    (void)hipEventDestroy(p.second);
  }
  if (c->own) (void)hipStreamDestroy(c->own);
  delete c;
  return PIC_OK;
}

const char* pic_last_error(const pic_ctx* c) {
  if (!c) return "null context";
  return c->msg.c_str();
}

}  // extern "C"
