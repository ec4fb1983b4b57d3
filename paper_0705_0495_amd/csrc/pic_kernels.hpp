// Device code of the gfx950 PIC-MCC step for the oxygen rf discharge
// (Bronold et al., Sec. II-III).  Included once by pic.hip.
//
// Layout in HBM (per species, structure of arrays):
//   cell  int32   cell index, DEAD for removed particles
//   off   R       position inside the cell, [0, 1)   (x = (cell + off) dx)
//   vx, vy, vz R  velocity, m/s (leapfrog: vx at half steps)
//   id    uint64  particle identity, key of its random streams
// The field moves only vx and the position, so a particle that does not
// collide reads cell/off/vx/id and writes cell/off/vx: 20 + 12 bytes (FP32).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace pic {

constexpr int NCH = 19;
constexpr int NPT = 897;
constexpr int TS = 20;                 // table row stride: sig[k * TS + channel]
constexpr int32_t DEAD = INT32_MIN;
// Launch shape of the fused particle kernel: TPB threads per workgroup, PPT
// consecutive particles per thread (a multiple of 4: 16-byte vectors); a tile
// is TPB * PPT consecutive particles, a wave's part of it WTILE.  The
// autotuner chooses among the shapes built (SHAPES); results do not depend on
// the shape.
template <int TPB_, int PPT_>
struct Shape {
  static constexpr int TPB = TPB_, PPT = PPT_, TILE = TPB_ * PPT_, WTILE = 64 * PPT_, NW = TPB_ / 64;
};
using Shape0 = Shape<256, 4>;
using Shape1 = Shape<512, 4>;
using Shape2 = Shape<256, 8>;
constexpr int SHAPES = 3;
constexpr int SHAPE_TPB[SHAPES] = {256, 512, 256}, SHAPE_PPT[SHAPES] = {4, 4, 8};
constexpr int TILE_MAX = 2048;         // the largest tile of the shapes built
constexpr int WTILE_MIN = 256;         // the smallest wave part
constexpr int WIN = 512;               // cells of the LDS deposit window
constexpr int EEDF_MAX = 256;
constexpr int FNEG_MAX = 2048;
constexpr int REQ_CAP = 4096;          // partner requests per step
constexpr int NBUCKET_BITS = 14;       // births are bucketed by the top bits of the creator id
constexpr int NBUCKET = 1 << NBUCKET_BITS;
constexpr uint64_t ID_MASK = (1ull << 40) - 1;
constexpr uint64_t F_MASK = (1ull << 40) - 1;
constexpr double TWO_PI = 6.283185307179586;

enum : int32_t { ERR_PMAX = 1, ERR_CAP = 2, ERR_NB = 4, ERR_REQ = 8, ERR_ID = 16, ERR_NAN = 32, ERR_SORT = 64,
                    ERR_COUL = 128 };

// constants of one discharge (computed once on the host, rounded once to R)
template <class R>
struct Consts {
  int32_t N, cmid, M, nsub;
  uint32_t seed_lo, seed_hi;
  R qmdt[3], dtdx[3], hk[3], vth0[3];
  R a_g[3], b_g[3], hmu_g[3], c2e_g[3];
  R vthg;
  R a_c[3], b_c[3], hmu_c[3], c2e_c[3], Mr_c[3];   // partner channels 12, 13, 17
  double KP[3];        // tau M_j W / (A dx): Eq. (1) slot per partner particle of the cell
  R ddf, adf, hme, hmn;
  R thr[NCH], loss[NCH];
  double PG[NCH];
  double PGtot[3];
  double cphi, cE, invdx, inv2dx;
  int32_t eedf_bins, fneg_xbins, fneg_ebins, inter;  // inter: unlike-species Coulomb collisions on
  R eedf_sc, fneg_sc, fneg_em;
  R ccoul[3], ccoul_h[3];   // Eq. (2) prefactor per particle in the cell: full and half interval
  R cinter[3], finter[3][2];  // unlike pairs (e,O-), (e,O2+), (O-,O2+): Eq. (2) with the reduced mass, mu/m_a, mu/m_b
  R sinc[10], cosc[11], logc[12], ln2, sqrt2;  // series of the samplers' elementary functions
  // compact copy of each species' gas channels for LDS: channel j keeps nodes
  // [tab_k0[j], NPT) (the nodes below are zero) at tab_off[j]; tab_n[s]
  // values for species s, 0 when they do not fit (then read from global)
  int32_t tab_k0[NCH], tab_off[NCH], tab_n[3];
  int32_t tab_base[3];  // where species s's compact copy starts in Dev::sigc (a multiple of 4)
};

// terms of the elementary-function series per precision
template <class R> struct Series;
template <> struct Series<float> { static constexpr int NS = 6, NC = 7, NL = 6; };
template <> struct Series<double> { static constexpr int NS = 10, NC = 11, NL = 12; };

struct Counters {
  int64_t step, next_id;
  int64_t events[NCH];
  int64_t absorbed[6];   // [electrode][species]
  int64_t psteps, births, cycles, tophits, nreq, nacc;
  int64_t step_push;     // the step the last push advanced (read by the step's end)
  int32_t err, pad;
};

// a workgroup's place in the grid of one discharge: its index and the
// number of workgroups working on that discharge
struct Blk {
  int x, n;
};

// in a batched launch over a 1-D grid, discharge i owns workgroups
// [off[i], off[i + 1]); returns i and the workgroup's place within it
__device__ __forceinline__ int batch_block(const int32_t* off, int nd, Blk& b) {
  int lo = 0, hi = nd;
  while (hi - lo > 1) {
    const int mid = (lo + hi) >> 1;
    if (off[mid] <= (int)blockIdx.x) lo = mid;
    else hi = mid;
  }
  b.x = (int)blockIdx.x - off[lo];
  b.n = off[lo + 1] - off[lo];
  return lo;
}

template <class R>
struct Birth {
  int32_t sp, idx, k, cell;
  uint64_t creator;
  R off, v0, v1, v2;
};

// a candidate of the null-collision test in the state the push leaves it in
template <class R>
struct Cand {
  int32_t slot, cell;
  R off, vx;
  uint64_t id;
};

template <class R>
struct Request {
  int32_t sp, chan, slot, cell;
  uint64_t id;
  R u_acc;
  int32_t partner, acc;
};

template <class R>
struct Store {
  int32_t* cell;
  R* off;
  R* vx;
  R* vyz;  // (vy, vz) interleaved: one 8- or 16-byte access per particle
  uint64_t* id;
};

template <class R> struct Pair2;
template <> struct Pair2<float> { using T = float2; };
template <> struct Pair2<double> { using T = double2; };

template <class R>
__device__ __forceinline__ void ld_yz(const Store<R>& s, int64_t i, R& y, R& z) {
  const typename Pair2<R>::T p = *(const typename Pair2<R>::T*)(s.vyz + 2 * i);
  y = p.x;
  z = p.y;
}
template <class R>
__device__ __forceinline__ void st_yz(const Store<R>& s, int64_t i, R y, R z) {
  typename Pair2<R>::T p;
  p.x = y;
  p.y = z;
  *(typename Pair2<R>::T*)(s.vyz + 2 * i) = p;
}

template <class R>
struct Dev {
  Store<R> st[3];
  Store<R> alt[3];
  int64_t* N;       // [3] store lengths (including dead slots until the next sort)
  int64_t* Nnew;    // [3]
  int64_t cap[3];
  int32_t* cnt;     // [3][Nc]    particles per cell
  int64_t* F;       // [3][Nc]    sum of the 24-bit fractional positions per cell
  int32_t* seg;     // [3][Nc+1]  cell segments of the last sort
  int32_t* cursor;  // [3][Nc]
  int32_t* segmax;  // [3]
  R* E2;            // [Nc][2]    (E_c, E_c+1)
  double* phi;      // [Nc+1]
  double* E;        // [Nc+1]
  const double* U;  // [M]
  const R* sig;     // [NPT][TS]
  const R* sigc;    // compact gas-channel copies per species (Consts::tab_*), staged into LDS
  Birth<R>* nb;
  int32_t nb_cap, req_cap;
  int32_t* nbc;     // [4] total, per species
  int32_t* bhist;   // [NBUCKET] births per creator-id bucket
  int32_t* perm;    // [nb_cap] births grouped by bucket
  Cand<R>* cand[3]; // candidates of the null-collision test: tile t of species s
                    // writes them to cand[s][t*TILE ...], wave w of the
                    // tile to cand[s][t*TILE + w*WTILE ...], count in tcnt[s][t*TILE/WTILE + w]
                    // (TILE, WTILE of the launch shape)
  int32_t* tcnt[3]; // candidates per tile
  int32_t* ncand;   // [3] (unused)
  Request<R>* req;
  int32_t* nreq;
  Counters* ctr;
  int64_t* Qcur;    // [3][Nc+1] node charge of the population the next push starts from
  int64_t* Qacc;
  int64_t* Qlast;
  int64_t* qnet;    // [Nc+1] net node charge of the step (k_charge), read by the field solve
  double* phiacc;
  double* philast;
  int64_t* eedf_acc;
  int64_t* eedf_last;
  int64_t* fneg_acc;
  int64_t* fneg_last;
  uint32_t* done;   // [4] last-workgroup counters
  int32_t* ncoul;   // cells above CoulCap<R>::M particles in this Coulomb pass
  int32_t* coul_big;  // [3 Nc] their (species, cell) indices
  int32_t* ncl;     // cells listed for the largest LDS class in this pass
  int32_t* clist;   // [3 Nc] their (species, cell) indices
  Request<R>* lreq; // accepted requests of one partner type of the per-cell collision list
  int32_t lreq_cap;
};

// ---------------------------------------------------------------------------
// random numbers: Philox4x32-10 (Salmon et al., SC'11)
// ---------------------------------------------------------------------------
__device__ __forceinline__ uint4 philox(uint32_t x0, uint32_t x1, uint32_t x2, uint32_t x3, uint32_t k0,
                                        uint32_t k1) {
#pragma unroll
  for (int r = 0; r < 10; r++) {
    uint64_t p0 = (uint64_t)0xD2511F53u * x0;
    uint64_t p1 = (uint64_t)0xCD9E8D57u * x2;
    uint32_t y0 = (uint32_t)(p1 >> 32) ^ x1 ^ k0;
    uint32_t y2 = (uint32_t)(p0 >> 32) ^ x3 ^ k1;
    x1 = (uint32_t)p1;
    x3 = (uint32_t)p0;
    x0 = y0;
    x2 = y2;
    k0 += 0x9E3779B9u;
    k1 += 0xBB67AE85u;
  }
  return make_uint4(x0, x1, x2, x3);
}

template <class R>
__device__ __forceinline__ uint4 rng(const Consts<R>& C, uint64_t id, uint32_t n, uint32_t k) {
  return philox((uint32_t)id, (uint32_t)(id >> 32), n, k, C.seed_lo, C.seed_hi);
}

template <class R> __device__ __forceinline__ R unif(uint32_t w);
template <> __device__ __forceinline__ float unif<float>(uint32_t w) {
  return ((float)(w >> 9) + 0.5f) * 0x1p-23f;
}
template <> __device__ __forceinline__ double unif<double>(uint32_t w) { return ((double)w + 0.5) * 0x1p-32; }

__device__ __forceinline__ double unif52(uint32_t a, uint32_t b) {
  uint64_t m = ((uint64_t)a << 20) | (uint64_t)(b >> 12);
  return ((double)m + 0.5) * 0x1p-52;
}

__device__ __forceinline__ float Sqrt(float x) { return sqrtf(x); }
__device__ __forceinline__ double Sqrt(double x) { return sqrt(x); }
__device__ __forceinline__ float Floor(float x) { return floorf(x); }
__device__ __forceinline__ double Floor(double x) { return floor(x); }

// samplers: fixed-term series evaluated in R (no library transcendentals)
// sin and cos of 2 pi u for u in (0,1): u = (k + f)/4 with |f| <= 1/2, Taylor
// series of sin(pi f/2) and cos(pi f/2) in f with a fixed number of terms in
// Horner order, then the quadrant k.  ln u for u > 0: u = m 2^e with m in
// [1/sqrt2, sqrt2), ln m = 2 atanh(s) = 2 s (1 + s^2/3 + s^4/5 + ...),
// s = (m-1)/(m+1).  The coefficients are formed on the host in double and
// rounded once (Consts::sinc, cosc, logc).
template <class R>
__device__ __forceinline__ void sincos2pi(const Consts<R>& C, R u, R& sn, R& cs) {
  const R x = u * (R)4;
  int k = (int)x;
  R f = x - (R)k;
  if (f > (R)0.5) {
    f = f - (R)1;
    k = k + 1;
  }
  const R z = f * f;
  R ps = C.sinc[Series<R>::NS - 1];
#pragma unroll
  for (int j = Series<R>::NS - 2; j >= 0; j--) ps = ps * z + C.sinc[j];
  const R s = f * ps;
  R pc = C.cosc[Series<R>::NC - 1];
#pragma unroll
  for (int j = Series<R>::NC - 2; j >= 0; j--) pc = pc * z + C.cosc[j];
  switch (k & 3) {
    case 0: sn = s; cs = pc; break;
    case 1: sn = pc; cs = -s; break;
    case 2: sn = -s; cs = -pc; break;
    default: sn = -pc; cs = s; break;
  }
}

__device__ __forceinline__ void split_exp(float u, float& m, int& e) {
  const uint32_t b = __float_as_uint(u);
  e = (int)((b >> 23) & 0xFFu) - 127;
  m = __uint_as_float((b & 0x7FFFFFu) | 0x3F800000u);
}
__device__ __forceinline__ void split_exp(double u, double& m, int& e) {
  const uint64_t b = (uint64_t)__double_as_longlong(u);
  e = (int)((b >> 52) & 0x7FFull) - 1023;
  m = __longlong_as_double((long long)((b & 0xFFFFFFFFFFFFFull) | 0x3FF0000000000000ull));
}

template <class R>
__device__ __forceinline__ R plog(const Consts<R>& C, R u) {
  R m;
  int e;
  split_exp(u, m, e);
  if (m > C.sqrt2) {
    m = m * (R)0.5;
    e = e + 1;
  }
  const R s = (m - (R)1) / (m + (R)1);
  const R z = s * s;
  R p = C.logc[Series<R>::NL - 1];
#pragma unroll
  for (int k = Series<R>::NL - 2; k >= 0; k--) p = p * z + C.logc[k];
  return (R)e * C.ln2 + (s + s) * p;
}

template <class R> __device__ __forceinline__ R bm_radius(const Consts<R>& C, R u) {
  return Sqrt((R)-2 * plog<R>(C, u));
}
template <class R> __device__ __forceinline__ R cos2pi(const Consts<R>& C, R u) {
  R s, c;
  sincos2pi<R>(C, u, s, c);
  return c;
}
template <class R> __device__ __forceinline__ R sin2pi(const Consts<R>& C, R u) {
  R s, c;
  sincos2pi<R>(C, u, s, c);
  return s;
}

template <class R>
__device__ __forceinline__ void iso_dir(const Consts<R>& C, uint32_t wc, uint32_t wp, R n[3]) {
  R u = unif<R>(wc);
  R ct = (R)1 - (R)2 * u;
  R st = Sqrt((R)1 - ct * ct);
  R up = unif<R>(wp);
  R sp, cp;
  sincos2pi<R>(C, up, sp, cp);
  n[0] = st * cp;
  n[1] = st * sp;
  n[2] = ct;
}

// ---------------------------------------------------------------------------
// cross-section tables: binade grid, index and weight from the bits of E
// ---------------------------------------------------------------------------
template <class R>
struct Lookup {
  int k;
  R t;
  int mode;  // 0 inside, 1 below the first node, 2 at/above the last node
};

__device__ __forceinline__ Lookup<float> lookup(float E) {
  uint32_t b = __float_as_uint(E);
  if (b < 0x38800000u) return {0, 0.0f, 1};
  if (b >= 0x46800000u) return {0, 0.0f, 2};
  return {(int)((b >> 18) - (0x38800000u >> 18)), (float)(b & 0x3FFFFu) * 0x1p-18f, 0};
}
__device__ __forceinline__ Lookup<double> lookup(double E) {
  uint64_t b = (uint64_t)__double_as_longlong(E);
  if (b < 0x3F10000000000000ull) return {0, 0.0, 1};
  if (b >= 0x40D0000000000000ull) return {0, 0.0, 2};
  return {(int)((b >> 47) - (0x3F10000000000000ull >> 47)), (double)(b & ((1ull << 47) - 1)) * 0x1p-47, 0};
}

// sigma of column j of a table with rows of `stride` values per node
template <class R>
__device__ __forceinline__ R sig_at(const R* tab, int stride, int j, const Lookup<R>& L) {
  if (L.mode == 2) return tab[(NPT - 1) * stride + j];
  R s0 = tab[L.k * stride + j];
  if (L.mode == 1) return s0;
  R s1 = tab[(L.k + 1) * stride + j];
  R d = s1 - s0;
  R p = L.t * d;
  return s0 + p;
}

// ---------------------------------------------------------------------------
// 128-bit integer to double, round to nearest even
// ---------------------------------------------------------------------------
__device__ __forceinline__ double u64_to_double_rn(uint64_t u) {
  // both halves convert exactly, the product by 2^32 is exact, the sum rounds once
  return (double)(uint32_t)(u >> 32) * 4294967296.0 + (double)(uint32_t)u;
}

__device__ inline double i128_to_double(__int128 x) {
  bool neg = x < 0;
  unsigned __int128 u = neg ? (unsigned __int128)(-x) : (unsigned __int128)x;
  uint64_t hi = (uint64_t)(u >> 64);
  double d;
  if (hi == 0) {
    d = u64_to_double_rn((uint64_t)u);
  } else {
    int p = 127 - __clzll(hi);  // position of the leading one, >= 64
    int sh = p - 63;
    uint64_t t = (uint64_t)(u >> sh);
    unsigned __int128 rest = u & (((unsigned __int128)1 << sh) - 1);
    if (rest != 0) t |= 1;  // sticky bit far below the rounding position
    d = ldexp(u64_to_double_rn(t), sh);
  }
  return neg ? -d : d;
}

// Global stores of this workgroup made visible to its other waves before
// they read them.  The workgroup barrier alone waits only for LDS: each wave
// first waits for its own vector memory operations (its stores reach the L2),
// and after the barrier the CU's vector L1 is invalidated so that the reads
// that follow come from the L2.  (A device-scope fence would also write the
// L2 back, many times dearer, and is not needed within one workgroup.)
__device__ __forceinline__ void wg_global_sync() {
  asm volatile("s_waitcnt vmcnt(0)" ::: "memory");
  __syncthreads();
  asm volatile("buffer_inv sc0" ::: "memory");
}

// ---------------------------------------------------------------------------
// helpers shared by the kernels
// ---------------------------------------------------------------------------
template <class R>
__device__ __forceinline__ int32_t frac24(R off) {
  return (int32_t)(off * (R)16777216);
}

template <class R>
__device__ __forceinline__ void deposit_global(const Dev<R>& D, int N, int sp, int cell, R off, int sign) {
  int32_t f = frac24(off);
  atomicAdd(&D.cnt[(size_t)sp * N + cell], sign);
  atomicAdd((unsigned long long*)&D.F[(size_t)sp * N + cell], (unsigned long long)(int64_t)(sign * (int64_t)f));
}

// Where a partner reaction's change of charge goes.  Without `direct` to the
// deposit counters, from which the field is formed afterwards.  With it the
// node charge of the step has already been formed from them (k_charge): the
// change goes to that node charge (per species and net, and the rf-cycle
// sums), and to the counters as well only for the ions when the next push
// does not move them (the counters then outlive the step).
struct ClaimDep {
  int direct;
  bool ion_next;  // the next push moves the ions (their counters are cleared)
};

template <class R>
__device__ __forceinline__ void deposit_claim(const Consts<R>& C, const Dev<R>& D, int sp, int cell, R off, int sign,
                                              ClaimDep dep) {
  if (!dep.direct || (sp != 0 && !dep.ion_next)) deposit_global(D, C.N, sp, cell, off, sign);
  if (!dep.direct) return;
  const int N = C.N;
  const int64_t f = frac24(off);
  const int64_t a = sign * ((int64_t(1) << 24) - f), b = sign * f;
  const int64_t qs = sp == 2 ? 1 : -1;
  const size_t o = (size_t)sp * (N + 1) + cell;
  atomicAdd((unsigned long long*)&D.Qcur[o], (unsigned long long)a);
  atomicAdd((unsigned long long*)&D.Qcur[o + 1], (unsigned long long)b);
  atomicAdd((unsigned long long*)&D.Qacc[o], (unsigned long long)a);
  atomicAdd((unsigned long long*)&D.Qacc[o + 1], (unsigned long long)b);
  atomicAdd((unsigned long long*)&D.qnet[cell], (unsigned long long)(qs * a));
  atomicAdd((unsigned long long*)&D.qnet[cell + 1], (unsigned long long)(qs * b));
}

__device__ __forceinline__ int birth_bucket(uint64_t creator, uint64_t next_id) {
  const int bits = 64 - __clzll((long long)(next_id | 1));
  const int sh = bits > NBUCKET_BITS ? bits - NBUCKET_BITS : 0;
  return (int)(creator >> sh);
}

template <class R>
__device__ void add_birth(const Consts<R>& C, const Dev<R>& D, int sp, uint64_t creator, int k, int cell, R off,
                          R v0, R v1, R v2, ClaimDep dep = ClaimDep{0, false}) {
  int b = atomicAdd(&D.nbc[0], 1);
  int bs = atomicAdd(&D.nbc[1 + sp], 1);
  if (b >= D.nb_cap) {
    atomicOr(&D.ctr->err, ERR_NB);
    return;
  }
  Birth<R> r;
  r.sp = sp;
  r.idx = bs;
  r.k = k;
  r.cell = cell;
  r.creator = creator;
  r.off = off;
  r.v0 = v0;
  r.v1 = v1;
  r.v2 = v2;
  if (D.N[sp] + bs >= D.cap[sp]) {
    atomicOr(&D.ctr->err, ERR_NB);
    r.sp = -1;
    r.creator = 0;
  }
  D.nb[b] = r;
  atomicAdd(&D.bhist[birth_bucket(r.creator, (uint64_t)D.ctr->next_id)], 1);
  if (r.sp >= 0) deposit_claim(C, D, sp, cell, off, 1, dep);
}

template <class R>
__device__ __forceinline__ uint64_t pick_key(const Consts<R>& C, uint64_t id_p, uint64_t id_t, uint32_t n) {
  uint4 w = philox((uint32_t)id_p, (uint32_t)(id_p >> 32), (uint32_t)id_t, (uint32_t)(id_t >> 32), C.seed_lo ^ n,
                   C.seed_hi ^ 0x5BD1E995u);
  return ((uint64_t)(w.x >> 8) << 40) | (id_p & ID_MASK);
}

// equal-mass isotropic elastic collision of two electrons
template <class R>
__device__ __forceinline__ void ee_elastic(R va[3], R vb[3], const R n[3]) {
  R V[3], g[3];
#pragma unroll
  for (int d = 0; d < 3; d++) {
    V[d] = (va[d] + vb[d]) * (R)0.5;
    g[d] = va[d] - vb[d];
  }
  R g2 = (g[0] * g[0] + g[1] * g[1]) + g[2] * g[2];
  R h = (R)0.5 * Sqrt(g2);
#pragma unroll
  for (int d = 0; d < 3; d++) {
    va[d] = V[d] + h * n[d];
    vb[d] = V[d] - h * n[d];
  }
}

// ---------------------------------------------------------------------------
// field: node charge from (count, fraction sum), exact Green's function of
// the 3-point Dirichlet problem, boundary field from Gauss on a half cell
// ---------------------------------------------------------------------------
constexpr int FIELD_TPB = 1024;
constexpr int NMAX_CELLS = 8192;

constexpr int FIELD_PER_MAX = (NMAX_CELLS + FIELD_TPB) / FIELD_TPB;

// mode 0: solve only (creation); mode 1: step (diagnostics, clear the
// accumulators of the species moved in this step).  A single workgroup.
// Global memory is read and written with node i = tid + k * FIELD_TPB
// (coalesced); the prefix sums run over LDS with each thread owning PER
// consecutive nodes.
struct FieldLds {
  union {
    int64_t q[NMAX_CELLS + 1];   // net charge per node, then
    double phi[NMAX_CELLS + 1];  // the potential (each slot read before it is overwritten)
  } v;
  __int128 wsA[FIELD_TPB / 64];
  __int128 wsB[FIELD_TPB / 64];
  int64_t fb[3][FIELD_PER_MAX][FIELD_TPB / 64];  // F of each wave's last node
  int64_t q0, qN;
};

// inclusive prefix sum of a 128-bit integer across the lanes of a wave
__device__ __forceinline__ __int128 wave_scan_i128(__int128 x) {
  const int lane = threadIdx.x & 63;
  uint64_t lo = (uint64_t)x, hi = (uint64_t)((unsigned __int128)x >> 64);
#pragma unroll
  for (int d = 1; d < 64; d <<= 1) {
    const uint64_t ylo = __shfl_up(lo, d), yhi = __shfl_up(hi, d);
    if (lane >= d) {
      const uint64_t s = lo + ylo;
      hi = hi + yhi + (s < lo ? 1 : 0);
      lo = s;
    }
  }
  return (__int128)(((unsigned __int128)hi << 64) | lo);
}

template <class R, int PER>
__device__ void field_phase(const Consts<R>& C, const Dev<R>& D, int mode, int64_t n, FieldLds& FL,
                            bool direct = false) {
  const int tid = threadIdx.x;
  const int lane = tid & 63, wv = tid >> 6;
  const int N = C.N;
  const bool ion = (n % C.nsub) == 0;
  if (direct) {
    // the net node charge of the step, formed by k_charge (partner reactions
    // since then included)
#pragma unroll
    for (int k = 0; k < PER; k++) {
      const int i = tid + k * FIELD_TPB;
      if (i > N) continue;
      const int64_t q = D.qnet[i];
      FL.v.q[i] = q;
      if (i == 0) FL.q0 = q;
      if (i == N) FL.qN = q;
    }
  } else {
    // 1. node charge Q_s[i] = 2^24 cnt[i] - F[i] + F[i-1], node i = tid + k *
    // FIELD_TPB (coalesced); F[i-1] is the left neighbour's F[i], by a shuffle
    // inside the wave and through LDS across waves.  With the step's
    // diagnostics (mode 1) the rf-cycle sums take one integer addition per node
    // and step, by the thread that owns the node: this workgroup is the only
    // writer, so a plain read-modify-write, its loads in flight with the others
    int32_t cn[3][PER];
    int64_t Fc[3][PER], qa[3][PER];
#pragma unroll
    for (int s = 0; s < 3; s++)
#pragma unroll
      for (int k = 0; k < PER; k++) {
        const int i = tid + k * FIELD_TPB;
        cn[s][k] = i < N ? D.cnt[s * N + i] : 0;
        Fc[s][k] = i < N ? D.F[s * N + i] : 0;
      }
#pragma unroll
    for (int s = 0; s < 3; s++)
#pragma unroll
      for (int k = 0; k < PER; k++) {
        const int i = tid + k * FIELD_TPB;
        qa[s][k] = (i <= N && mode == 1) ? D.Qacc[s * (N + 1) + i] : 0;
      }
    if (lane == 63) {
#pragma unroll
      for (int s = 0; s < 3; s++)
#pragma unroll
        for (int k = 0; k < PER; k++) FL.fb[s][k][wv] = Fc[s][k];
    }
    __syncthreads();
#pragma unroll
    for (int k = 0; k < PER; k++) {
      const int i = tid + k * FIELD_TPB;
      int64_t Qs[3];
#pragma unroll
      for (int s = 0; s < 3; s++) {
        int64_t left = __shfl_up(Fc[s][k], 1);
        if (lane == 0) left = wv > 0 ? FL.fb[s][k][wv - 1] : (k > 0 ? FL.fb[s][k - 1][FIELD_TPB / 64 - 1] : 0);
        const int64_t Fm = (i >= 1 && i <= N) ? left : 0;
        const int64_t v = (((int64_t)cn[s][k] << 24) - Fc[s][k]) + Fm;
        Qs[s] = v;
        if (i <= N) {
          D.Qcur[s * (N + 1) + i] = v;
          if (mode == 1) D.Qacc[s * (N + 1) + i] = qa[s][k] + v;
        }
      }
      if (i > N) continue;
      const int64_t q = (Qs[2] - Qs[0]) - Qs[1];
      FL.v.q[i] = q;
      if (i == 0) FL.q0 = q;
      if (i == N) FL.qN = q;
    }
    if (mode == 1) {
      // the passes of this step deposit every moved particle afresh
#pragma unroll
      for (int s = 0; s < 3; s++) {
        if (s != 0 && !ion) continue;
#pragma unroll
        for (int k = 0; k < PER; k++) {
          const int i = tid + k * FIELD_TPB;
          if (i < N) {
            D.cnt[s * N + i] = 0;
            D.F[s * N + i] = 0;
          }
        }
      }
    }
  }
  __syncthreads();
  // 2. potential from the exact discrete Green's function, contiguous nodes
  const double U = D.U[n % C.M];  // the driven electrode's potential
  const int i0 = min(tid * PER, N + 1);
  const int i1 = min(i0 + PER, N + 1);
  int64_t qloc[PER];
  __int128 a = 0, b = 0;
#pragma unroll
  for (int k = 0; k < PER; k++) {
    const int i = i0 + k;
    qloc[k] = i < i1 ? FL.v.q[i] : 0;
    if (i >= 1 && i <= N - 1 && i < i1) {
      a += (__int128)i * qloc[k];
      b += (__int128)(N - i) * qloc[k];
    }
  }
  // block-wide exclusive prefix sums of a and b: waves by shuffles, then the
  // 16 wave totals (integer sums: exact in any order)
  const __int128 ia = wave_scan_i128(a), ib = wave_scan_i128(b);
  if (lane == 63) {
    FL.wsA[wv] = ia;
    FL.wsB[wv] = ib;
  }
  __syncthreads();
  __int128 S1 = ia - a;   // sum_{j < i0} j q_j
  __int128 PB = ib - b;   // sum_{j < i0} (N-j) q_j
  __int128 TB = 0;
#pragma unroll
  for (int w = 0; w < FIELD_TPB / 64; w++) {
    if (w < wv) {
      S1 += FL.wsA[w];
      PB += FL.wsB[w];
    }
    TB += FL.wsB[w];
  }
#pragma unroll
  for (int k = 0; k < PER; k++) {
    const int i = i0 + k;
    if (i >= i1) continue;
    const int64_t q = qloc[k];
    if (i >= 1 && i <= N - 1) {
      S1 += (__int128)i * q;
      PB += (__int128)(N - i) * q;
    }
    double ph;
    if (i == 0) ph = U;
    else if (i == N) ph = 0.0;
    else {
      const __int128 S2 = TB - PB;  // sum_{j > i} (N-j) q_j
      const __int128 T = (__int128)(N - i) * S1 + (__int128)i * S2;
      const double x = U * (double)(N - i);
      const double y = C.cphi * i128_to_double(T);
      ph = (x + y) / (double)N;
    }
    FL.v.phi[i] = ph;
  }
  // the potential's cycle sums (in flight while the workgroup meets)
  double pa[PER];
#pragma unroll
  for (int k = 0; k < PER; k++) {
    const int i = tid + k * FIELD_TPB;
    pa[k] = (i <= N && mode == 1) ? D.phiacc[i] : 0.0;
  }
  __syncthreads();
  // 3. field, with the half-cell Gauss law at the electrodes (coalesced)
  const double* phis = FL.v.phi;
#pragma unroll
  for (int k = 0; k < PER; k++) {
    const int i = tid + k * FIELD_TPB;
    if (i > N) continue;
    double e;
    if (i == 0) e = (phis[0] - phis[1]) * C.invdx - C.cE * (double)FL.q0;
    else if (i == N) e = (phis[N - 1] - phis[N]) * C.invdx + C.cE * (double)FL.qN;
    else e = (phis[i - 1] - phis[i + 1]) * C.inv2dx;
    D.E[i] = e;
    D.phi[i] = phis[i];
    const R er = (R)e;
    if (i < N) D.E2[2 * i] = er;
    if (i >= 1) D.E2[2 * (i - 1) + 1] = er;
    if (mode == 1) D.phiacc[i] = pa[k] + phis[i];
  }
}

template <class R, int PER>
__device__ __forceinline__ void k_field_body(const Consts<R>& C, const Dev<R>& D, int mode) {
  __shared__ FieldLds FL;
  field_phase<R, PER>(C, D, mode, D.ctr->step, FL);
}

template <class R, int PER>
__global__ void __launch_bounds__(FIELD_TPB) k_field(Consts<R> C, Dev<R> D, int mode) {
  k_field_body<R, PER>(C, D, mode);
}

// the same for a batch of discharges, one per blockIdx.y
template <class R, int PER>
__global__ void __launch_bounds__(FIELD_TPB) k_field_b(const Consts<R>* __restrict__ Cs, const Dev<R>* __restrict__ Ds, int mode) {
  k_field_body<R, PER>(Cs[blockIdx.y], Ds[blockIdx.y], mode);
}

template <class R>
inline hipError_t launch_field(const Consts<R>& C, const Dev<R>& D, int mode, hipStream_t st) {
  const int per = (C.N + 1 + FIELD_TPB - 1) / FIELD_TPB;
  switch (per) {
    case 1: hipLaunchKernelGGL((k_field<R, 1>), dim3(1), dim3(FIELD_TPB), 0, st, C, D, mode); break;
    case 2: hipLaunchKernelGGL((k_field<R, 2>), dim3(1), dim3(FIELD_TPB), 0, st, C, D, mode); break;
    case 3: hipLaunchKernelGGL((k_field<R, 3>), dim3(1), dim3(FIELD_TPB), 0, st, C, D, mode); break;
    case 4: hipLaunchKernelGGL((k_field<R, 4>), dim3(1), dim3(FIELD_TPB), 0, st, C, D, mode); break;
    case 5: hipLaunchKernelGGL((k_field<R, 5>), dim3(1), dim3(FIELD_TPB), 0, st, C, D, mode); break;
    case 6: case 7: hipLaunchKernelGGL((k_field<R, 7>), dim3(1), dim3(FIELD_TPB), 0, st, C, D, mode); break;
    default: hipLaunchKernelGGL((k_field<R, FIELD_PER_MAX>), dim3(1), dim3(FIELD_TPB), 0, st, C, D, mode); break;
  }
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// diagnostics accumulated per workgroup in LDS
// ---------------------------------------------------------------------------
struct DiagLds {
  int32_t eedf[EEDF_MAX + 1];
  int32_t fneg[FNEG_MAX];
  int32_t ev[NCH];
  int32_t absorbed[6];
  int32_t tophits;
  int32_t psteps;
};

__device__ inline void diag_init(DiagLds& G) {
  for (int i = threadIdx.x; i < EEDF_MAX + 1; i += blockDim.x) G.eedf[i] = 0;
  for (int i = threadIdx.x; i < FNEG_MAX; i += blockDim.x) G.fneg[i] = 0;
  if (threadIdx.x < NCH) G.ev[threadIdx.x] = 0;
  if (threadIdx.x < 6) G.absorbed[threadIdx.x] = 0;
  if (threadIdx.x == 0) {
    G.tophits = 0;
    G.psteps = 0;
  }
}

template <class R>
__device__ inline void diag_flush(const Consts<R>& C, const Dev<R>& D, DiagLds& G) {
  const int tid = threadIdx.x;
  if (tid == 0 && G.psteps) atomicAdd((unsigned long long*)&D.ctr->psteps, (unsigned long long)G.psteps);
  if (tid < NCH && G.ev[tid]) atomicAdd((unsigned long long*)&D.ctr->events[tid], (unsigned long long)G.ev[tid]);
  if (tid < 6 && G.absorbed[tid])
    atomicAdd((unsigned long long*)&D.ctr->absorbed[tid], (unsigned long long)G.absorbed[tid]);
  if (tid == 0 && G.tophits) atomicAdd((unsigned long long*)&D.ctr->tophits, (unsigned long long)G.tophits);
  if (C.eedf_bins > 0)
    for (int i = tid; i <= C.eedf_bins; i += blockDim.x)
      if (G.eedf[i]) atomicAdd((unsigned long long*)&D.eedf_acc[i], (unsigned long long)G.eedf[i]);
  const int nf = C.fneg_xbins * C.fneg_ebins;
  for (int i = tid; i < nf; i += blockDim.x)
    if (G.fneg[i]) atomicAdd((unsigned long long*)&D.fneg_acc[i], (unsigned long long)G.fneg[i]);
}

template <class R, int S>
__device__ __forceinline__ void diag_alive(const Consts<R>& C, DiagLds& G, int cell, R vx, R vy, R vz) {
  if (S == 0) {
    if (cell == C.cmid && C.eedf_bins > 0) {
      const R e2 = (vx * vx + vy * vy) + vz * vz;
      const R Ek = C.hme * e2;
      const R bf = Ek * C.eedf_sc;
      const int bin = (bf >= (R)C.eedf_bins) ? C.eedf_bins : (int)bf;
      atomicAdd(&G.eedf[bin], 1);
    }
  } else if (S == 1) {
    if (C.fneg_xbins > 0 && C.fneg_ebins > 0) {
      R Ex = C.hmn * (vx * vx);
      if (vx < (R)0) Ex = -Ex;
      const R bf = (Ex + C.fneg_em) * C.fneg_sc;
      const int eb = bf < (R)0 ? 0 : (bf >= (R)C.fneg_ebins ? C.fneg_ebins - 1 : (int)bf);
      const int xb = (int)(((int64_t)cell * C.fneg_xbins) / C.N);
      atomicAdd(&G.fneg[xb * C.fneg_ebins + eb], 1);
    }
  }
}

// ---------------------------------------------------------------------------
// collisions of the candidates of the null-collision test (Eq. (1)): channel
// decision, gas-target and partner reactions, kinematics, births.  The push
// kernel already deposited every candidate at its post-push position; a
// candidate that is removed here takes its deposit back.
// ---------------------------------------------------------------------------
template <class R, int S>
__device__ __forceinline__ bool gas_event(const Consts<R>& C, const Dev<R>& D, int j, int cell, R off, uint64_t id, R v[3],
                          const R vt[3], R g, R Erel, uint32_t n, uint32_t kr) {
  const uint4 w = rng(C, id, n, kr);
  R n1[3], n2[3];
  iso_dir<R>(C, w.x, w.y, n1);
  iso_dir<R>(C, w.z, w.w, n2);
  const R a = C.a_g[S], b = C.b_g[S];
  R vc[3];
#pragma unroll
  for (int d = 0; d < 3; d++) vc[d] = b * v[d] + a * vt[d];
  if (S == 0 && j == 10) {  // (15) dissociative attachment: O- born at v_cm
    add_birth(C, D, 1, id, 0, cell, off, vc[0], vc[1], vc[2]);
    return false;
  }
  if (S == 1 && (j == 15 || j == 16)) {  // (16) direct / (17) associative detachment
    const R f = (j == 15) ? C.ddf : C.adf;
    const R sp = f * g;
    add_birth(C, D, 0, id, 0, cell, off, vc[0] + sp * n1[0], vc[1] + sp * n1[1], vc[2] + sp * n1[2]);
    return false;
  }
  R gp = g;
  if (C.loss[j] > (R)0) {
    const R Ep = Erel - C.loss[j];
    gp = Sqrt(Ep * C.c2e_g[S]);
  }
  const R ag = a * gp, bg = b * gp;
  if (S == 0 && j == 11) {  // (18) impact ionisation
    R ve[3], vo[3], vn[3];
#pragma unroll
    for (int d = 0; d < 3; d++) {
      ve[d] = vc[d] + ag * n1[d];
      vo[d] = vc[d] - bg * n1[d];
      vn[d] = vo[d];
    }
    ee_elastic<R>(ve, vn, n2);
    v[0] = ve[0];
    v[1] = ve[1];
    v[2] = ve[2];
    add_birth(C, D, 0, id, 0, cell, off, vn[0], vn[1], vn[2]);
    add_birth(C, D, 2, id, 1, cell, off, vo[0], vo[1], vo[2]);
    return true;
  }
#pragma unroll
  for (int d = 0; d < 3; d++) v[d] = vc[d] + ag * n1[d];
  return true;
}

// gas channels of species S: first channel and count (decision order)
template <int S> struct GasCh {
  static constexpr int G0 = (S == 0) ? 0 : (S == 1 ? 14 : 18);
  static constexpr int NG = (S == 0) ? 12 : (S == 1 ? 3 : 1);
};

// the cross sections the decision reads: the compact LDS copy of the
// species' gas channels (lds) or the full table in global memory
template <class R>
struct TabRef {
  const R* p;
  bool lds;
};

// sigma of channel j from the compact copy: nodes below tab_k0[j] are zero
template <class R>
__device__ __forceinline__ R sig_compact(const Consts<R>& C, const R* tab, int j, const Lookup<R>& L) {
  const int k0 = C.tab_k0[j];
  const R* t = tab + C.tab_off[j] - k0;
  if (L.mode == 2) return (NPT - 1 >= k0) ? t[NPT - 1] : (R)0;
  if (L.k < k0) return (R)0;
  R s0 = t[L.k];
  if (L.mode == 1) return s0;
  R s1 = t[L.k + 1];
  R d = s1 - s0;
  R p = L.t * d;
  return s0 + p;
}

template <class R>
__device__ __forceinline__ R sig_of(const Consts<R>& C, const TabRef<R>& T, int j, const Lookup<R>& L) {
  return T.lds ? sig_compact(C, T.p, j, L) : sig_at(T.p, TS, j, L);
}

// what a candidate's collision reads besides its record: (vy, vz) of its
// slot and the partner populations of its cell (segment lengths of the
// last sort), loaded for several candidates before any of them is collided
template <class R>
struct CandIn {
  Cand<R> k;
  R vy, vz;
  int32_t Lc[2];
};

template <class R, int S>
__device__ __forceinline__ void cand_partners(const Consts<R>& C, const Dev<R>& D, CandIn<R>& a) {
  const int N = C.N;
  constexpr int NP = (S == 0) ? 2 : (S == 1 ? 1 : 0);
#pragma unroll
  for (int q = 0; q < NP; q++) {
    const int chan = (S == 0) ? 12 + q : 17;
    const int t = (chan == 13) ? 1 : 2;
    a.Lc[q] = D.seg[t * (N + 1) + a.k.cell + 1] - D.seg[t * (N + 1) + a.k.cell];
  }
}

template <class R, int S>
__device__ __forceinline__ void collide_apply(const Consts<R>& C, const Dev<R>& D, DiagLds& G, const TabRef<R>& T,
                                              const CandIn<R>& a, uint32_t n) {
  const Store<R> st = D.st[S];
  const int N = C.N;
  const int slot = a.k.slot;
  const int cell = a.k.cell;
  const R off = a.k.off;
  R v[3];
  v[0] = a.k.vx;
  v[1] = a.vy;
  v[2] = a.vz;
  const uint64_t id = a.k.id;
  const uint4 w = rng(C, id, n, 0);
  const double U = unif52(w.x, w.y);
  double cum = 0.0;
  // partner channels first: slot size tau n_t(c) M_j (thinned at the step's end)
  constexpr int NP = (S == 0) ? 2 : (S == 1 ? 1 : 0);
#pragma unroll
  for (int q = 0; q < NP; q++) {
    const int pi = (S == 0) ? q : 2;
    const int chan = (S == 0) ? 12 + q : 17;
    cum = cum + (double)a.Lc[q] * C.KP[pi];
    if (U < cum) {
      const int r = atomicAdd(D.nreq, 1);
      if (r < D.req_cap) {
        Request<R> rq;
        rq.sp = S;
        rq.chan = chan;
        rq.slot = slot;
        rq.cell = cell;
        rq.id = id;
        rq.u_acc = unif<R>(w.z);
        rq.partner = -1;
        rq.acc = 0;
        D.req[r] = rq;
      } else {
        atomicOr(&D.ctr->err, ERR_REQ);
      }
      diag_alive<R, S>(C, G, cell, v[0], v[1], v[2]);
      return;
    }
  }
  // gas target drawn from the Maxwellian at T_gas
  const uint4 u = rng(C, id, n, 1);
  const R r1 = bm_radius<R>(C, unif<R>(u.x)), a1 = unif<R>(u.y);
  const R r2 = bm_radius<R>(C, unif<R>(u.z)), a2 = unif<R>(u.w);
  R vt[3];
  vt[0] = C.vthg * (r1 * cos2pi<R>(C, a1));
  vt[1] = C.vthg * (r1 * sin2pi<R>(C, a1));
  vt[2] = C.vthg * (r2 * cos2pi<R>(C, a2));
  const R gx = v[0] - vt[0], gy = v[1] - vt[1], gz = v[2] - vt[2];
  const R g2 = (gx * gx + gy * gy) + gz * gz;
  const R g = Sqrt(g2);
  const R Erel = C.hmu_g[S] * g2;
  if (Erel >= (R)16384) atomicAdd(&G.tophits, 1);
  const Lookup<R> Lk = lookup(Erel);
  constexpr int G0 = GasCh<S>::G0, NG = GasCh<S>::NG;
  int hit = -1;
#pragma unroll
  for (int q = 0; q < NG; q++) {
    const int j = G0 + q;
    R sg = 0;
    if (Erel >= C.thr[j]) sg = sig_of(C, T, j, Lk) * g;
    cum = cum + C.PG[j] * (double)sg;
    if (hit < 0 && U < cum) hit = j;
  }
  if (hit >= 0) {
    atomicAdd(&G.ev[hit], 1);
    if (gas_event<R, S>(C, D, hit, cell, off, id, v, vt, g, Erel, n, 2)) {
      st.vx[slot] = v[0];
      st_yz(st, slot, v[1], v[2]);
    } else {
      st.cell[slot] = DEAD;
      deposit_global(D, N, S, cell, off, -1);
      return;
    }
  }
  diag_alive<R, S>(C, G, cell, v[0], v[1], v[2]);
}

// The collisions of candidates e = tid, tid + TPB, ... < tot of a batch (rec(e):
// record index), two per round and thread: both records, then both
// candidates' other inputs are loaded before either is collided, so that each
// dependent load is waited for once per pair.
template <class R, int S, int TPB, class Rec>
__device__ __forceinline__ void collide_range(const Consts<R>& C, const Dev<R>& D, DiagLds& G, const TabRef<R>& T,
                                              int tot, Rec rec, uint32_t n) {
  const Store<R> st = D.st[S];
  for (int e = threadIdx.x; e < tot; e += 2 * TPB) {
    const bool two = e + TPB < tot;
    CandIn<R> a, b;
    a.k = D.cand[S][rec(e)];
    if (two) b.k = D.cand[S][rec(e + TPB)];
    ld_yz(st, a.k.slot, a.vy, a.vz);
    cand_partners<R, S>(C, D, a);
    if (two) {
      ld_yz(st, b.k.slot, b.vy, b.vz);
      cand_partners<R, S>(C, D, b);
    }
    collide_apply<R, S>(C, D, G, T, a, n);
    if (two) collide_apply<R, S>(C, D, G, T, b, n);
  }
}

// ---------------------------------------------------------------------------
// fused particle step: gather, leapfrog, absorption, null-collision test,
// deposit; then the collisions of the workgroup's own candidates
// ---------------------------------------------------------------------------
// node field staged in LDS by k_push when the grid is small enough (16 KB)
constexpr int PUSH_ELDS_BYTES = 16 * 1024 + 16;
template <class R> struct PushE {
  static constexpr int MAXN = PUSH_ELDS_BYTES / (int)sizeof(R) - 1;  // cells
};

// LDS bytes for the cross sections of one species during its collisions:
// the same bytes as the push phase's deposit windows and node field, so that
// the kernel's LDS (34 KB) still lets four workgroups share a CU.  The
// electrons' twelve gas channels in full would take 43 KB, which leaves room
// for two; stored from the first nonzero node of each channel up they take
// 22 KB in FP32.
constexpr int TAB_LDS_BYTES = 24576;
constexpr int FB = 64;  // tiles per collision batch (a species' tiles of one workgroup in the large discharge)

// LDS of the fused particle kernel.  The push phase uses the two deposit
// windows of consecutive tiles (alternating) and, with ELDS, the node field;
// the collision phase reuses the same bytes for the compact cross sections of
// the gas channels of the species it collides
template <class R, bool ELDS, class SH>
struct PushLds {
  union __attribute__((aligned(16))) {
    struct {
      uint64_t win[2][WIN];
      R El[ELDS ? PushE<R>::MAXN + 1 : 1];
    } p;
    R tab[TAB_LDS_BYTES / sizeof(R)];
  } u;
  DiagLds G;
  int32_t cpre[FB * SH::NW + 1];
  int32_t wsum[SH::NW];
};

template <class R> struct Vec4;
template <> struct Vec4<float> {
  static __device__ __forceinline__ void load(const float* p, float o[4]) {
    const float4 v = *(const float4*)p;
    o[0] = v.x; o[1] = v.y; o[2] = v.z; o[3] = v.w;
  }
  static __device__ __forceinline__ void store(float* p, const float o[4]) {
    *(float4*)p = make_float4(o[0], o[1], o[2], o[3]);
  }
};
template <> struct Vec4<double> {
  static __device__ __forceinline__ void load(const double* p, double o[4]) {
    const double2 a = *(const double2*)p, b = *(const double2*)(p + 2);
    o[0] = a.x; o[1] = a.y; o[2] = b.x; o[3] = b.y;
  }
  static __device__ __forceinline__ void store(double* p, const double o[4]) {
    *(double2*)p = make_double2(o[0], o[1]);
    *(double2*)(p + 2) = make_double2(o[2], o[3]);
  }
};

// add a packed (count << 40 | sum of 24-bit fractions) to one cell
__device__ __forceinline__ void deposit_win(uint64_t* win, int32_t* cnt, int64_t* F, int base, int cell,
                                            uint64_t packed) {
  const int idx = cell - base;
  if ((unsigned)idx < (unsigned)WIN) {
    atomicAdd((unsigned long long*)&win[idx], (unsigned long long)packed);
  } else {
    atomicAdd(&cnt[cell], (int)(packed >> 40));
    atomicAdd((unsigned long long*)&F[cell], (unsigned long long)(packed & F_MASK));
  }
}

// one thread's PPT consecutive particles of a tile (16-byte vector loads)
template <class R, int PPT>
struct TileRegs {
  int32_t c[PPT];
  R off[PPT], vx[PPT];
  uint64_t id[PPT];
};

template <class R, int PPT>
__device__ __forceinline__ void load_tile(const Store<R>& st, int64_t t0, int64_t Ns, TileRegs<R, PPT>& P) {
  const int64_t s0 = t0 + (int64_t)PPT * threadIdx.x;
  if (s0 + PPT - 1 < Ns) {
#pragma unroll
    for (int h = 0; h < PPT; h += 4) {
      const int4 cv = *(const int4*)(st.cell + s0 + h);
      P.c[h] = cv.x; P.c[h + 1] = cv.y; P.c[h + 2] = cv.z; P.c[h + 3] = cv.w;
      Vec4<R>::load(st.off + s0 + h, P.off + h);
      Vec4<R>::load(st.vx + s0 + h, P.vx + h);
      const ulonglong2 ia = *(const ulonglong2*)(st.id + s0 + h), ib = *(const ulonglong2*)(st.id + s0 + h + 2);
      P.id[h] = ia.x; P.id[h + 1] = ia.y; P.id[h + 2] = ib.x; P.id[h + 3] = ib.y;
    }
  } else {
#pragma unroll
    for (int q = 0; q < PPT; q++) {
      const bool in = s0 + q < Ns;
      P.c[q] = in ? st.cell[s0 + q] : DEAD;
      P.off[q] = in ? st.off[s0 + q] : (R)0;
      P.vx[q] = in ? st.vx[s0 + q] : (R)0;
      P.id[q] = in ? st.id[s0 + q] : 0;
    }
  }
}

struct TileCount {
  int pushed, abs0, abs1;
  int32_t next_cell;  // first cell of the workgroup's next tile, read before this tile's barrier
};

// the deposit window of a tile starts 64 cells below its first particle's
// cell, as that cell was before the push: every wave must use the same base,
// so the cell is read before any wave of the workgroup can have pushed the
// tile (at kernel start, or before the previous tile's barrier)
__device__ __forceinline__ int win_base(int32_t first_cell) { return (first_cell == DEAD ? 0 : first_cell) - 64; }

// One workgroup pushes one tile of TILE consecutive particles.  Deposits go
// to an LDS window of WIN cells (one 64-bit LDS atomic per run of a thread's
// particles in one cell), flushed to global memory after the tile's single
// barrier; consecutive tiles alternate between two windows, so the next tile
// starts while this one is flushed.  Each wave writes its candidates to its
// own region of the list.  next_first points at the first cell of the
// workgroup's next tile (null if none).
template <class R, int S, bool ELDS, class SH>
__device__ __forceinline__ TileCount push_tile(const Consts<R>& C, const Dev<R>& D, uint64_t* win, DiagLds& G,
                                               const R* El, const TileRegs<R, SH::PPT>& P, int64_t t0, int64_t Ns,
                                               uint32_t n, uint64_t T0, double pmax, int base,
                                               const int32_t* next_first) {
  constexpr int TPB = SH::TPB, PPT = SH::PPT, WTILE = SH::WTILE;
  TileCount tc = {0, 0, 0, DEAD};
  const int tid = threadIdx.x;
  const int lane = tid & 63;
  const int N = C.N;
  const Store<R> st = D.st[S];
  int32_t* cnt_s = D.cnt + (size_t)S * N;
  int64_t* F_s = D.F + (size_t)S * N;
  if (next_first) tc.next_cell = *next_first;
  const int64_t s0 = t0 + (int64_t)PPT * tid;
  int32_t c[PPT];
  R off[PPT], vx[PPT];
  uint64_t id[PPT];
#pragma unroll
  for (int q = 0; q < PPT; q++) {
    c[q] = P.c[q];
    off[q] = P.off[q];
    vx[q] = P.vx[q];
    id[q] = P.id[q];
  }
  const bool full = s0 + PPT - 1 < Ns;
  bool was_dead[PPT];
#pragma unroll
  for (int q = 0; q < PPT; q++) {
    // a cell outside the grid can only come from a corrupted store: report it
    // and leave the slot alone rather than read past the field arrays
    if (c[q] != DEAD && (unsigned)c[q] >= (unsigned)N) {
      atomicOr(&D.ctr->err, ERR_NAN);
      c[q] = DEAD;
    }
    was_dead[q] = c[q] == DEAD;
  }
  int candmask = 0;
  // a thread's consecutive particles mostly share a cell: one atomic per run
  int run_cell = -1;
  uint64_t run_val = 0;
#pragma unroll
  for (int q = 0; q < PPT; q++) {
    if (was_dead[q]) continue;
    tc.pushed++;
    R E0, E1;
    if (ELDS) {
      E0 = El[c[q]];
      E1 = El[c[q] + 1];
    } else {
      E0 = D.E2[2 * c[q]];
      E1 = D.E2[2 * c[q] + 1];
    }
    const R dE = E1 - E0;
    const R tt = off[q] * dE;
    const R Ep = E0 + tt;
    const R dv = C.qmdt[S] * Ep;
    vx[q] = vx[q] + dv;
    const R dxp = vx[q] * C.dtdx[S];
    R o = off[q] + dxp;
    const R fl = Floor(o);
    if (!(fl == fl) || fl > (R)1e9 || fl < (R)-1e9) {
      c[q] = DEAD;
      atomicOr(&D.ctr->err, ERR_NAN);
      continue;
    }
    int32_t cn = c[q] + (int32_t)fl;
    o = o - fl;
    if (o >= (R)1) {
      o = 0;
      cn += 1;
    }
    off[q] = o;
    if (cn < 0) {
      c[q] = DEAD;
      tc.abs0++;
      continue;
    }
    if (cn >= N) {
      c[q] = DEAD;
      tc.abs1++;
      continue;
    }
    c[q] = cn;
    if (cn != run_cell) {
      if (run_cell >= 0) deposit_win(win, cnt_s, F_s, base, run_cell, run_val);
      run_cell = cn;
      run_val = 0;
    }
    run_val += (1ull << 40) + (uint64_t)frac24(o);
    bool cand = false;
    if (T0 != 0) {
      const uint4 w = rng(C, id[q], n, 0);
      cand = (uint64_t)w.x < T0 && unif52(w.x, w.y) < pmax;
    }
    if (cand) {
      candmask |= 1 << q;
    } else if (S == 0) {
      if (cn == C.cmid) {
        R vy, vz;
        ld_yz(st, s0 + q, vy, vz);
        diag_alive<R, S>(C, G, cn, vx[q], vy, vz);
      }
    } else if (S == 1) {
      diag_alive<R, S>(C, G, cn, vx[q], (R)0, (R)0);
    }
  }
  if (run_cell >= 0) deposit_win(win, cnt_s, F_s, base, run_cell, run_val);
  if (full) {
#pragma unroll
    for (int h = 0; h < PPT; h += 4) {
      *(int4*)(st.cell + s0 + h) = make_int4(c[h], c[h + 1], c[h + 2], c[h + 3]);
      Vec4<R>::store(st.off + s0 + h, off + h);
      Vec4<R>::store(st.vx + s0 + h, vx + h);
    }
  } else {
#pragma unroll
    for (int q = 0; q < PPT; q++) {
      if (s0 + q < Ns && !was_dead[q]) {
        st.cell[s0 + q] = c[q];
        st.off[s0 + q] = off[q];
        st.vx[s0 + q] = vx[q];
      }
    }
  }
  // candidates go to the wave's own region of the list (its 256 slots)
  const int mine = __popc(candmask);
  int incl = mine;
#pragma unroll
  for (int d = 1; d < 64; d <<= 1) {
    const int y = __shfl_up(incl, d);
    if (lane >= d) incl += y;
  }
  const int64_t r0 = t0 + (int64_t)(tid >> 6) * WTILE;
  int pos = incl - mine;
#pragma unroll
  for (int q = 0; q < PPT; q++)
    if (candmask & (1 << q)) {
      Cand<R> k;
      k.slot = (int32_t)(s0 + q);
      k.cell = c[q];
      k.off = off[q];
      k.vx = vx[q];
      k.id = id[q];
      D.cand[S][r0 + pos++] = k;
    }
  if (lane == 63) D.tcnt[S][r0 / WTILE] = incl;
  __syncthreads();
  for (int i = tid; i < WIN; i += TPB) {
    const uint64_t v = win[i];
    if (v) {
      const int cc = base + i;
      atomicAdd(&cnt_s[cc], (int)(v >> 40));
      atomicAdd((unsigned long long*)&F_s[cc], (unsigned long long)(v & F_MASK));
      win[i] = 0;
    }
  }
  return tc;
}

template <class R>
__device__ __forceinline__ double pmax_of(const Consts<R>& C, const Dev<R>& D, int s) {
  double P = C.PGtot[s];
  if (s == 0) {
    P = P + (double)D.segmax[2] * C.KP[0];
    P = P + (double)D.segmax[1] * C.KP[1];
  } else if (s == 1) {
    P = P + (double)D.segmax[2] * C.KP[2];
  }
  return P;
}

// The workgroup's tiles of species S: tiles tb + u of the species' tile
// sequence, u = u0, u0 + B.n, ... < nts (u0: this workgroup's first).  The deposit
// window of a tile starts 64 cells below its first particle's cell as stored
// before the push; every wave must use the same base, so the cell of the
// segment's first tile is read before a barrier, and each next tile's during
// the previous tile (before that tile's barrier).  (Loading each tile's
// particles a tile ahead was measured no faster and costs 20 registers.)
template <class R, int S, bool ELDS, class SH>
__device__ __forceinline__ void push_loop(const Consts<R>& C, const Dev<R>& D, uint64_t (*win)[WIN], DiagLds& G,
                                          const R* El, int64_t u0, int64_t nts, Blk B, int& buf, int64_t Ns,
                                          uint32_t n, uint64_t T0, double pm, int& ps, int& abs0, int& abs1) {
  constexpr int TILE = SH::TILE;
  const Store<R> st = D.st[S];
  int base = u0 < nts ? win_base(st.cell[u0 * TILE]) : 0;
  __syncthreads();
  for (int64_t u = u0; u < nts; u += B.n, buf ^= 1) {
    const bool more = u + B.n < nts;
    const int32_t* nf = more ? st.cell + (u + B.n) * TILE : nullptr;
    TileRegs<R, SH::PPT> P;
    load_tile(st, u * TILE, Ns, P);
    const TileCount k = push_tile<R, S, ELDS, SH>(C, D, win[buf], G, El, P, u * TILE, Ns, n, T0, pm, base, nf);
    abs0 += k.abs0;
    abs1 += k.abs1;
    ps += k.pushed;
    base = win_base(k.next_cell);
  }
}

// The collisions of the candidates of this workgroup's tiles of species S
// (the tiles u0, u0 + B.n, ... < nts of the species), in batches of up to FB
// tiles.  The candidate records and counts were stored by every wave of the
// workgroup (global memory), and the last window flush has to end before the
// cross sections take its LDS.
template <class R, int S, bool ELDS, class SH>
__device__ __forceinline__ void collide_species(const Consts<R>& C, const Dev<R>& D, PushLds<R, ELDS, SH>& L,
                                                int64_t u0, int64_t nts, Blk B, uint32_t n) {
  constexpr int TPB = SH::TPB, TILE = SH::TILE, WTILE = SH::WTILE, NW = SH::NW;
  const int tid = threadIdx.x;
  wg_global_sync();
  if (u0 >= nts) return;
  const int tab_n = C.tab_n[S];
  if (tab_n > 0) {
    // the species' compact table into LDS: 16-byte vectors, every load of a
    // thread issued before its first store
    constexpr int V4 = (TAB_LDS_BYTES / (int)sizeof(R) / 4 + TPB - 1) / TPB;
    const int n4 = (tab_n + 3) / 4;
    const R* src = D.sigc + C.tab_base[S];
    R v[V4][4];
#pragma unroll
    for (int b = 0; b < V4; b++) {
      const int i = tid + b * TPB;
      if (i < n4) Vec4<R>::load(src + 4 * i, v[b]);
    }
#pragma unroll
    for (int b = 0; b < V4; b++) {
      const int i = tid + b * TPB;
      if (i < n4) Vec4<R>::store(L.u.tab + 4 * i, v[b]);
    }
  }
  const TabRef<R> T = tab_n > 0 ? TabRef<R>{L.u.tab, true} : TabRef<R>{D.sig, false};
  for (int64_t u = u0; u < nts;) {
    int nbt = 0;
    for (int64_t x = u; nbt < FB && x < nts; x += B.n) nbt++;
    // prefix of the candidate counts of the batch's wave regions (one per thread)
    {
      static_assert(FB * NW <= TPB, "one wave region per thread");
      const int lane = tid & 63, wv = tid >> 6;
      int x = 0;
      if (tid < nbt * NW) {
        const int64_t tile = u + (int64_t)(tid / NW) * B.n;
        x = D.tcnt[S][tile * NW + (tid % NW)];
      }
#pragma unroll
      for (int d = 1; d < 64; d <<= 1) {
        const int y = __shfl_up(x, d);
        if (lane >= d) x += y;
      }
      if (lane == 63) L.wsum[wv] = x;
      __syncthreads();
      for (int w = 0; w < wv; w++) x += L.wsum[w];
      L.cpre[tid + 1] = x;
      if (tid == 0) L.cpre[0] = 0;
    }
    __syncthreads();
    const int tot = L.cpre[nbt * NW];
    // candidate e of the batch: record index in the species' list
    auto rec = [&](int e) -> int64_t {
      int lo = 0, hi = nbt * NW;
      while (hi - lo > 1) {
        const int mid = (lo + hi) >> 1;
        if (L.cpre[mid] <= e) lo = mid;
        else hi = mid;
      }
      const int64_t tile = u + (int64_t)(lo / NW) * B.n;
      return tile * TILE + (lo % NW) * WTILE + (e - L.cpre[lo]);
    };
    collide_range<R, S, TPB>(C, D, L.G, T, tot, rec, n);
    __syncthreads();
    u += (int64_t)nbt * B.n;
  }
}

// ELDS: the node field (rounded to R, the values of E2) is staged in LDS
// and the gather reads it there; for grids up to PushE<R>::MAXN cells.
// The step's tiles (species by species, TILE particles each) are dealt to
// the workgroups round robin.  A workgroup pushes all its tiles, then
// collides their candidates species by species.  (Colliding each species
// right after its tiles, with the species order reversed in every other
// workgroup so that collisions overlap other workgroups' pushes, was
// measured no faster: the push phase slowed by what the collisions gained.)
template <class R, bool ELDS, class SH>
__device__ __forceinline__ void k_push_body(const Consts<R>& C, const Dev<R>& D, Blk B) {
  constexpr int TPB = SH::TPB, TILE = SH::TILE;
  __shared__ PushLds<R, ELDS, SH> L;
  R* El = L.u.p.El;
  const int tid = threadIdx.x;
  const int64_t nstep = D.ctr->step;
  const uint32_t n = (uint32_t)nstep;
  const bool ion = (nstep % C.nsub) == 0;
  if (B.x == 0 && tid == 0) D.ctr->step_push = nstep;
  diag_init(L.G);
  for (int i = tid; i < 2 * WIN; i += TPB) L.u.p.win[i / WIN][i % WIN] = 0;
  if (ELDS)
    for (int i = tid; i <= C.N; i += TPB) El[i] = (R)D.E[i];
  int64_t Ns[3], nt[3];
  double pm[3];
  uint64_t T0[3];
  for (int s = 0; s < 3; s++) {
    Ns[s] = (s == 0 || ion) ? D.N[s] : 0;
    nt[s] = (Ns[s] + TILE - 1) / TILE;
    pm[s] = pmax_of(C, D, s);
    const double t = ceil(pm[s] * 4294967296.0);
    T0[s] = t >= 4294967296.0 ? (1ull << 32) : (uint64_t)t;
    if (Ns[s] > 0 && pm[s] > 1.0 && B.x == 0 && tid == 0) atomicOr(&D.ctr->err, ERR_PMAX);
  }
  // this workgroup's first tile of each species: tiles are numbered through
  // the species in order e, O-, O2+ and tile t goes to workgroup t mod B.n
  int64_t u0[3];
  {
    int64_t tb = 0;
    for (int s = 0; s < 3; s++) {
      u0[s] = ((int64_t)B.x - tb % B.n + B.n) % B.n;
      tb += nt[s];
    }
  }
  int ps = 0, ab[3][2] = {{0, 0}, {0, 0}, {0, 0}};
  int buf = 0;
  push_loop<R, 0, ELDS, SH>(C, D, L.u.p.win, L.G, El, u0[0], nt[0], B, buf, Ns[0], n, T0[0], pm[0], ps, ab[0][0],
                        ab[0][1]);
  push_loop<R, 1, ELDS, SH>(C, D, L.u.p.win, L.G, El, u0[1], nt[1], B, buf, Ns[1], n, T0[1], pm[1], ps, ab[1][0],
                        ab[1][1]);
  push_loop<R, 2, ELDS, SH>(C, D, L.u.p.win, L.G, El, u0[2], nt[2], B, buf, Ns[2], n, T0[2], pm[2], ps, ab[2][0],
                        ab[2][1]);
  // (no collision phase where the null-collision bound is zero: the per-cell
  // collision list replaces it)
  if (T0[0] != 0) collide_species<R, 0, ELDS, SH>(C, D, L, u0[0], nt[0], B, n);
  if (T0[1] != 0) collide_species<R, 1, ELDS, SH>(C, D, L, u0[1], nt[1], B, n);
  if (T0[2] != 0) collide_species<R, 2, ELDS, SH>(C, D, L, u0[2], nt[2], B, n);
  // [electrode][species]
  for (int s = 0; s < 3; s++) {
    if (ab[s][0]) atomicAdd(&L.G.absorbed[s], ab[s][0]);
    if (ab[s][1]) atomicAdd(&L.G.absorbed[3 + s], ab[s][1]);
  }
  if (ps) atomicAdd(&L.G.psteps, ps);
  __syncthreads();
  diag_flush(C, D, L.G);
}

// the constants and device state are read from device memory (a copy per
// buffer parity), not passed by value: a kilobyte of kernel arguments held in
// scalar registers would spill into vector registers this kernel needs
template <class R, bool ELDS, class SH>
__global__ void __launch_bounds__(SH::TPB, 3) k_push(const Consts<R>* __restrict__ Cp,
                                                                   const Dev<R>* __restrict__ Dp) {
  k_push_body<R, ELDS, SH>(*Cp, *Dp, Blk{(int)blockIdx.x, (int)gridDim.x});
}

// the same for a batch of discharges over a 1-D grid (workgroups of discharge i:
// [off[i], off[i + 1]))
template <class R, bool ELDS, class SH>
__global__ void __launch_bounds__(SH::TPB, 3) k_push_b(const Consts<R>* __restrict__ Cs,
                                                                     const Dev<R>* __restrict__ Ds,
                                                                     const int32_t* __restrict__ off, int nd) {
  Blk b;
  const int i = batch_block(off, nd, b);
  k_push_body<R, ELDS, SH>(Cs[i], Ds[i], b);
}

// ---------------------------------------------------------------------------
// last-workgroup detection (no spinning: the final workgroup to arrive does
// the serial part)
// ---------------------------------------------------------------------------
__device__ __forceinline__ bool last_block(uint32_t* counter, int grid) {
  __shared__ bool is_last;
  __threadfence();
  __syncthreads();
  if (threadIdx.x == 0) is_last = (atomicAdd(counter, 1u) == (uint32_t)grid - 1);
  __syncthreads();
  if (is_last) __threadfence();
  return is_last;
}

// ---------------------------------------------------------------------------
// end of the step, one workgroup:
//  1. partner reactions (13), (14), (19): pick in the cell segment of the last
//     sort, acceptance sigma g / M_j, claims (smallest test id wins; electron
//     requests before O- requests), kinematics, births, charge corrections;
//  2. births: counting sort of this step's births over creator-id buckets
// ---------------------------------------------------------------------------
constexpr int TAIL_TPB = 1024;

template <class R>
__device__ void kill_particle(const Consts<R>& C, const Dev<R>& D, int sp, int slot, ClaimDep dep = ClaimDep{0, false}) {
  const Store<R> st = D.st[sp];
  const int cell = st.cell[slot];
  if (cell == DEAD) return;
  const R off = st.off[slot];
  deposit_claim(C, D, sp, cell, off, -1, dep);
  st.cell[slot] = DEAD;
}

// (19): inelastic collision of test electron `slot` (id) with partner O- `p`:
// the O- splits into O + e (loss dE of Eq. (5)), the two electrons scatter
// elastically; directions from the electron's stream kr
template <class R>
__device__ void impact_detach(const Consts<R>& C, const Dev<R>& D, int slot, int p, uint64_t id, uint32_t n, uint32_t kr,
                              ClaimDep dep = ClaimDep{0, false}) {
  const Store<R> es = D.st[0], ns = D.st[1];
  R T[3], P[3];
  T[0] = es.vx[slot];
  ld_yz(es, slot, T[1], T[2]);
  P[0] = ns.vx[p];
  ld_yz(ns, p, P[1], P[2]);
  const int pc = ns.cell[p];  // the O-'s place, loaded with the velocities
  const R po = ns.off[p];
  const R a = C.a_c[1], b = C.b_c[1];
  const R gx = T[0] - P[0], gy = T[1] - P[1], gz = T[2] - P[2];
  const R g2 = (gx * gx + gy * gy) + gz * gz;
  const R Erel = C.hmu_c[1] * g2;
  const uint4 w = rng(C, id, n, kr);
  R n1[3], n2[3];
  iso_dir<R>(C, w.x, w.y, n1);
  iso_dir<R>(C, w.z, w.w, n2);
  const R Ep = Erel - C.loss[13];
  const R gp = Sqrt(Ep * C.c2e_c[1]);
  const R ag = a * gp, bg = b * gp;
  R ve[3], vn[3];
#pragma unroll
  for (int d = 0; d < 3; d++) {
    const R vc = b * T[d] + a * P[d];
    ve[d] = vc + ag * n1[d];
    vn[d] = vc - bg * n1[d];
  }
  ee_elastic<R>(ve, vn, n2);
  es.vx[slot] = ve[0];
  st_yz(es, slot, ve[1], ve[2]);
  if (pc != DEAD) {  // the O- is removed (as kill_particle does, its place known)
    deposit_claim(C, D, 1, pc, po, -1, dep);
    ns.cell[p] = DEAD;
  }
  add_birth(C, D, 0, id, 0, pc, po, vn[0], vn[1], vn[2], dep);
}

constexpr int REQ_LDS = 64;  // requests kept in LDS while they are resolved (the rest read from global memory)
struct ClaimLds {
  int32_t rpart[REQ_CAP];
  uint64_t rid[REQ_CAP];
  uint8_t racc[REQ_CAP];
  uint8_t rwin[REQ_CAP];
  alignas(16) unsigned char rq[REQ_LDS * sizeof(Request<double>)];
};
static_assert(sizeof(Request<float>) <= sizeof(Request<double>), "request slots");

template <class R>
__device__ void resolve_claims(const Consts<R>& C, const Dev<R>& D, ClaimLds& L, int nr, uint32_t n, ClaimDep dep) {
  const int tid = threadIdx.x;
  const int lane = tid & 63, wv = tid >> 6;
  constexpr int NWV = TAIL_TPB / 64;
  const int N = C.N;
  __shared__ uint64_t kmin[NWV];
  // the first REQ_LDS requests are read once (one round trip), then from LDS
  Request<R>* rq = reinterpret_cast<Request<R>*>(L.rq);
  if (tid < min(nr, REQ_LDS)) rq[tid] = D.req[tid];
  __syncthreads();
  auto req = [&](int r) -> Request<R> { return r < REQ_LDS ? rq[r] : D.req[r]; };
  // the smallest key over lanes sub*64 + lane, stepping per*64, of request
  // r's partner segment (keys end in the partner id, so they are distinct);
  // four loads in flight per lane
  auto scan = [&](int r, int sub, int per, uint64_t& best, int32_t& bslot) {
    const Request<R> q = req(r);
    const int t = (q.chan == 13) ? 1 : 2;
    const int32_t lo = D.seg[t * (N + 1) + q.cell], hi = D.seg[t * (N + 1) + q.cell + 1];
    const uint64_t* ids = D.st[t].id;
    const int stride = per * 64;
    best = ~0ull;
    bslot = -1;
    for (int32_t i = lo + sub * 64 + lane; i < hi; i += 4 * stride) {
      uint64_t id4[4];
#pragma unroll
      for (int u = 0; u < 4; u++) id4[u] = (i + u * stride < hi) ? ids[i + u * stride] : 0;
#pragma unroll
      for (int u = 0; u < 4; u++) {
        if (i + u * stride >= hi) continue;
        const uint64_t k = pick_key(C, id4[u], q.id, n);
        if (k < best) {
          best = k;
          bslot = i + u * stride;
        }
      }
    }
#pragma unroll
    for (int d = 32; d > 0; d >>= 1) {
      const uint64_t ok = __shfl_xor(best, d);
      const int32_t os = __shfl_xor(bslot, d);
      if (ok < best) {
        best = ok;
        bslot = os;
      }
    }
  };
  // acceptance of request r with partner p (-1: none), one lane
  auto accept = [&](int r, int32_t p) {
    const Request<R> q = req(r);
    const int t = (q.chan == 13) ? 1 : 2;
    int acc = 0;
    if (p >= 0) {
      // the partner's cell and both velocities in flight together (the slot
      // lies in the partner segment: in bounds whether alive or not)
      const Store<R> ts = D.st[q.sp], ps = D.st[t];
      const int32_t pcell = ps.cell[p];
      R ty, tz, py, pz;
      ld_yz(ts, q.slot, ty, tz);
      ld_yz(ps, p, py, pz);
      const R tvx = ts.vx[q.slot], pvx = ps.vx[p];
      if (pcell != DEAD) {
        const int pi = (q.chan == 12) ? 0 : (q.chan == 13 ? 1 : 2);
        const R gx = tvx - pvx, gy = ty - py, gz = tz - pz;
        const R g2 = (gx * gx + gy * gy) + gz * gz;
        const R g = Sqrt(g2);
        const R Erel = C.hmu_c[pi] * g2;
        R sg = 0;
        if (Erel >= C.thr[q.chan]) sg = sig_at(D.sig, TS, q.chan, lookup(Erel)) * g;
        acc = (q.u_acc * C.Mr_c[pi] < sg) ? 1 : 0;
      }
    }
    L.rpart[r] = p;
    L.rid[r] = q.id;
    L.racc[r] = (uint8_t)acc;
    L.rwin[r] = 0;
  };
  if (nr >= NWV) {
    // one wave per request
    for (int r = wv; r < nr; r += NWV) {
      uint64_t best;
      int32_t bslot;
      scan(r, 0, 1, best, bslot);
      if (lane == 0) accept(r, bslot);
    }
  } else {
    // fewer requests than waves: NWV / nr waves share each segment (a dense
    // discharge has thousands of partners per cell), minimum through LDS
    const int per = NWV / nr;
    const int r = wv / per, sub = wv % per;
    if (tid < nr) kmin[tid] = ~0ull;
    __syncthreads();
    uint64_t best = ~0ull;
    int32_t bslot = -1;
    if (r < nr) {
      scan(r, sub, per, best, bslot);
      if (lane == 0 && bslot >= 0) atomicMin((unsigned long long*)&kmin[r], (unsigned long long)best);
    }
    __syncthreads();
    if (r < nr && lane == 0) {
      if (kmin[r] == ~0ull) {
        if (sub == 0) accept(r, -1);
      } else if (bslot >= 0 && best == kmin[r]) {
        accept(r, bslot);
      }
    }
  }
  __syncthreads();
  // stage 1: electron test particles; (13) takes an O2+, (19) an O-
  for (int r = tid; r < nr; r += TAIL_TPB) {
    const Request<R> q = req(r);
    const int chan = q.chan;
    if (q.sp != 0 || !L.racc[r]) continue;
    int win = 1;
    for (int r2 = 0; r2 < nr && win; r2++) {
      if (r2 == r || !L.racc[r2] || req(r2).chan != chan) continue;
      if (L.rpart[r2] == L.rpart[r] && L.rid[r2] < L.rid[r]) win = 0;
    }
    L.rwin[r] = (uint8_t)win;
  }
  __syncthreads();
  int nacc = 0;
  for (int r = tid; r < nr; r += TAIL_TPB) {
    if (!L.rwin[r]) continue;
    const Request<R> q = req(r);
    nacc++;
    atomicAdd((unsigned long long*)&D.ctr->events[q.chan], 1ull);
    if (q.chan == 12) {
      kill_particle(C, D, 0, q.slot, dep);
      kill_particle(C, D, 2, L.rpart[r], dep);
      continue;
    }
    impact_detach(C, D, q.slot, L.rpart[r], q.id, n, 2, dep);
  }
  __syncthreads();
  // stage 2: O- test particles (14); the O- must not have been taken by a
  // (19) winner and the O2+ not by a (13) winner
  for (int r = tid; r < nr; r += TAIL_TPB) {
    const Request<R> q = req(r);
    if (q.sp != 1 || !L.racc[r]) continue;
    const int slot = q.slot;
    int ok = 1;
    for (int r2 = 0; r2 < nr && ok; r2++) {
      if (L.rwin[r2] != 1) continue;
      const int c2 = req(r2).chan;
      if (c2 == 13 && L.rpart[r2] == slot) ok = 0;
      if (c2 == 12 && L.rpart[r2] == L.rpart[r]) ok = 0;
    }
    L.racc[r] = (uint8_t)(ok ? 2 : 0);
  }
  __syncthreads();
  for (int r = tid; r < nr; r += TAIL_TPB) {
    if (L.racc[r] != 2) continue;
    int win = 1;
    for (int r2 = 0; r2 < nr && win; r2++) {
      if (r2 == r || L.racc[r2] != 2) continue;
      if (L.rpart[r2] == L.rpart[r] && L.rid[r2] < L.rid[r]) win = 0;
    }
    if (win) L.rwin[r] = 3;
  }
  __syncthreads();
  for (int r = tid; r < nr; r += TAIL_TPB) {
    if (L.rwin[r] != 3) continue;
    const Request<R> q = req(r);
    nacc++;
    atomicAdd((unsigned long long*)&D.ctr->events[17], 1ull);
    kill_particle(C, D, 1, q.slot, dep);
    kill_particle(C, D, 2, L.rpart[r], dep);
  }
  if (nacc) atomicAdd((unsigned long long*)&D.ctr->nacc, (unsigned long long)nacc);
  if (tid == 0) atomicAdd((unsigned long long*)&D.ctr->nreq, (unsigned long long)nr);
}

// ---------------------------------------------------------------------------
// end of step n and start of step n+1, one workgroup of 1024 threads:
//  1. partner reactions;
//  2. births: counting sort over creator-id buckets, rank inside the bucket
//     (canonical ids: rank by creator id, then k), append to the stores;
//  3. close the step (store lengths, id counter, rf-cycle sums);
//  4. unless a sort follows, the field of step n+1.
// ---------------------------------------------------------------------------
// exclusive prefix sum of one value per thread over a workgroup of TPB
// threads (shuffles inside waves, wsum[TPB/64] in LDS across them)
template <int TPB>
__device__ __forceinline__ int block_excl_scan(int x, int32_t* wsum, int* total) {
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  int incl = x;
#pragma unroll
  for (int d = 1; d < 64; d <<= 1) {
    const int y = __shfl_up(incl, d);
    if (lane >= d) incl += y;
  }
  if (lane == 63) wsum[wv] = incl;
  __syncthreads();
  int base = 0, tot = 0;
#pragma unroll
  for (int w = 0; w < TPB / 64; w++) {
    const int v = wsum[w];
    if (w < wv) base += v;
    tot += v;
  }
  *total = tot;
  __syncthreads();
  return base + incl - x;
}

constexpr int BKEYS = 8192;  // births whose rank keys are kept in LDS

template <class R>
__device__ void births_phase(const Consts<R>& C, const Dev<R>& D, int32_t* cur, int32_t* part, uint64_t* keys) {
  const int tid = threadIdx.x;
  int B = D.nbc[0];
  if (B > D.nb_cap) B = D.nb_cap;
  if (B == 0) return;
  constexpr int PER = NBUCKET / TAIL_TPB;
  static_assert(NBUCKET % TAIL_TPB == 0, "whole buckets per thread");
  // bucket counts to LDS (coalesced, every load in flight before the first
  // store), exclusive scan over consecutive buckets per thread
  {
    int32_t h[PER];
#pragma unroll
    for (int q = 0; q < PER; q++) h[q] = D.bhist[tid + q * TAIL_TPB];
#pragma unroll
    for (int q = 0; q < PER; q++) {
      cur[tid + q * TAIL_TPB] = h[q];
      D.bhist[tid + q * TAIL_TPB] = 0;
    }
  }
  __syncthreads();
  int loc[PER];
  int sum = 0;
#pragma unroll
  for (int q = 0; q < PER; q++) {
    loc[q] = cur[tid * PER + q];
    sum += loc[q];
  }
  int total;
  int run = block_excl_scan<TAIL_TPB>(sum, part, &total);
#pragma unroll
  for (int q = 0; q < PER; q++) {
    cur[tid * PER + q] = run;
    run += loc[q];
  }
  __syncthreads();
  // keys grouped by bucket: in LDS when they fit, else through perm in global
  // memory; afterwards cur[b] is the end of bucket b (= start of b + 1)
  const bool lds = B <= BKEYS;
  const uint64_t next = (uint64_t)D.ctr->next_id;
  for (int b = tid; b < B; b += TAIL_TPB) {
    const Birth<R> rec = D.nb[b];
    const int bkt = birth_bucket(rec.creator, next);
    const int slot = atomicAdd(&cur[bkt], 1);
    if (lds) keys[slot] = (rec.creator << 2) | (uint64_t)rec.k;
    else D.perm[slot] = b;
  }
  __syncthreads();
  for (int b = tid; b < B; b += TAIL_TPB) {
    const Birth<R> rec = D.nb[b];
    const uint64_t key = (rec.creator << 2) | (uint64_t)rec.k;
    const int bk = birth_bucket(rec.creator, next);
    const int lo = bk > 0 ? cur[bk - 1] : 0, hi = cur[bk];
    int rank = lo;
    for (int i = lo; i < hi; i++) {
      uint64_t ok;
      if (lds) {
        ok = keys[i];
      } else {
        const Birth<R>& o = D.nb[D.perm[i]];
        ok = (o.creator << 2) | (uint64_t)o.k;
      }
      rank += ok < key;
    }
    if (rec.sp >= 0) {
      const int sp = rec.sp;
      const int64_t slot = D.N[sp] + rec.idx;
      if (slot < D.cap[sp]) {
        const Store<R> st = D.st[sp];
        st.cell[slot] = rec.cell;
        st.off[slot] = rec.off;
        st.vx[slot] = rec.v0;
        st_yz(st, slot, rec.v1, rec.v2);
        st.id[slot] = next + (uint64_t)rank;
      }
    }
  }
}

// after births_phase (one thread): the births join the store lengths and the
// id counter; the birth and request lists are emptied
template <class R>
__device__ void close_births(const Dev<R>& D) {
  // every load before the first store (one round trip)
  int B = D.nbc[0];
  int64_t len[3];
  int32_t add[3];
#pragma unroll
  for (int s = 0; s < 3; s++) {
    len[s] = D.N[s];
    add[s] = D.nbc[1 + s];
  }
  const int64_t next = D.ctr->next_id, births = D.ctr->births;
  if (B > D.nb_cap) B = D.nb_cap;
#pragma unroll
  for (int s = 0; s < 3; s++) {
    int64_t nn = len[s] + add[s];
    if (nn > D.cap[s]) {
      nn = D.cap[s];
      atomicOr(&D.ctr->err, ERR_CAP);
    }
    D.N[s] = nn;
    D.nbc[1 + s] = 0;
  }
  D.ctr->next_id = next + B;
  D.ctr->births = births + B;
  if ((uint64_t)(next + B) > ID_MASK) atomicOr(&D.ctr->err, ERR_ID);
  D.nbc[0] = 0;
  *D.nreq = 0;
}

// close the rf cycle: move the accumulated sums to the last-cycle buffers
template <class R>
__device__ void close_cycle(const Consts<R>& C, const Dev<R>& D, bool q_done = false) {
  const int tid = threadIdx.x;
  const int N = C.N;
  // (q_done: k_charge has closed the node-charge sums already)
  for (int i = tid; i < 3 * (N + 1) && !q_done; i += TAIL_TPB) {
    D.Qlast[i] = D.Qacc[i];
    D.Qacc[i] = 0;
  }
  for (int i = tid; i <= N; i += TAIL_TPB) {
    D.philast[i] = D.phiacc[i];
    D.phiacc[i] = 0;
  }
  for (int i = tid; i <= C.eedf_bins; i += TAIL_TPB) {
    D.eedf_last[i] = D.eedf_acc[i];
    D.eedf_acc[i] = 0;
  }
  for (int i = tid; i < C.fneg_xbins * C.fneg_ebins; i += TAIL_TPB) {
    D.fneg_last[i] = D.fneg_acc[i];
    D.fneg_acc[i] = 0;
  }
  if (tid == 0) D.ctr->cycles += 1;
}

// clear the deposit counters of the species the next push moves (it deposits
// them afresh): electrons always, the ions when the next push moves them
template <class R>
__device__ void clear_counters(const Consts<R>& C, const Dev<R>& D, bool ion_next) {
  const int N = C.N;
  for (int s = 0; s < 3; s++) {
    if (s != 0 && !ion_next) continue;
    for (int i = threadIdx.x; i < N; i += TAIL_TPB) {
      D.cnt[s * N + i] = 0;
      D.F[s * N + i] = 0;
    }
  }
}

// End of step n, the step the push advanced.  Two workgroups: when no
// partner request is pending, the second computes the field of the next step
// (with the cycle sums) while the first places the births; with requests the
// first does everything in order, since the claims change the deposits the
// field is made from.
template <class R, int PER>
__device__ __forceinline__ void k_serial_body(const Consts<R>& C, const Dev<R>& D, int do_field) {
  __shared__ union {
    FieldLds field;
    ClaimLds claims;
    int32_t cur[NBUCKET];
  } U;
  __shared__ int32_t part[TAIL_TPB];
  __shared__ uint64_t bkeys[BKEYS];
  const int tid = threadIdx.x;
  const int64_t n = D.ctr->step_push;
  int nr = *D.nreq;
  if (nr > D.req_cap) nr = D.req_cap;
  const bool split = nr == 0 && do_field;
  const bool cyc = (n + 1) % C.M == 0;
  // do_field 2: k_charge has formed the step's node charge from the deposit
  // counters; the field is solved from it, the counters of the species the
  // next push moves are cleared by the workgroup that does not solve the
  // field (the partner reactions never touch those), and the reactions
  // change the node charge directly
  const bool direct = do_field == 2;
  const bool ion_next = ((n + 1) % C.nsub) == 0;
  const ClaimDep dep{direct ? 1 : 0, ion_next};
  if (blockIdx.x == 1) {
    if (!split) {
      if (direct) clear_counters(C, D, ion_next);
      return;
    }
    if (cyc) close_cycle(C, D, direct);
    __syncthreads();
    field_phase<R, PER>(C, D, 1, n + 1, U.field, direct);
    return;
  }
  // within the workgroup, barriers order the global writes of one phase
  // before the reads of the next (no device-scope fence needed)
  if (nr > 0) resolve_claims(C, D, U.claims, nr, (uint32_t)n, dep);
  __syncthreads();
  births_phase(C, D, U.cur, part, bkeys);
  __syncthreads();
  if (tid == 0) {
    close_births(D);
    D.ctr->step = n + 1;
  }
  if (split) {
    // the field is the other workgroup's, which reads only the net charge
    if (direct) clear_counters(C, D, ion_next);
    return;
  }
  if (cyc) close_cycle(C, D, direct);
  if (!do_field) return;
  __syncthreads();
  field_phase<R, PER>(C, D, 1, n + 1, U.field, direct);
}

template <class R, int PER>
__global__ void __launch_bounds__(TAIL_TPB) k_serial(Consts<R> C, Dev<R> D, int do_field) {
  k_serial_body<R, PER>(C, D, do_field);
}

// the same for a batch of discharges, one per blockIdx.y
template <class R, int PER>
__global__ void __launch_bounds__(TAIL_TPB) k_serial_b(const Consts<R>* __restrict__ Cs, const Dev<R>* __restrict__ Ds, int do_field) {
  k_serial_body<R, PER>(Cs[blockIdx.y], Ds[blockIdx.y], do_field);
}

template <class R>
inline hipError_t launch_serial(const Consts<R>& C, const Dev<R>& D, int do_field, hipStream_t st) {
  const int per = (C.N + 1 + FIELD_TPB - 1) / FIELD_TPB;
  switch (per) {
    case 1: hipLaunchKernelGGL((k_serial<R, 1>), dim3(2), dim3(TAIL_TPB), 0, st, C, D, do_field); break;
    case 2: hipLaunchKernelGGL((k_serial<R, 2>), dim3(2), dim3(TAIL_TPB), 0, st, C, D, do_field); break;
    case 3: hipLaunchKernelGGL((k_serial<R, 3>), dim3(2), dim3(TAIL_TPB), 0, st, C, D, do_field); break;
    case 4: hipLaunchKernelGGL((k_serial<R, 4>), dim3(2), dim3(TAIL_TPB), 0, st, C, D, do_field); break;
    case 5: hipLaunchKernelGGL((k_serial<R, 5>), dim3(2), dim3(TAIL_TPB), 0, st, C, D, do_field); break;
    case 6: case 7: hipLaunchKernelGGL((k_serial<R, 7>), dim3(2), dim3(TAIL_TPB), 0, st, C, D, do_field); break;
    default: hipLaunchKernelGGL((k_serial<R, FIELD_PER_MAX>), dim3(2), dim3(TAIL_TPB), 0, st, C, D, do_field); break;
  }
  return hipGetLastError();
}

// The node charge of step n+1 from the deposit counters, one thread per node
// (many workgroups, so that the single-workgroup field solve only reads the
// net charge): per species into Qcur and the rf-cycle sums (the cycle's sum
// moved to Qlast at its end), net into qnet.  The counters are only read.
constexpr int CHARGE_TPB = 256;
template <class R>
__device__ __forceinline__ void k_charge_body(const Consts<R>& C, const Dev<R>& D, int bx) {
  const int N = C.N;
  const int i = bx * CHARGE_TPB + (int)threadIdx.x;
  if (i > N) return;  // (batches launch for their largest grid)
  const bool cyc = (D.ctr->step_push + 1) % C.M == 0;
  int32_t cn[3];
  int64_t Fc[3], Fm[3], qa[3];
#pragma unroll
  for (int s = 0; s < 3; s++) {
    cn[s] = i < N ? D.cnt[s * N + i] : 0;
    Fc[s] = i < N ? D.F[s * N + i] : 0;
    Fm[s] = i >= 1 ? D.F[s * N + i - 1] : 0;
    qa[s] = D.Qacc[s * (N + 1) + i];
  }
  int64_t Qs[3];
#pragma unroll
  for (int s = 0; s < 3; s++) {
    const int64_t v = (((int64_t)cn[s] << 24) - Fc[s]) + Fm[s];
    Qs[s] = v;
    const int o = s * (N + 1) + i;
    D.Qcur[o] = v;
    if (cyc) {
      D.Qlast[o] = qa[s];
      D.Qacc[o] = v;
    } else {
      D.Qacc[o] = qa[s] + v;
    }
  }
  D.qnet[i] = (Qs[2] - Qs[0]) - Qs[1];
}

template <class R>
__global__ void __launch_bounds__(CHARGE_TPB) k_charge(Consts<R> C, Dev<R> D) {
  k_charge_body<R>(C, D, (int)blockIdx.x);
}

// the same for a batch of discharges, one per blockIdx.y
template <class R>
__global__ void __launch_bounds__(CHARGE_TPB) k_charge_b(const Consts<R>* __restrict__ Cs,
                                                          const Dev<R>* __restrict__ Ds) {
  k_charge_body<R>(Cs[blockIdx.y], Ds[blockIdx.y], (int)blockIdx.x);
}

template <class R>
inline hipError_t launch_charge(const Consts<R>& C, const Dev<R>& D, hipStream_t st) {
  hipLaunchKernelGGL(k_charge<R>, dim3((C.N + 1 + CHARGE_TPB - 1) / CHARGE_TPB), dim3(CHARGE_TPB), 0, st, C, D);
  return hipGetLastError();
}

// maxN: the largest grid of the batch
template <class R>
inline hipError_t launch_charge_b(const Consts<R>* C, const Dev<R>* D, int nd, int maxN, hipStream_t st) {
  hipLaunchKernelGGL(k_charge_b<R>, dim3((maxN + 1 + CHARGE_TPB - 1) / CHARGE_TPB, nd), dim3(CHARGE_TPB), 0, st, C, D);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// cell sort (counting sort by cell, dead particles dropped); the segments it
// produces are the partner populations of the cells until the next sort
// ---------------------------------------------------------------------------
constexpr int SCAN_TPB = 1024;

template <class R>
__device__ __forceinline__ void k_sort_scan_body(const Consts<R>& C, const Dev<R>& D) {
  __shared__ int64_t part[SCAN_TPB];
  __shared__ int32_t pmax[SCAN_TPB];
  const int s = blockIdx.x;
  const int tid = threadIdx.x;
  const int N = C.N;
  const int per = (N + SCAN_TPB - 1) / SCAN_TPB;
  const int i0 = tid * per, i1 = min(i0 + per, N);
  int64_t sum = 0;
  int32_t mx = 0;
  for (int i = i0; i < i1; i++) {
    int32_t c = D.cnt[s * N + i];
    sum += c;
    mx = max(mx, c);
  }
  part[tid] = sum;
  pmax[tid] = mx;
  __syncthreads();
  for (int d = 1; d < SCAN_TPB; d <<= 1) {
    int64_t x = (tid >= d) ? part[tid - d] : 0;
    int32_t y = (tid >= d) ? pmax[tid - d] : 0;
    __syncthreads();
    part[tid] += x;
    pmax[tid] = max(pmax[tid], y);
    __syncthreads();
  }
  // segments never reach past the store's capacity, whatever the counts say
  const int64_t cap = D.cap[s];
  int64_t run = part[tid] - sum;
  for (int i = i0; i < i1; i++) {
    D.seg[s * (N + 1) + i] = (int32_t)min(run, cap);
    D.cursor[s * N + i] = (int32_t)min(run, cap);
    run += D.cnt[s * N + i];
  }
  if (tid == SCAN_TPB - 1) {
    const int64_t total = part[SCAN_TPB - 1];
    if (total > cap) atomicOr(&D.ctr->err, ERR_SORT);
    D.seg[s * (N + 1) + N] = (int32_t)min(total, cap);
    D.Nnew[s] = min(total, cap);
    D.segmax[s] = pmax[SCAN_TPB - 1];
  }
}

template <class R>
__global__ void __launch_bounds__(SCAN_TPB) k_sort_scan(Consts<R> C, Dev<R> D) {
  k_sort_scan_body<R>(C, D);
}

// the same for a batch of discharges, one per blockIdx.y
template <class R>
__global__ void __launch_bounds__(SCAN_TPB) k_sort_scan_b(const Consts<R>* __restrict__ Cs, const Dev<R>* __restrict__ Ds) {
  k_sort_scan_body<R>(Cs[blockIdx.y], Ds[blockIdx.y]);
}

// 2048-particle chunks in 512-thread workgroups, two per CU (LDS): the cost
// of a chunk is mostly its fixed phases (ranks, run reservation, barriers),
// so larger chunks beat more workgroups of smaller ones
constexpr int SORT_TPB = 512;
constexpr int SORT_PER = 4;
constexpr int SORT_CHUNK = SORT_TPB * SORT_PER;
constexpr int SORT_WIN = 512;  // cells around the middle of a chunk

template <class R>
struct SortRegs {
  int32_t cell[SORT_PER];
  R off[SORT_PER], vx[SORT_PER], vy[SORT_PER], vz[SORT_PER];
  uint64_t id[SORT_PER];
};

template <class R>
struct SortLds {
  int32_t cnt[SORT_WIN];   // particles of the chunk per window cell
  int32_t lst[SORT_WIN];   // their first position in the staged chunk
  int32_t gb[SORT_WIN];    // their first destination in the sorted store
  int32_t wsum[SORT_TPB / 64];
  int32_t wbase, nst;
  int32_t cell[SORT_CHUNK];
  R off[SORT_CHUNK];
  R vx[SORT_CHUNK];
  typename Pair2<R>::T vyz[SORT_CHUNK];
  uint64_t id[SORT_CHUNK];
};

// Each workgroup sorts one contiguous chunk of a store in LDS and writes it
// out in cell runs, so that consecutive threads write consecutive addresses of
// the destination.  Ranks inside a wave come from ballots (one LDS atomic per
// wave and cell); one global atomic per (chunk, cell) reserves the run.  The
// order inside a cell is arbitrary: no result depends on it.  Particles whose
// cell lies outside the chunk's window take a global atomic of their own.
template <class R>
__device__ __forceinline__ void k_sort_scatter_body(const Consts<R>& C, const Dev<R>& D, Blk B) {
  __shared__ SortLds<R> L;
  const int N = C.N;
  const int tid = threadIdx.x;
  const int lane = tid & 63, wv = tid >> 6;
  const uint64_t below = (1ull << lane) - 1;
  int64_t Ns[3], nch[3];
  for (int s = 0; s < 3; s++) {
    Ns[s] = D.N[s];
    nch[s] = (Ns[s] + SORT_CHUNK - 1) / SORT_CHUNK;
  }
  const int64_t total = nch[0] + nch[1] + nch[2];
  // chunk t: species and first slot
  auto chunk = [&](int64_t t, int& s, int64_t& c0) {
    s = 0;
    int64_t c = t;
    if (c >= nch[0]) {
      c -= nch[0];
      s = 1;
      if (c >= nch[1]) {
        c -= nch[1];
        s = 2;
      }
    }
    c0 = c * SORT_CHUNK;
  };
  // the thread's particles of chunk t (dead past the store's end)
  auto load = [&](int64_t t, SortRegs<R>& q) {
    int s;
    int64_t c0;
    chunk(t, s, c0);
    const Store<R> a = D.st[s];
#pragma unroll
    for (int j = 0; j < SORT_PER; j++) {
      const int64_t slot = c0 + (int64_t)j * SORT_TPB + tid;
      const bool in = slot < Ns[s];
      q.cell[j] = in ? a.cell[slot] : DEAD;
      q.off[j] = in ? a.off[slot] : (R)0;
      q.vx[j] = in ? a.vx[slot] : (R)0;
      q.vy[j] = (R)0;
      q.vz[j] = (R)0;
      if (in) ld_yz(a, slot, q.vy[j], q.vz[j]);
      q.id[j] = in ? a.id[slot] : 0;
    }
  };
  // the next chunk's particles are loaded while this one is ranked, staged
  // and written
  SortRegs<R> P;
  if (B.x < total) load(B.x, P);
  for (int64_t t = B.x; t < total; t += B.n) {
    int s;
    int64_t c0;
    chunk(t, s, c0);
    const Store<R> b = D.alt[s];
    int32_t* cur = D.cursor + (size_t)s * N;
    const int32_t* seg = D.seg + (size_t)s * (N + 1);
    if (tid == 0) {
      // the window is centred on the chunk's middle particle (thread 0 holds
      // slot c0 + SORT_CHUNK / 2); where it sits changes only which cells
      // take the global path
      const int32_t cm = P.cell[SORT_PER / 2] != DEAD ? P.cell[SORT_PER / 2] : (P.cell[0] != DEAD ? P.cell[0] : 0);
      L.wbase = cm - SORT_WIN / 2;
    }
    for (int i = tid; i < SORT_WIN; i += SORT_TPB) L.cnt[i] = 0;
    int32_t rank[SORT_PER];
    int32_t* cell = P.cell;
    R* off = P.off;
    R* vx = P.vx;
    R* vy = P.vy;
    R* vz = P.vz;
    uint64_t* id = P.id;
    SortRegs<R> Q;
    const bool more = t + B.n < total;
    if (more) load(t + B.n, Q);
    __syncthreads();
    const int base = L.wbase;
#pragma unroll
    for (int j = 0; j < SORT_PER; j++) {
      const bool alive = cell[j] != DEAD;
      const int key = alive ? cell[j] : -1;
      rank[j] = -1;
      uint64_t pending = __ballot(alive);
      while (pending) {
        const int leader = __ffsll((unsigned long long)pending) - 1;
        const int lkey = __shfl(key, leader);
        const uint64_t peers = __ballot(key == lkey);
        const int cnt = __popcll(peers);
        int gb = 0;
        if (lane == leader) {
          const int idx = lkey - base;
          // window cells: rank in the chunk; others: their destination now
          gb = ((unsigned)idx < (unsigned)SORT_WIN) ? atomicAdd(&L.cnt[idx], cnt)
                                                     : (atomicAdd(&cur[lkey], cnt) | (1 << 30));
        }
        gb = __shfl(gb, leader);
        if (key == lkey) rank[j] = gb + __popcll(peers & below);
        pending &= ~peers;
      }
    }
    __syncthreads();
    // global runs and the exclusive scan of the window counts
    int32_t loc[SORT_WIN / SORT_TPB];
    int32_t sum = 0;
#pragma unroll
    for (int q = 0; q < SORT_WIN / SORT_TPB; q++) {
      const int i = tid * (SORT_WIN / SORT_TPB) + q;
      loc[q] = L.cnt[i];
      if (loc[q] > 0) L.gb[i] = atomicAdd(&cur[base + i], loc[q]);
      sum += loc[q];
    }
    int32_t x = sum;
#pragma unroll
    for (int d = 1; d < 64; d <<= 1) {
      const int32_t y = __shfl_up(x, d);
      if (lane >= d) x += y;
    }
    if (lane == 63) L.wsum[wv] = x;
    __syncthreads();
    int32_t run = x - sum;
    for (int w = 0; w < wv; w++) run += L.wsum[w];
#pragma unroll
    for (int q = 0; q < SORT_WIN / SORT_TPB; q++) {
      L.lst[tid * (SORT_WIN / SORT_TPB) + q] = run;
      run += loc[q];
    }
    if (tid == SORT_TPB - 1) L.nst = run;
    __syncthreads();
#pragma unroll
    for (int j = 0; j < SORT_PER; j++) {
      if (cell[j] == DEAD) continue;
      const int idx = cell[j] - base;
      if ((unsigned)idx < (unsigned)SORT_WIN) {
        const int p = L.lst[idx] + rank[j];
        L.cell[p] = cell[j];
        L.off[p] = off[j];
        L.vx[p] = vx[j];
        typename Pair2<R>::T yz;
        yz.x = vy[j];
        yz.y = vz[j];
        L.vyz[p] = yz;
        L.id[p] = id[j];
      } else {
        const int32_t dst = rank[j] & ~(1 << 30);
        if (dst < seg[cell[j]] || dst >= seg[cell[j] + 1] || dst >= D.cap[s]) {
          atomicOr(&D.ctr->err, ERR_SORT);
          continue;
        }
        b.cell[dst] = cell[j];
        b.off[dst] = off[j];
        b.vx[dst] = vx[j];
        st_yz(b, dst, vy[j], vz[j]);
        b.id[dst] = id[j];
      }
    }
    __syncthreads();
    const int nst = L.nst;
    for (int k = tid; k < nst; k += SORT_TPB) {
      const int32_t cl = L.cell[k];
      const int idx = cl - base;
      const int32_t dst = L.gb[idx] + (k - L.lst[idx]);
      if (dst < seg[cl] || dst >= seg[cl + 1] || dst >= D.cap[s]) {
        atomicOr(&D.ctr->err, ERR_SORT);
        continue;
      }
      b.cell[dst] = cl;
      b.off[dst] = L.off[k];
      b.vx[dst] = L.vx[k];
      *(typename Pair2<R>::T*)(b.vyz + 2 * (int64_t)dst) = L.vyz[k];
      b.id[dst] = L.id[k];
    }
    __syncthreads();
    if (more) P = Q;
  }
  if (!last_block(&D.done[2], B.n)) return;
  if (threadIdx.x == 0) {
    D.done[2] = 0;
    for (int s = 0; s < 3; s++) D.N[s] = D.Nnew[s];
  }
}

template <class R>
__global__ void __launch_bounds__(SORT_TPB) k_sort_scatter(Consts<R> C, Dev<R> D) {
  k_sort_scatter_body<R>(C, D, Blk{(int)blockIdx.x, (int)gridDim.x});
}

// the same for a batch of discharges over a 1-D grid (workgroups of discharge i:
// [off[i], off[i + 1]))
template <class R>
__global__ void __launch_bounds__(SORT_TPB) k_sort_scatter_b(const Consts<R>* __restrict__ Cs, const Dev<R>* __restrict__ Ds,
    const int32_t* __restrict__ off, int nd) {
  Blk b;
  const int i = batch_block(off, nd, b);
  k_sort_scatter_body<R>(Cs[i], Ds[i], b);
}

// ---------------------------------------------------------------------------
// intra-species Coulomb collisions (1)-(3): binary model of Takizuka and Abe
// with a Gaussian tan(chi/2) of the Eq. (2) variance and a uniform azimuth,
// run right after a sort, when each cell's particles are one segment
// ---------------------------------------------------------------------------
constexpr int COUL_TPB = 1024;
constexpr int COUL_MAXC = 16384;                 // particles of one species in one cell

// one binary collision; cc = prefactor times the cell count.  The relative
// velocity u = va - vb turns by the sampled angle; va takes fa and vb -fb of
// its change (mu/m of each particle: 1/2 for like particles)
template <class R>
__device__ __forceinline__ void ta_pair_m(const Consts<R>& C, R va[3], R vb[3], R cc, uint64_t rid, uint32_t n,
                                          uint32_t k, R fa, R fb) {
  const R ux = va[0] - vb[0], uy = va[1] - vb[1], uz = va[2] - vb[2];
  const R up2 = ux * ux + uy * uy;
  const R u2 = up2 + uz * uz;
  if (!(u2 > (R)0)) return;
  const R u = Sqrt(u2);
  const R var = cc / (u2 * u);
  const uint4 w = rng(C, rid, n, k);
  R st, omc;
  if (var > (R)1) {  // beyond the small-angle model: isotropic
    const R ct = (R)1 - (R)2 * unif<R>(w.w);
    st = Sqrt((R)1 - ct * ct);
    omc = (R)1 - ct;
  } else {
    const R nrm = bm_radius<R>(C, unif<R>(w.x)) * cos2pi<R>(C, unif<R>(w.y));
    const R d = Sqrt(var) * nrm;
    const R d2 = d * d;
    const R inv = (R)1 / ((R)1 + d2);
    st = (d + d) * inv;
    omc = (d2 + d2) * inv;
  }
  const R ph = unif<R>(w.z);
  R sph, cph;
  sincos2pi<R>(C, ph, sph, cph);
  const R s1 = st * cph, s2 = st * sph;
  R du[3];
  if (up2 > (R)0) {
    const R up = Sqrt(up2);
    const R iup = (R)1 / up;
    const R r = uz * s1, t = u * s2;
    du[0] = (ux * r - uy * t) * iup - ux * omc;
    du[1] = (uy * r + ux * t) * iup - uy * omc;
    du[2] = -(up * s1) - uz * omc;
  } else {
    du[0] = u * s1;
    du[1] = u * s2;
    du[2] = -(u * omc);
  }
#pragma unroll
  for (int d = 0; d < 3; d++) {
    va[d] = va[d] + fa * du[d];
    vb[d] = vb[d] - fb * du[d];
  }
}

// one collision of two equal-mass particles: each takes half of the change
template <class R>
__device__ __forceinline__ void ta_pair(const Consts<R>& C, R va[3], R vb[3], R cc, uint64_t rid, uint32_t n,
                                        uint32_t k) {
  ta_pair_m<R>(C, va, vb, cc, rid, n, k, (R)0.5, (R)0.5);
}

// exclusive prefix sum of a[0..n) in LDS by one 1024-thread workgroup
__device__ inline void block_scan_excl(int32_t* a, int n, int32_t* wsum) {
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  const int per = (n + COUL_TPB - 1) / COUL_TPB;
  const int i0 = min(tid * per, n), i1 = min(i0 + per, n);
  int32_t loc = 0;
  for (int i = i0; i < i1; i++) loc += a[i];
  int32_t x = loc;
#pragma unroll
  for (int d = 1; d < 64; d <<= 1) {
    const int32_t y = __shfl_up(x, d);
    if (lane >= d) x += y;
  }
  if (lane == 63) wsum[wv] = x;
  __syncthreads();
  if (tid < 64) {
    int32_t z = tid < COUL_TPB / 64 ? wsum[tid] : 0;
#pragma unroll
    for (int d = 1; d < 64; d <<= 1) {
      const int32_t y = __shfl_up(z, d);
      if (lane >= d) z += y;
    }
    if (tid < COUL_TPB / 64) wsum[tid] = z;
  }
  __syncthreads();
  int32_t run = x - loc + (wv > 0 ? wsum[wv - 1] : 0);
  for (int i = i0; i < i1; i++) {
    const int32_t v = a[i];
    a[i] = run;
    run += v;
  }
  __syncthreads();
}

__device__ __forceinline__ int coul_bucket(uint32_t h, int nb) { return (int)(((uint64_t)h * (uint32_t)nb) >> 32); }


// Pairing order of the Coulomb pass: the particles of one (species, cell)
// segment ordered by (Philox(id, n, 16).x, id).  A counting sort into
// nb = ceil(m/per) LDS buckets on the hash (monotone in it); a particle's rank
// is its bucket start plus the members of its bucket that precede it.
// Returns through ordp[r] (or ordg[a + r]) the position of the particle of rank r.
template <class R>
__device__ void coul_rank(const Consts<R>& C, const Store<R>& S, int32_t a, int m, int per, uint32_t n, uint32_t* h,
                          uint16_t* list, int32_t* bend, int32_t* wsum, uint16_t* ordp, int32_t* ordg,
                          uint32_t k = 16) {
  const int tid = threadIdx.x;
  const int nb = (m + per - 1) / per;
  for (int i = tid; i < nb; i += COUL_TPB) bend[i] = 0;
  __syncthreads();
  for (int i = tid; i < m; i += COUL_TPB) {
    const uint32_t x = rng(C, S.id[a + i], n, k).x;
    h[i] = x;
    atomicAdd(&bend[coul_bucket(x, nb)], 1);
  }
  __syncthreads();
  block_scan_excl(bend, nb, wsum);
  for (int i = tid; i < m; i += COUL_TPB) {
    const int pos = atomicAdd(&bend[coul_bucket(h[i], nb)], 1);
    list[pos] = (uint16_t)i;
  }
  __syncthreads();
  for (int i = tid; i < m; i += COUL_TPB) {
    const uint32_t hi = h[i];
    const int b = coul_bucket(hi, nb);
    const int b0 = b > 0 ? bend[b - 1] : 0, b1 = bend[b];
    int r = b0;
    for (int k = b0; k < b1; k++) {
      const int j = list[k];
      const uint32_t hj = h[j];
      if (hj < hi || (hj == hi && j != i && S.id[a + j] < S.id[a + i])) r++;
    }
    if (ordp) ordp[r] = (uint16_t)i;
    else ordg[a + r] = a + i;
  }
  if (ordg) wg_global_sync();  // other waves read the order from global memory
  else __syncthreads();
}

// Collisions of a cell whose velocities are in (vx, vy, vz)[0..m) (LDS or
// global, indexed by segment position through ord); one thread per pair, an
// odd cell first runs the triangle (o0,o1), (o1,o2), (o2,o0) with half the
// interval, in that order, on one thread.  The random numbers of the collision
// whose first particle has rank q are keyed by ((s N + cell) 2^32 + q).
template <class R, class ORD, class VX, class VYZ>
__device__ __forceinline__ void coul_pairs(const Consts<R>& C, const Dev<R>& D, int s, int cell, int m, uint32_t n,
                                           ORD ord, VX vx, VYZ vyz, int tpb) {
  const uint64_t key = (uint64_t)(s * C.N + cell) << 32;
  const int first = (m & 1) ? 3 : 0;
  const int npairs = (m - first) >> 1;
  const R cf = C.ccoul[s] * (R)m;
  for (int p = threadIdx.x; p < npairs + (first ? 1 : 0); p += tpb) {
    if (first && p == npairs) {
      const R ch = C.ccoul_h[s] * (R)m;
      const int i0 = ord(0), i1 = ord(1), i2 = ord(2);
      if (i0 >= m || i1 >= m || i2 >= m) {
        atomicOr(&D.ctr->err, ERR_COUL);
        continue;
      }
      R v0[3], v1[3], v2[3];
      v0[0] = vx(i0);
      vyz.get(i0, v0[1], v0[2]);
      v1[0] = vx(i1);
      vyz.get(i1, v1[1], v1[2]);
      v2[0] = vx(i2);
      vyz.get(i2, v2[1], v2[2]);
      ta_pair<R>(C, v0, v1, ch, key | 0u, n, 17);
      ta_pair<R>(C, v1, v2, ch, key | 1u, n, 18);
      ta_pair<R>(C, v2, v0, ch, key | 2u, n, 19);
      vx(i0) = v0[0];
      vyz.set(i0, v0[1], v0[2]);
      vx(i1) = v1[0];
      vyz.set(i1, v1[1], v1[2]);
      vx(i2) = v2[0];
      vyz.set(i2, v2[1], v2[2]);
      continue;
    }
    const int q = first + 2 * p;
    const int ia = ord(q), ib = ord(q + 1);
    if (ia >= m || ib >= m) {  // not a permutation: ids were not unique
      atomicOr(&D.ctr->err, ERR_COUL);
      continue;
    }
    R va[3], vb[3];
    va[0] = vx(ia);
    vyz.get(ia, va[1], va[2]);
    vb[0] = vx(ib);
    vyz.get(ib, vb[1], vb[2]);
    ta_pair<R>(C, va, vb, cf, key | (uint64_t)q, n, 17);
    vx(ia) = va[0];
    vyz.set(ia, va[1], va[2]);
    vx(ib) = vb[0];
    vyz.set(ib, vb[1], vb[2]);
  }
}

// exclusive prefix sum of a[0..n) in LDS by one workgroup of TPB threads:
// each wave scans a contiguous chunk with consecutive lanes on consecutive
// elements (no bank conflicts), then the wave totals are added
template <int TPB>
__device__ inline void block_scan_chunked(int32_t* a, int n, int32_t* wsum) {
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  constexpr int NW = TPB / 64;
  const int chunk = ((n + NW * 64 - 1) / (NW * 64)) * 64;
  const int base = wv * chunk;
  int run = 0;
  for (int j = 0; j < chunk; j += 64) {
    const int i = base + j + lane;
    const int x = i < n ? a[i] : 0;
    int incl = x;
#pragma unroll
    for (int d = 1; d < 64; d <<= 1) {
      const int y = __shfl_up(incl, d);
      if (lane >= d) incl += y;
    }
    if (i < n) a[i] = run + incl - x;
    run += __shfl(incl, 63);
  }
  if (lane == 0) wsum[wv] = run;
  __syncthreads();
  int off = 0;
  for (int w = 0; w < wv; w++) off += wsum[w];
  if (off)
    for (int j = 0; j < chunk; j += 64) {
      const int i = base + j + lane;
      if (i < n) a[i] += off;
    }
  __syncthreads();
}

// The pairing order of a cell that fits in LDS: one bucket per particle on
// average (nb = m); a thread keeps the hashes of its PT positions in
// registers; bucket members are (hash << 16 | position) entries, so that the
// rank of a particle reads one LDS word per member.
template <class R, int PT, int TPB>
__device__ void coul_rank_lds(const Consts<R>& C, const Store<R>& S, int32_t a, int m, uint32_t n, uint64_t* list,
                              int32_t* bend, int32_t* wsum, uint16_t* ord) {
  const int tid = threadIdx.x;
  const int nb = m;
  for (int i = tid; i < nb; i += TPB) bend[i] = 0;
  __syncthreads();
  uint32_t hr[PT];
#pragma unroll
  for (int j = 0; j < PT; j++) {
    const int i = tid + j * TPB;
    hr[j] = 0;
    if (i < m) {
      hr[j] = rng(C, S.id[a + i], n, 16).x;
      atomicAdd(&bend[coul_bucket(hr[j], nb)], 1);
    }
  }
  __syncthreads();
  block_scan_chunked<TPB>(bend, nb, wsum);
#pragma unroll
  for (int j = 0; j < PT; j++) {
    const int i = tid + j * TPB;
    if (i < m) {
      const int pos = atomicAdd(&bend[coul_bucket(hr[j], nb)], 1);
      list[pos] = ((uint64_t)hr[j] << 16) | (uint64_t)i;
    }
  }
  __syncthreads();
#pragma unroll
  for (int j = 0; j < PT; j++) {
    const int i = tid + j * TPB;
    if (i < m) {
      const uint32_t hi = hr[j];
      const int b = coul_bucket(hi, nb);
      const int b0 = b > 0 ? bend[b - 1] : 0, b1 = bend[b];
      int r = b0;
      for (int k = b0; k < b1; k++) {
        const uint64_t e = list[k];
        const uint32_t hj = (uint32_t)(e >> 16);
        const int pj = (int)(e & 0xFFFFu);
        if (hj < hi || (hj == hi && pj != i && S.id[a + pj] < S.id[a + i])) r++;
      }
      ord[r] = (uint16_t)i;
    }
  }
  __syncthreads();
}

template <class R>
struct LdsVyz {
  R* y;
  R* z;
  __device__ void get(int i, R& a, R& b) const { a = y[i]; b = z[i]; }
  __device__ void set(int i, R a, R b) const { y[i] = a; z[i] = b; }
};
template <class R>
struct GlobVyz {
  Store<R> S;
  int32_t a;
  __device__ void get(int i, R& y, R& z) const { ld_yz(S, a + i, y, z); }
  __device__ void set(int i, R y, R z) const { st_yz(S, a + i, y, z); }
};

// Coulomb pass of the cells that fit in LDS: one workgroup per (species,
// cell).  The pairing order is built in LDS, then the cell's velocities are
// staged in LDS (reusing the sort's arrays), collided there and written back,
// so that every global access is coalesced.  Size classes: up to 2048
// particles in a 256-thread workgroup (several per CU), up to 5120 in a
// 512-thread workgroup (FP32: two per CU), up to CoulCap<R>::M in a
// 1024-thread workgroup; larger cells are listed for k_coul_big.
template <class R> struct CoulCap;
template <> struct CoulCap<float> { static constexpr int M = 8192; };
template <> struct CoulCap<double> { static constexpr int M = 4096; };
constexpr int COUL_TINY = 512;   // one wave: many workgroups per CU for the many small cells
constexpr int COUL_TTPB = 64;
constexpr int COUL_SMALL = 2048;
constexpr int COUL_STPB = 256;
constexpr int COUL_MID = 5120;   // two workgroups per CU in FP32 (one per LDS half)
constexpr int COUL_MTPB = 1024;  // with at most 64 VGPRs: eight waves per SIMD

template <class R, int M, int TPB>
struct CoulLds {
  union {
    struct {
      uint64_t list[M];  // (hash << 16 | position), grouped by bucket
      int32_t bend[M];
    } o;
    struct {
      R vx[M], vy[M], vz[M];
    } v;
  } u;
  uint16_t ord[M];
  int32_t wsum[TPB / 64];
};

// collisions of one cell (species s, m particles from segment position a)
// with its velocities staged in LDS
template <class R, int M, int TPB>
__device__ __forceinline__ void coul_cell(const Consts<R>& C, const Dev<R>& D, CoulLds<R, M, TPB>& L, int s, int cell,
                                          int32_t a, int m, uint32_t n) {
  const int tid = threadIdx.x;
  const Store<R> S = D.st[s];
  // the velocities are loaded with the ids and parked in registers while the
  // order is built in the LDS they will occupy
  constexpr int PT = M / TPB;
  R pvx[PT], pvy[PT], pvz[PT];
#pragma unroll
  for (int j = 0; j < PT; j++) {
    const int i = tid + j * TPB;
    pvx[j] = pvy[j] = pvz[j] = (R)0;
    if (i < m) {
      pvx[j] = S.vx[a + i];
      ld_yz(S, a + i, pvy[j], pvz[j]);
    }
  }
  coul_rank_lds<R, PT, TPB>(C, S, a, m, n, L.u.o.list, L.u.o.bend, L.wsum, L.ord);
#pragma unroll
  for (int j = 0; j < PT; j++) {
    const int i = tid + j * TPB;
    if (i < m) {
      L.u.v.vx[i] = pvx[j];
      L.u.v.vy[i] = pvy[j];
      L.u.v.vz[i] = pvz[j];
    }
  }
  __syncthreads();
  R* vx = L.u.v.vx;
  coul_pairs<R>(C, D, s, cell, m, n, [&](int r) -> int { return L.ord[r]; }, [&](int i) -> R& { return vx[i]; },
                LdsVyz<R>{L.u.v.vy, L.u.v.vz}, TPB);
  __syncthreads();
  for (int i = tid; i < m; i += TPB) {
    S.vx[a + i] = L.u.v.vx[i];
    st_yz(S, a + i, L.u.v.vy[i], L.u.v.vz[i]);
  }
}

// one workgroup per cell: cells with MLO < m <= M; LIST: cells above M go to
// the list of the largest class (clist), else they are left to later kernels
template <class R, int M, int TPB, int MLO, bool LIST>
__device__ __forceinline__ void k_coulomb_body(const Consts<R>& C, const Dev<R>& D, Blk B) {
  const uint32_t n = (uint32_t)D.ctr->step_push;
  __shared__ CoulLds<R, M, TPB> L;
  const int N = C.N;
  const int w = B.x;
  if (w >= 3 * N) return;  // batches launch for their largest grid
  const int s = w / N, cell = w - s * N;
  const int32_t a = D.seg[s * (N + 1) + cell];
  const int m = D.seg[s * (N + 1) + cell + 1] - a;
  if (m < 2 || m <= MLO) return;
  if (m > M) {
    if (LIST && threadIdx.x == 0) {
      const int k = atomicAdd(D.ncl, 1);
      if (k < 3 * N) D.clist[k] = w;
    }
    return;
  }
  coul_cell<R, M, TPB>(C, D, L, s, cell, a, m, n);
}

// the cells listed for the largest class, taken by persistent workgroups
// (few cells, and workgroups that need most of a CU's LDS); cells above M go
// to the big-cell list
template <class R, int M, int TPB>
__device__ __forceinline__ void k_coul_large_body(const Consts<R>& C, const Dev<R>& D, Blk B) {
  const uint32_t n = (uint32_t)D.ctr->step_push;
  __shared__ CoulLds<R, M, TPB> L;
  const int N = C.N;
  const int nc = min(*D.ncl, 3 * N);
  for (int u = B.x; u < nc; u += B.n) {
    const int w = D.clist[u];
    const int s = w / N, cell = w - s * N;
    const int32_t a = D.seg[s * (N + 1) + cell];
    const int m = D.seg[s * (N + 1) + cell + 1] - a;
    if (m > M) {
      if (threadIdx.x == 0) {
        const int k = atomicAdd(D.ncoul, 1);
        if (k < 3 * N) D.coul_big[k] = w;
      }
      continue;
    }
    coul_cell<R, M, TPB>(C, D, L, s, cell, a, m, n);
    __syncthreads();  // the next cell reuses the LDS
  }
}

template <class R, int M, int TPB>
__global__ void __launch_bounds__(TPB) k_coul_large(Consts<R> C, Dev<R> D) {
  k_coul_large_body<R, M, TPB>(C, D, Blk{(int)blockIdx.x, (int)gridDim.x});
}

// Batches: the cells listed by every discharge are numbered in one sequence
// (discharge by discharge) and taken by the persistent workgroups of a
// single launch, so that discharges with many such cells share the GPU.
constexpr int BATCH_MAX = 1024;  // discharges of one batched launch

// prefix of the discharges' list lengths in LDS (pre[nd] = total)
template <class R, bool BIG>
__device__ __forceinline__ int batch_list_prefix(const Consts<R>* Cs, const Dev<R>* Ds, int nd, int32_t* pre) {
  if (threadIdx.x == 0) {
    int t = 0;
    for (int i = 0; i < nd; i++) {
      pre[i] = t;
      t += min(BIG ? *Ds[i].ncoul : *Ds[i].ncl, 3 * Cs[i].N);
    }
    pre[nd] = t;
  }
  __syncthreads();
  return pre[nd];
}

__device__ __forceinline__ int batch_list_owner(const int32_t* pre, int nd, int u) {
  int lo = 0, hi = nd;
  while (hi - lo > 1) {
    const int mid = (lo + hi) >> 1;
    if (pre[mid] <= u) lo = mid;
    else hi = mid;
  }
  return lo;
}

template <class R, int M, int TPB>
__global__ void __launch_bounds__(TPB) k_coul_large_b(const Consts<R>* __restrict__ Cs, const Dev<R>* __restrict__ Ds,
                                                      int nd) {
  __shared__ CoulLds<R, M, TPB> L;
  __shared__ int32_t pre[BATCH_MAX + 1];
  const int tot = batch_list_prefix<R, false>(Cs, Ds, nd, pre);
  for (int u = blockIdx.x; u < tot; u += gridDim.x) {
    const int i = batch_list_owner(pre, nd, u);
    const Consts<R>& C = Cs[i];
    const Dev<R>& D = Ds[i];
    const uint32_t n = (uint32_t)D.ctr->step_push;
    const int N = C.N;
    const int w = D.clist[u - pre[i]];
    const int s = w / N, cell = w - s * N;
    const int32_t a = D.seg[s * (N + 1) + cell];
    const int m = D.seg[s * (N + 1) + cell + 1] - a;
    if (m > M) {
      if (threadIdx.x == 0) {
        const int k = atomicAdd(D.ncoul, 1);
        if (k < 3 * N) D.coul_big[k] = w;
      }
      continue;
    }
    coul_cell<R, M, TPB>(C, D, L, s, cell, a, m, n);
    __syncthreads();
  }
}

// (the 1024-thread class asks for eight waves per SIMD, two workgroups per CU)
template <class R, int M, int TPB, int MLO, bool LIST>
__global__ void __launch_bounds__(TPB, TPB == 1024 ? 8 : 1) k_coulomb(Consts<R> C, Dev<R> D) {
  k_coulomb_body<R, M, TPB, MLO, LIST>(C, D, Blk{(int)blockIdx.x, (int)gridDim.x});
}

// the same for a batch of discharges over a 1-D grid (workgroups of discharge i:
// [off[i], off[i + 1]))
template <class R, int M, int TPB, int MLO, bool LIST>
__global__ void __launch_bounds__(TPB) k_coulomb_b(const Consts<R>* __restrict__ Cs, const Dev<R>* __restrict__ Ds,
    const int32_t* __restrict__ off, int nd) {
  Blk b;
  const int i = batch_block(off, nd, b);
  k_coulomb_body<R, M, TPB, MLO, LIST>(Cs[i], Ds[i], b);
}

// cells listed by k_coulomb (more than CoulCap<R>::M particles, at most
// COUL_MAXC): the order goes to the cell array of the sort's other buffer and
// the collisions read and write the store directly
// one listed big cell w (species, cell index), the order kept in global memory
template <class R>
__device__ __forceinline__ void coul_big_cell(const Consts<R>& C, const Dev<R>& D, int w, uint32_t n, uint32_t* h,
                                              uint16_t* list, int32_t* bend, int32_t* wsum) {
  const int N = C.N;
  const int s = w / N, cell = w - s * N;
  const int32_t a = D.seg[s * (N + 1) + cell];
  const int m = D.seg[s * (N + 1) + cell + 1] - a;
  if (m > COUL_MAXC) {
    if (threadIdx.x == 0) atomicOr(&D.ctr->err, ERR_COUL);
    return;
  }
  const Store<R> S = D.st[s];
  int32_t* ordg = D.alt[s].cell;
  coul_rank<R>(C, S, a, m, 4, n, h, list, bend, wsum, nullptr, ordg);
  coul_pairs<R>(C, D, s, cell, m, n, [&](int r) -> int { return ordg[a + r] - a; },
                [&](int i) -> R& { return S.vx[a + i]; }, GlobVyz<R>{S, a}, COUL_TPB);
  __syncthreads();
}

template <class R>
__device__ __forceinline__ void k_coul_big_body(const Consts<R>& C, const Dev<R>& D, Blk B) {
  const uint32_t n = (uint32_t)D.ctr->step_push;
  __shared__ uint32_t h[COUL_MAXC];
  __shared__ uint16_t list[COUL_MAXC];
  __shared__ int32_t bend[COUL_MAXC / 4];
  __shared__ int32_t wsum[COUL_TPB / 64];
  const int nunits = min(*D.ncoul, 3 * C.N);
  for (int u = B.x; u < nunits; u += B.n) coul_big_cell<R>(C, D, D.coul_big[u], n, h, list, bend, wsum);
}

template <class R>
__global__ void __launch_bounds__(COUL_TPB) k_coul_big(Consts<R> C, Dev<R> D) {
  k_coul_big_body<R>(C, D, Blk{(int)blockIdx.x, (int)gridDim.x});
}

// the same for a batch: the big cells of every discharge in one numbering
template <class R>
__global__ void __launch_bounds__(COUL_TPB) k_coul_big_b(const Consts<R>* __restrict__ Cs, const Dev<R>* __restrict__ Ds,
                                                         int nd) {
  __shared__ uint32_t h[COUL_MAXC];
  __shared__ uint16_t list[COUL_MAXC];
  __shared__ int32_t bend[COUL_MAXC / 4];
  __shared__ int32_t wsum[COUL_TPB / 64];
  __shared__ int32_t pre[BATCH_MAX + 1];
  const int tot = batch_list_prefix<R, true>(Cs, Ds, nd, pre);
  for (int u = blockIdx.x; u < tot; u += gridDim.x) {
    const int i = batch_list_owner(pre, nd, u);
    coul_big_cell<R>(Cs[i], Ds[i], Ds[i].coul_big[u - pre[i]], (uint32_t)Ds[i].ctr->step_push, h, list, bend, wsum);
  }
}

// The parts of a binary collision that do not depend on the velocities,
// from the Philox words w: the Gaussian factor of tan(chi/2) (before the
// variance), the isotropic branch's sin and 1 - cos of chi, and the azimuth.
// ta_apply finishes the collision exactly as ta_pair_m does.
template <class R>
struct TaPre {
  R nrm, sti, omci, cph, sph;
};
template <class R>
__device__ __forceinline__ TaPre<R> ta_pre(const Consts<R>& C, uint4 w) {
  TaPre<R> p;
  p.nrm = bm_radius<R>(C, unif<R>(w.x)) * cos2pi<R>(C, unif<R>(w.y));
  const R ct = (R)1 - (R)2 * unif<R>(w.w);
  p.sti = Sqrt((R)1 - ct * ct);
  p.omci = (R)1 - ct;
  sincos2pi<R>(C, unif<R>(w.z), p.sph, p.cph);
  return p;
}
// Every branch of the collision is evaluated and the result selected (the
// same IEEE operations as ta_pair_m for the case taken): a chain that runs on
// one lane is bound by instruction latency, and without divergent control
// flow the square root and reciprocal of u_perp leave its critical path.
// ok = false (or u = 0) leaves both velocities unchanged.
template <class R>
__device__ __forceinline__ void ta_apply(bool ok, R va[3], R vb[3], R cc, R nrm, R sti, R omci, R cph, R sph, R fa,
                                         R fb) {
  const R ux = va[0] - vb[0], uy = va[1] - vb[1], uz = va[2] - vb[2];
  const R up2 = ux * ux + uy * uy;
  const R u2 = up2 + uz * uz;
  const R u = Sqrt(u2);
  const R up = Sqrt(up2);
  const R iup = (R)1 / up;
  const R var = cc / (u2 * u);
  const R d = Sqrt(var) * nrm;
  const R d2 = d * d;
  const R inv = (R)1 / ((R)1 + d2);
  const bool iso = var > (R)1;  // beyond the small-angle model: isotropic
  const R st = iso ? sti : (d + d) * inv;
  const R omc = iso ? omci : (d2 + d2) * inv;
  const R s1 = st * cph, s2 = st * sph;
  const R r = uz * s1, t = u * s2;
  const bool perp = up2 > (R)0;
  R du[3];
  du[0] = perp ? (ux * r - uy * t) * iup - ux * omc : u * s1;
  du[1] = perp ? (uy * r + ux * t) * iup - uy * omc : u * s2;
  du[2] = perp ? -(up * s1) - uz * omc : -(u * omc);
  const bool hit = ok && u2 > (R)0;
#pragma unroll
  for (int k = 0; k < 3; k++) {
    const R na = va[k] + fa * du[k], nb = vb[k] - fb * du[k];
    va[k] = hit ? na : va[k];
    vb[k] = hit ? nb : vb[k];
  }
}

// collisions of the unlike pass staged per chunk of ICH partners
template <class R> struct InterChunk { static constexpr int ICH = sizeof(R) == 4 ? 2048 : 1024; };

// LDS of the unlike pass: the ranking's arrays, then the staged chunk
template <class R>
union InterLds {
  struct {
    uint32_t h[COUL_MAXC];
    uint16_t list[COUL_MAXC];
    int32_t bend[COUL_MAXC / 4];
  } r;
  struct {
    R vx[InterChunk<R>::ICH], vy[InterChunk<R>::ICH], vz[InterChunk<R>::ICH];
    R nrm[InterChunk<R>::ICH], sti[InterChunk<R>::ICH], omci[InterChunk<R>::ICH];
    R cph[InterChunk<R>::ICH], sph[InterChunk<R>::ICH];
    int32_t pos[InterChunk<R>::ICH];
  } c;
};

// Unlike-species Coulomb collisions of one cell, after the like-species pass:
// the pairs (e, O-), (e, O2+), (O-, O2+) in turn.  Every particle of the more
// numerous species of the pair (the first on a tie) collides once, the one of
// rank i with the particle of rank i mod N_min of the other species, in
// increasing i; so a thread per particle of the less numerous species runs
// its partners i = j, j + N_min, ... in that order.  Ranks: each species'
// pairing order (Philox(id, n, 20).x, ties by id), kept in the cell array of
// the sort's other buffer.  Randoms: counter ((q N + cell) 2^32 + i, n, 21).
// The variance of tan(chi/2) is that of Eq. (2) with the reduced mass of the
// pair and the lower density W N_min / (A dx).
//
// When N_min <= COUL_TPB (the long chains: a few particles of one species
// among thousands of the other, as in the sheaths) the partners are taken in
// chunks: the workgroup stages their velocities in LDS and computes the parts
// of each collision that do not depend on velocities, then each chain runs
// through the chunk on LDS alone.  Larger N_min (chains of at most
// COUL_MAXC / COUL_TPB links) collide directly in global memory.
template <class R>
__device__ __forceinline__ void coul_inter_cell(const Consts<R>& C, const Dev<R>& D, int cell, uint32_t n,
                                                InterLds<R>& L, int32_t* wsum) {
  constexpr int ICH = InterChunk<R>::ICH;
  const int N = C.N;
  const int tid = threadIdx.x;
  int32_t a[3];
  int m[3];
#pragma unroll
  for (int s = 0; s < 3; s++) {
    a[s] = D.seg[s * (N + 1) + cell];
    m[s] = D.seg[s * (N + 1) + cell + 1] - a[s];
  }
  if (m[0] > COUL_MAXC || m[1] > COUL_MAXC || m[2] > COUL_MAXC) {
    if (tid == 0) atomicOr(&D.ctr->err, ERR_COUL);
    return;
  }
  // a species meets another only if both are present
  const bool need[3] = {m[0] > 0 && (m[1] > 0 || m[2] > 0), m[1] > 0 && (m[0] > 0 || m[2] > 0),
                        m[2] > 0 && (m[0] > 0 || m[1] > 0)};
#pragma unroll
  for (int s = 0; s < 3; s++)
    if (need[s])
      coul_rank<R>(C, D.st[s], a[s], m[s], 4, n, L.r.h, L.r.list, L.r.bend, wsum, nullptr, D.alt[s].cell, 20);
  constexpr int PA[3] = {0, 0, 1}, PB[3] = {1, 2, 2};
#pragma unroll
  for (int q = 0; q < 3; q++) {
    const int sa = PA[q], sb = PB[q];
    const int na = m[sa], nb = m[sb];
    if (na == 0 || nb == 0) continue;
    const bool abig = na >= nb;
    const int nbig = abig ? na : nb, nsml = abig ? nb : na;
    const int32_t abg = abig ? a[sa] : a[sb], asm_ = abig ? a[sb] : a[sa];
    const R fbig = C.finter[q][abig ? 0 : 1], fsml = C.finter[q][abig ? 1 : 0];
    const R cf = C.cinter[q] * (R)nsml;
    const uint64_t key = (uint64_t)(q * N + cell) << 32;
    const Store<R> SB = D.st[abig ? sa : sb], SS = D.st[abig ? sb : sa];
    const int32_t* ob = D.alt[abig ? sa : sb].cell + abg;
    const int32_t* os = D.alt[abig ? sb : sa].cell + asm_;
    if (nsml <= COUL_TPB) {
      const bool own = tid < nsml;
      int32_t pb = -1;
      R vb[3] = {(R)0, (R)0, (R)0};
      if (own) {
        pb = os[tid];
        if (pb < asm_ || pb >= asm_ + nsml) {  // not a permutation: ids were not unique
          atomicOr(&D.ctr->err, ERR_COUL);
          pb = -1;
        } else {
          vb[0] = SS.vx[pb];
          ld_yz(SS, pb, vb[1], vb[2]);
        }
      }
      for (int c0 = 0; c0 < nbig; c0 += ICH) {
        const int cn = min(ICH, nbig - c0);
        for (int t = tid; t < cn; t += COUL_TPB) {
          const int i = c0 + t;
          int32_t pa = ob[i];
          if (pa < abg || pa >= abg + nbig) {
            atomicOr(&D.ctr->err, ERR_COUL);
            pa = -1;
          }
          L.c.pos[t] = pa;
          R y = (R)0, z = (R)0;
          if (pa >= 0) {
            L.c.vx[t] = SB.vx[pa];
            ld_yz(SB, pa, y, z);
          }
          L.c.vy[t] = y;
          L.c.vz[t] = z;
          const TaPre<R> p = ta_pre<R>(C, rng(C, key | (uint64_t)i, n, 21));
          L.c.nrm[t] = p.nrm;
          L.c.sti[t] = p.sti;
          L.c.omci[t] = p.omci;
          L.c.cph[t] = p.cph;
          L.c.sph[t] = p.sph;
        }
        __syncthreads();
        if (own && pb >= 0) {
          int i = tid >= c0 ? tid : tid + ((c0 - tid + nsml - 1) / nsml) * nsml;
          for (; i < c0 + cn; i += nsml) {
            const int t = i - c0;
            // slots of a failed rank check collide with nothing (their
            // velocities are not written back)
            R va[3] = {L.c.vx[t], L.c.vy[t], L.c.vz[t]};
            ta_apply<R>(L.c.pos[t] >= 0, va, vb, cf, L.c.nrm[t], L.c.sti[t], L.c.omci[t], L.c.cph[t], L.c.sph[t],
                        fbig, fsml);
            L.c.vx[t] = va[0];
            L.c.vy[t] = va[1];
            L.c.vz[t] = va[2];
          }
        }
        __syncthreads();
        for (int t = tid; t < cn; t += COUL_TPB) {
          const int32_t pa = L.c.pos[t];
          if (pa >= 0) {
            SB.vx[pa] = L.c.vx[t];
            st_yz(SB, pa, L.c.vy[t], L.c.vz[t]);
          }
        }
        // the next chunk's staging writes slots only this thread reads here
      }
      if (own && pb >= 0) {
        SS.vx[pb] = vb[0];
        st_yz(SS, pb, vb[1], vb[2]);
      }
    } else {
      for (int j = tid; j < nsml; j += COUL_TPB) {
        const int32_t pb = os[j];
        if (pb < asm_ || pb >= asm_ + nsml) {
          atomicOr(&D.ctr->err, ERR_COUL);
          continue;
        }
        R vb[3];
        vb[0] = SS.vx[pb];
        ld_yz(SS, pb, vb[1], vb[2]);
        for (int i = j; i < nbig; i += nsml) {
          const int32_t pa = ob[i];
          if (pa < abg || pa >= abg + nbig) {
            atomicOr(&D.ctr->err, ERR_COUL);
            continue;
          }
          R va[3];
          va[0] = SB.vx[pa];
          ld_yz(SB, pa, va[1], va[2]);
          ta_pair_m<R>(C, va, vb, cf, key | (uint64_t)i, n, 21, fbig, fsml);
          SB.vx[pa] = va[0];
          st_yz(SB, pa, va[1], va[2]);
        }
        SS.vx[pb] = vb[0];
        st_yz(SS, pb, vb[1], vb[2]);
      }
    }
    wg_global_sync();  // the next pair may take the same particles
  }
}

// the cells of the two sheaths hold the longest chains: workgroup b takes
// cell b/2 from the left electrode (b even) or from the right (b odd), so
// both start in the first wave of workgroups
__device__ __forceinline__ int inter_cell_of(int b, int N) { return (b & 1) ? N - 1 - (b >> 1) : (b >> 1); }

template <class R>
__global__ void __launch_bounds__(COUL_TPB) k_coul_inter(Consts<R> C, Dev<R> D) {
  __shared__ InterLds<R> L;
  __shared__ int32_t wsum[COUL_TPB / 64];
  if (!C.inter) return;
  coul_inter_cell<R>(C, D, inter_cell_of(blockIdx.x, C.N), (uint32_t)D.ctr->step_push, L, wsum);
}

// the same for a batch: blockIdx.y is the discharge, the grid spans the
// largest cell count
template <class R>
__global__ void __launch_bounds__(COUL_TPB) k_coul_inter_b(const Consts<R>* __restrict__ Cs,
                                                           const Dev<R>* __restrict__ Ds) {
  __shared__ InterLds<R> L;
  __shared__ int32_t wsum[COUL_TPB / 64];
  const Consts<R>& C = Cs[blockIdx.y];
  const Dev<R>& D = Ds[blockIdx.y];
  if (!C.inter || (int)blockIdx.x >= C.N) return;
  coul_inter_cell<R>(C, D, inter_cell_of(blockIdx.x, C.N), (uint32_t)D.ctr->step_push, L, wsum);
}

template <class R>
__device__ __forceinline__ void k_coul_reset_body(const Consts<R>& C, const Dev<R>& D) {
  if (threadIdx.x == 0) {
    *D.ncoul = 0;
    *D.ncl = 0;
  }
}

template <class R>
__global__ void k_coul_reset(Consts<R> C, Dev<R> D) {
  k_coul_reset_body<R>(C, D);
}

// the same for a batch of discharges, one per blockIdx.y
template <class R>
__global__ void k_coul_reset_b(const Consts<R>* __restrict__ Cs, const Dev<R>* __restrict__ Ds) {
  k_coul_reset_body<R>(Cs[blockIdx.y], Ds[blockIdx.y]);
}

// the Coulomb pass after a sort: reset of the big-cell list, cells that fit
// in LDS, then the big cells on a persistent grid
template <class R>
inline hipError_t launch_coulomb(const Consts<R>& C, const Dev<R>& D, int ncu, hipStream_t st) {
  constexpr int MB = CoulCap<R>::M;
  hipLaunchKernelGGL(k_coul_reset<R>, dim3(1), dim3(64), 0, st, C, D);
  hipLaunchKernelGGL((k_coulomb<R, COUL_TINY, COUL_TTPB, 0, false>), dim3(3 * C.N), dim3(COUL_TTPB), 0, st, C, D);
  if constexpr (MB > COUL_MID) {
    hipLaunchKernelGGL((k_coulomb<R, COUL_SMALL, COUL_STPB, COUL_TINY, false>), dim3(3 * C.N), dim3(COUL_STPB), 0, st,
                       C, D);
    hipLaunchKernelGGL((k_coulomb<R, COUL_MID, COUL_MTPB, COUL_SMALL, true>), dim3(3 * C.N), dim3(COUL_MTPB), 0, st,
                       C, D);
  } else {
    hipLaunchKernelGGL((k_coulomb<R, COUL_SMALL, COUL_STPB, COUL_TINY, true>), dim3(3 * C.N), dim3(COUL_STPB), 0, st,
                       C, D);
  }
  hipLaunchKernelGGL((k_coul_large<R, MB, COUL_TPB>), dim3(ncu), dim3(COUL_TPB), 0, st, C, D);
  hipLaunchKernelGGL(k_coul_big<R>, dim3(ncu), dim3(COUL_TPB), 0, st, C, D);
  if (C.inter) hipLaunchKernelGGL(k_coul_inter<R>, dim3(C.N), dim3(COUL_TPB), 0, st, C, D);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// launches of one step for a batch of nd discharges: constants and device
// state in device arrays, one launch per kernel.  Kernels that stride a
// discharge's particles or cells use 1-D grids split by offset tables; the
// others use blockIdx.y as the discharge.  per is the largest field template
// parameter of the batch (the field loops check every node against N).
// ---------------------------------------------------------------------------
struct BatchGrids {
  const int32_t* push;  // [nd + 1] workgroup offsets of each discharge
  const int32_t* scat;
  const int32_t* coul;
  const int32_t* big;
  int n_push, n_scat, n_coul, n_big;  // totals
};

template <class R, int PER>
inline void launch_serial_field_b(const Consts<R>* C, const Dev<R>* D, int nd, int do_field, int field_mode,
                                  bool serial, hipStream_t st) {
  if (serial) hipLaunchKernelGGL((k_serial_b<R, PER>), dim3(2, nd), dim3(TAIL_TPB), 0, st, C, D, do_field);
  else hipLaunchKernelGGL((k_field_b<R, PER>), dim3(1, nd), dim3(FIELD_TPB), 0, st, C, D, field_mode);
}

template <class R>
inline hipError_t launch_tail_b(const Consts<R>* C, const Dev<R>* D, int nd, int per, bool serial, int arg,
                                hipStream_t st) {
  switch (per) {
    case 1: launch_serial_field_b<R, 1>(C, D, nd, arg, arg, serial, st); break;
    case 2: launch_serial_field_b<R, 2>(C, D, nd, arg, arg, serial, st); break;
    case 3: launch_serial_field_b<R, 3>(C, D, nd, arg, arg, serial, st); break;
    case 4: launch_serial_field_b<R, 4>(C, D, nd, arg, arg, serial, st); break;
    case 5: launch_serial_field_b<R, 5>(C, D, nd, arg, arg, serial, st); break;
    case 6: case 7: launch_serial_field_b<R, 7>(C, D, nd, arg, arg, serial, st); break;
    default: launch_serial_field_b<R, FIELD_PER_MAX>(C, D, nd, arg, arg, serial, st); break;
  }
  return hipGetLastError();
}

template <class R, class SH>
inline void launch_push_b_sh(const Consts<R>* C, const Dev<R>* D, int nd, const BatchGrids& g, bool elds,
                             hipStream_t st) {
  if (elds) hipLaunchKernelGGL((k_push_b<R, true, SH>), dim3(g.n_push), dim3(SH::TPB), 0, st, C, D, g.push, nd);
  else hipLaunchKernelGGL((k_push_b<R, false, SH>), dim3(g.n_push), dim3(SH::TPB), 0, st, C, D, g.push, nd);
}
// shape: index into the shapes built (SHAPE_TPB, SHAPE_PPT)
template <class R>
inline hipError_t launch_push_b(const Consts<R>* C, const Dev<R>* D, int nd, const BatchGrids& g, bool elds,
                                int shape, hipStream_t st) {
  if (shape == 1) launch_push_b_sh<R, Shape1>(C, D, nd, g, elds, st);
  else if (shape == 2) launch_push_b_sh<R, Shape2>(C, D, nd, g, elds, st);
  else launch_push_b_sh<R, Shape0>(C, D, nd, g, elds, st);
  return hipGetLastError();
}

template <class R>
inline hipError_t launch_sort_b(const Consts<R>* C, const Dev<R>* D, int nd, const BatchGrids& g, hipStream_t st) {
  hipLaunchKernelGGL(k_sort_scan_b<R>, dim3(3, nd), dim3(SCAN_TPB), 0, st, C, D);
  hipLaunchKernelGGL(k_sort_scatter_b<R>, dim3(g.n_scat), dim3(SORT_TPB), 0, st, C, D, g.scat, nd);
  return hipGetLastError();
}

template <class R>
inline hipError_t launch_coulomb_b(const Consts<R>* C, const Dev<R>* D, int nd, const BatchGrids& g, int inter_cells,
                                   hipStream_t st) {
  constexpr int MB = CoulCap<R>::M;
  hipLaunchKernelGGL(k_coul_reset_b<R>, dim3(1, nd), dim3(64), 0, st, C, D);
  // batches of many small discharges have few cells above the small class:
  // those are listed and shared by the persistent largest-class workgroups
  // rather than given a 512-thread launch slot per cell of every discharge
  hipLaunchKernelGGL((k_coulomb_b<R, COUL_TINY, COUL_TTPB, 0, false>), dim3(g.n_coul), dim3(COUL_TTPB), 0, st, C, D,
                     g.coul, nd);
  hipLaunchKernelGGL((k_coulomb_b<R, COUL_SMALL, COUL_STPB, COUL_TINY, true>), dim3(g.n_coul), dim3(COUL_STPB), 0, st,
                     C, D, g.coul, nd);
  hipLaunchKernelGGL((k_coul_large_b<R, MB, COUL_TPB>), dim3(g.n_big), dim3(COUL_TPB), 0, st, C, D, nd);
  hipLaunchKernelGGL(k_coul_big_b<R>, dim3(g.n_big), dim3(COUL_TPB), 0, st, C, D, nd);
  // inter_cells: the largest cell count of the discharges with unlike-species
  // collisions on, 0 if none has them
  if (inter_cells > 0) hipLaunchKernelGGL(k_coul_inter_b<R>, dim3(inter_cells, nd), dim3(COUL_TPB), 0, st, C, D);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// creation: initial load, charge deposit, leapfrog half step back
// ---------------------------------------------------------------------------
template <class R>
__global__ void k_load(Consts<R> C, Dev<R> D, int64_t n_e, int64_t n_n, int64_t n_p) {
  const int64_t id = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t tot = n_e + n_n + n_p;
  if (id >= tot) return;
  int s = 0;
  int64_t i = id;
  if (i >= n_e) {
    i -= n_e;
    s = 1;
    if (i >= n_n) {
      i -= n_n;
      s = 2;
    }
  }
  uint4 w = rng(C, (uint64_t)id, 0xFFFFFFFFu, 0);
  uint4 u = rng(C, (uint64_t)id, 0xFFFFFFFFu, 1);
  const Store<R> st = D.st[s];
  st.id[i] = (uint64_t)id;
  st.cell[i] = (int32_t)(((uint64_t)w.x * (uint64_t)C.N) >> 32);
  st.off[i] = unif<R>(w.y);
  R r1 = bm_radius<R>(C, unif<R>(u.x)), a1 = unif<R>(u.y);
  R r2 = bm_radius<R>(C, unif<R>(u.z)), a2 = unif<R>(u.w);
  st.vx[i] = C.vth0[s] * (r1 * cos2pi<R>(C, a1));
  st_yz(st, i, C.vth0[s] * (r1 * sin2pi<R>(C, a1)), C.vth0[s] * (r2 * cos2pi<R>(C, a2)));
}

template <class R>
__global__ void k_deposit_all(Consts<R> C, Dev<R> D) {
  const int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  int64_t i = g;
  int s = 0;
  while (s < 3 && i >= D.N[s]) {
    i -= D.N[s];
    s++;
  }
  if (s >= 3) return;
  const int32_t cell = D.st[s].cell[i];
  if (cell == DEAD) return;
  deposit_global(D, C.N, s, cell, D.st[s].off[i], 1);
}

template <class R>
__global__ void k_halfkick(Consts<R> C, Dev<R> D) {
  const int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  int64_t i = g;
  int s = 0;
  while (s < 3 && i >= D.N[s]) {
    i -= D.N[s];
    s++;
  }
  if (s >= 3) return;
  const Store<R> st = D.st[s];
  const int32_t c = st.cell[i];
  if (c == DEAD) return;
  const R E0 = D.E2[2 * c], E1 = D.E2[2 * c + 1];
  const R dE = E1 - E0;
  const R tt = st.off[i] * dE;
  const R Ep = E0 + tt;
  const R dv = C.hk[s] * Ep;
  st.vx[i] = st.vx[i] - dv;
}

}  // namespace pic
