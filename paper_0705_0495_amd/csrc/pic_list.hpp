// The per-cell collision list of Sec. II (the pic_gas switch dsmc): every
// sort_every steps, after the sort, the particles of each cell go through the
// collision types (4)-(19) of Table I in the table's order, type (4 + t)
// with the probability of Eq. (1), P = n_j sigma_j u tau, tau = sort_every dt
// for all of them.  Products of a type are placed with canonical ids before
// the next type and take part in the later ones; a partner type sees the
// populations at its start.  Included once by pic.hip after pic_kernels.hpp.
//
// One kernel per group of types that leaves the populations alone (gas types
// of one or all species), and for each partner type three: decisions and
// partner choice, claims (smallest test id per partner), collisions.  Births
// are placed by a one-workgroup kernel after each type that can make them;
// they join the end of their store, where the partner choice of a later type
// finds them (the O- of (15) for (19)); the sort after the pass puts them
// into their cells.
#pragma once
#include "pic_kernels.hpp"

namespace pic {

// the list in the order of Table I: test species, first channel and channel
// count of type (4 + t); a count of 0 marks a partner type
constexpr int LIST_N = 16;
constexpr int LIST_SP[LIST_N] = {0, 1, 2, 0, 0, 0, 0, 0, 0, 0, 1, 0, 1, 1, 0, 0};
constexpr int LIST_CH0[LIST_N] = {0, 14, 18, 1, 5, 6, 7, 8, 9, 12, 17, 10, 15, 16, 11, 13};
constexpr int LIST_NCH[LIST_N] = {1, 1, 1, 4, 1, 1, 1, 1, 1, 0, 0, 1, 1, 1, 1, 0};
constexpr int LIST_TPB = 256;

// random streams of type (4 + t): decision, gas molecule, scattering angles
__host__ __device__ constexpr uint32_t lk_dec(int t) { return 32u + 3u * (uint32_t)t; }
__host__ __device__ constexpr uint32_t lk_gas(int t) { return 33u + 3u * (uint32_t)t; }
__host__ __device__ constexpr uint32_t lk_ang(int t) { return 34u + 3u * (uint32_t)t; }

// constants of the list (host double)
struct ListK {
  double B[LIST_N];    // gas type: the largest probability, tau n_target max(sum sigma g)
  double PGl[NCH];     // gas channel: tau n_target
  double KPl;          // tau W / (A dx): Eq. (1) per partner particle of the cell and unit sigma g
  double KM[3];        // KPl M_j of the partner channels 12, 13, 17
};

struct ListLds {
  int32_t ev[NCH];
  int32_t tophits, nreq, nacc;
};

__device__ inline void list_init(ListLds& G) {
  if (threadIdx.x < NCH) G.ev[threadIdx.x] = 0;
  if (threadIdx.x == 0) G.tophits = G.nreq = G.nacc = 0;
}

template <class R>
__device__ inline void list_flush(const Dev<R>& D, ListLds& G) {
  const int tid = threadIdx.x;
  if (tid < NCH && G.ev[tid]) atomicAdd((unsigned long long*)&D.ctr->events[tid], (unsigned long long)G.ev[tid]);
  if (tid == 0) {
    if (G.tophits) atomicAdd((unsigned long long*)&D.ctr->tophits, (unsigned long long)G.tophits);
    if (G.nreq) atomicAdd((unsigned long long*)&D.ctr->nreq, (unsigned long long)G.nreq);
    if (G.nacc) atomicAdd((unsigned long long*)&D.ctr->nacc, (unsigned long long)G.nacc);
  }
}

// the step whose end the pass belongs to (k_serial has advanced the counter)
template <class R>
__device__ __forceinline__ uint32_t list_step(const Dev<R>& D) {
  return (uint32_t)(D.ctr->step - 1);
}

// One gas type t of species S for one particle whose decision uniform U
// (stream lk_dec(t)) is below the type's largest probability: a molecule from
// the Maxwellian at T_gas, then the channels of the type in order against U.
// Returns false when the particle is consumed; moved is set when it collided.
// (t is a constant wherever this is inlined: the callers' loops unroll.)
template <class R, int S>
__device__ __forceinline__ bool list_gas(const Consts<R>& C, const Dev<R>& D, const ListK& K, ListLds& G, int t,
                                         int cell, R off, uint64_t id, R v[3], uint32_t n, double U, bool& moved) {
  const int J0 = LIST_CH0[t], NC = LIST_NCH[t];
  const uint4 u = rng(C, id, n, lk_gas(t));
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
  double cum = 0.0;
  int hit = -1;
#pragma unroll
  for (int q = 0; q < NC; q++) {
    const int j = J0 + q;
    R sg = 0;
    if (Erel >= C.thr[j]) sg = sig_at(D.sig, TS, j, Lk) * g;
    cum = cum + K.PGl[j] * (double)sg;
    if (hit < 0 && U < cum) hit = j;
  }
  if (hit < 0) return true;
  atomicAdd(&G.ev[hit], 1);
  moved = true;
  return gas_event<R, S>(C, D, hit, cell, off, id, v, vt, g, Erel, n, lk_ang(t));
}

// The gas types Ts... (in order) for every alive particle of species S.  The
// decision uniforms of all the types are drawn first (independent streams,
// so their generators overlap); a particle below none of the bounds is done
// without reading its velocity.
template <class R, int S, int... Ts>
__device__ __forceinline__ void list_species(const Consts<R>& C, const Dev<R>& D, const ListK& K, ListLds& G,
                                             uint32_t n) {
  constexpr int NT = sizeof...(Ts);
  constexpr int TT[NT] = {Ts...};
  const Store<R> st = D.st[S];
  const int64_t Ns = D.N[S];
  const int64_t step = (int64_t)gridDim.x * blockDim.x;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < Ns; i += step) {
    const int cell = st.cell[i];
    if (cell == DEAD) continue;
    const uint64_t id = st.id[i];
    double U[NT];
    bool any = false;
#pragma unroll
    for (int q = 0; q < NT; q++) {
      const uint4 w = rng(C, id, n, lk_dec(TT[q]));
      U[q] = unif52(w.x, w.y);
      any = any || U[q] < K.B[TT[q]];
    }
    if (!any) continue;
    const R off = st.off[i];
    R v[3];
    v[0] = st.vx[i];
    ld_yz(st, i, v[1], v[2]);
    bool moved = false, alive = true;
#pragma unroll
    for (int q = 0; q < NT; q++) {
      if (alive && U[q] < K.B[TT[q]]) alive = list_gas<R, S>(C, D, K, G, TT[q], cell, off, id, v, n, U[q], moved);
    }
    if (!alive) {
      st.cell[i] = DEAD;
      deposit_global(D, C.N, S, cell, off, -1);
    } else if (moved) {
      st.vx[i] = v[0];
      st_yz(st, i, v[1], v[2]);
    }
  }
}

// types (4)-(12): elastic and energy-loss scattering of all species, which
// neither make nor remove particles
template <class R>
__global__ void __launch_bounds__(LIST_TPB) k_list_scatter(const Consts<R>* __restrict__ Cp,
                                                           const Dev<R>* __restrict__ Dp, ListK K) {
  const Consts<R>& C = *Cp;
  const Dev<R>& D = *Dp;
  __shared__ ListLds G;
  list_init(G);
  __syncthreads();
  const uint32_t n = list_step(D);
  list_species<R, 0, 0, 3, 4, 5, 6, 7, 8>(C, D, K, G, n);
  list_species<R, 1, 1>(C, D, K, G, n);
  list_species<R, 2, 2>(C, D, K, G, n);
  __syncthreads();
  list_flush(D, G);
}

// one gas type T that can make or remove particles: (15), (16), (17), (18)
template <class R, int T>
__global__ void __launch_bounds__(LIST_TPB) k_list_gas(const Consts<R>* __restrict__ Cp,
                                                       const Dev<R>* __restrict__ Dp, ListK K) {
  const Consts<R>& C = *Cp;
  const Dev<R>& D = *Dp;
  __shared__ ListLds G;
  list_init(G);
  __syncthreads();
  list_species<R, LIST_SP[T], T>(C, D, K, G, list_step(D));
  __syncthreads();
  list_flush(D, G);
}

// partner type T: species of the partner, index of the channel among 12, 13, 17
template <int T> struct ListPair {
  static constexpr int S = LIST_SP[T], J = LIST_CH0[T];
  static constexpr int P = (J == 13) ? 1 : 2;
  static constexpr int PI = (J == 12) ? 0 : (J == 13 ? 1 : 2);
};

// Partner type T, decisions: each alive test particle draws its uniform;
// below N_t(c) KPl M_j (N_t(c) the partners alive in its cell now) it takes
// the partner of its cell with the smallest hash of the two ids (the cell's
// segment of the last sort and the partners born since, dead ones skipped)
// and accepts with U < N_t(c) KPl sigma g.  Accepted requests go to the list
// and reset their partner's claim word (the id array of the partner
// species' idle sort buffer).  The waves walk the test particles 64 at a time; a wave scans the
// segment of each of its requests with all its lanes (a segment holds
// thousands of partners in a dense discharge) and reduces the keys by
// shuffles (keys end in the partner id, so they are distinct).
template <class R, int T>
__global__ void __launch_bounds__(LIST_TPB) k_list_pick(const Consts<R>* __restrict__ Cp,
                                                        const Dev<R>* __restrict__ Dp, ListK K) {
  using PT = ListPair<T>;
  const Consts<R>& C = *Cp;
  const Dev<R>& D = *Dp;
  __shared__ ListLds G;
  list_init(G);
  __syncthreads();
  const uint32_t n = list_step(D);
  const int N = C.N;
  const int lane = threadIdx.x & 63;
  const Store<R> st = D.st[PT::S], ps = D.st[PT::P];
  uint64_t* claim = D.alt[PT::P].id;
  const int32_t* cnt = D.cnt + (size_t)PT::P * N;
  const int32_t* seg = D.seg + (size_t)PT::P * (N + 1);
  const int64_t Ns = D.N[PT::S];
  const int64_t tail0 = seg[N], Np = D.N[PT::P];  // partners placed since the sort: [tail0, Np)
  const int64_t wave = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) >> 6;
  const int64_t nwaves = ((int64_t)gridDim.x * blockDim.x) >> 6;
  for (int64_t base = wave * 64; base < Ns; base += nwaves * 64) {
    const int64_t i = base + lane;
    int cell = DEAD;
    uint64_t id = 0;
    double U = 0.0, Nt = 0.0;
    bool want = false;
    if (i < Ns) cell = st.cell[i];
    if (cell != DEAD) {
      Nt = (double)cnt[cell];
      if (Nt * K.KM[PT::PI] > 1.0) {
        atomicOr(&D.ctr->err, ERR_PMAX);
      } else {
        id = st.id[i];
        const uint4 w = rng(C, id, n, lk_dec(T));
        U = unif52(w.x, w.y);
        want = U < Nt * K.KM[PT::PI];
      }
    }
    uint64_t pending = __ballot(want);
    while (pending) {
      const int leader = __ffsll((unsigned long long)pending) - 1;
      pending &= pending - 1;
      const int lc = __shfl(cell, leader);
      const uint64_t lid = __shfl(id, leader);
      uint64_t best = ~0ull;
      int32_t b = -1;
      for (int32_t k = seg[lc] + lane; k < seg[lc + 1]; k += 64) {
        if (ps.cell[k] == DEAD) continue;
        const uint64_t key = pick_key(C, ps.id[k], lid, n);
        if (key < best) {
          best = key;
          b = k;
        }
      }
      // partners born since the sort (the O- of (15) for (19)) follow the
      // sorted stores, in any cell
      for (int64_t k = tail0 + lane; k < Np; k += 64) {
        if (ps.cell[k] != lc) continue;
        const uint64_t key = pick_key(C, ps.id[k], lid, n);
        if (key < best) {
          best = key;
          b = (int32_t)k;
        }
      }
#pragma unroll
      for (int d = 32; d > 0; d >>= 1) {
        const uint64_t ok = __shfl_xor(best, d);
        const int32_t ob = __shfl_xor(b, d);
        if (ok < best) {
          best = ok;
          b = ob;
        }
      }
      if (lane != leader) continue;
      atomicAdd(&G.nreq, 1);
      if (b < 0) continue;
      R ty, tz, py, pz;
      ld_yz(st, i, ty, tz);
      ld_yz(ps, b, py, pz);
      const R gx = st.vx[i] - ps.vx[b], gy = ty - py, gz = tz - pz;
      const R g2 = (gx * gx + gy * gy) + gz * gz;
      const R g = Sqrt(g2);
      const R Erel = C.hmu_c[PT::PI] * g2;
      R sg = 0;
      if (Erel >= C.thr[PT::J]) sg = sig_at(D.sig, TS, PT::J, lookup(Erel)) * g;
      if (!(U < (Nt * K.KPl) * (double)sg)) continue;
      const int r = atomicAdd(D.nreq, 1);
      if (r < D.lreq_cap) {
        Request<R> q;
        q.sp = PT::S;
        q.chan = PT::J;
        q.slot = (int32_t)i;
        q.cell = cell;
        q.id = id;
        q.u_acc = (R)0;
        q.partner = b;
        q.acc = 0;
        D.lreq[r] = q;
        claim[b] = ~0ull;
      } else {
        atomicOr(&D.ctr->err, ERR_REQ);
      }
    }
  }
  __syncthreads();
  list_flush(D, G);
}

// claims: the smallest test id per partner
template <class R, int T>
__global__ void __launch_bounds__(LIST_TPB) k_list_claim(const Dev<R>* __restrict__ Dp) {
  const Dev<R>& D = *Dp;
  uint64_t* claim = D.alt[ListPair<T>::P].id;
  const int nr = min(*D.nreq, D.lreq_cap);
  for (int r = blockIdx.x * blockDim.x + threadIdx.x; r < nr; r += gridDim.x * blockDim.x) {
    const Request<R>& q = D.lreq[r];
    atomicMin((unsigned long long*)&claim[q.partner], (unsigned long long)q.id);
  }
}

// collisions of the winners: (13) and (14) remove both, (19) splits the O-
template <class R, int T>
__global__ void __launch_bounds__(LIST_TPB) k_list_apply(const Consts<R>* __restrict__ Cp,
                                                         const Dev<R>* __restrict__ Dp) {
  using PT = ListPair<T>;
  const Consts<R>& C = *Cp;
  const Dev<R>& D = *Dp;
  __shared__ ListLds G;
  list_init(G);
  __syncthreads();
  const uint32_t n = list_step(D);
  const uint64_t* claim = D.alt[PT::P].id;
  const int nr = min(*D.nreq, D.lreq_cap);
  for (int r = blockIdx.x * blockDim.x + threadIdx.x; r < nr; r += gridDim.x * blockDim.x) {
    const Request<R> q = D.lreq[r];
    if (claim[q.partner] != q.id) continue;
    atomicAdd(&G.nacc, 1);
    atomicAdd(&G.ev[PT::J], 1);
    if constexpr (PT::J == 13) {
      impact_detach(C, D, q.slot, q.partner, q.id, n, lk_ang(T));
    } else {
      kill_particle(C, D, PT::S, q.slot);
      kill_particle(C, D, PT::P, q.partner);
    }
  }
  __syncthreads();
  list_flush(D, G);
}

// the births of the last type: canonical ids, appended to the stores; the
// request list is emptied
template <class R>
__global__ void __launch_bounds__(TAIL_TPB) k_list_commit(const Consts<R>* __restrict__ Cp,
                                                          const Dev<R>* __restrict__ Dp) {
  const Consts<R>& C = *Cp;
  const Dev<R>& D = *Dp;
  __shared__ int32_t cur[NBUCKET];
  __shared__ int32_t part[TAIL_TPB];
  __shared__ uint64_t bkeys[BKEYS];
  births_phase(C, D, cur, part, bkeys);
  __syncthreads();
  if (threadIdx.x == 0) close_births(D);
}

}  // namespace pic
