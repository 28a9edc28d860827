// Device code of the cn library (gfx950).
//
// One launch of cn_interval advances every cell group through one chunk of a minimum-delay interval (at most M
// steps). Cells exchange spikes only once per interval because every NetCon delay is at least M steps (Sec. 2), so
// a workgroup can keep its group's voltages, synaptic conductances and the interval's events on chip for the whole
// chunk and loop the per-step operations of Sec. 2 itself:
//   A  deliver the events due at this step (sorted keys in LDS; one thread per synapse run, in key order);
//   C  per compartment: advance the channel states with v_n (the state update of the previous step, done here so
//      the states are read and written once per step), then the currents and analytic conductances at
//      (v_n, states_n) into d and rhs (Sec. 2 matrix assembly; Sec. 3.5 CONDUCTANCE), point processes, background
//      events drawn from a counter-based stream (Sec. 3.5, Random123), and the compartment's own axial terms;
//   T  elimination from the leaves, one tree level at a time: each node gathers its children's contributions from
//      LDS, then publishes its own (Sec. 2, Gaussian elimination of the tree; Sec. 4.4 constant-depth ordering);
//   R  the roots: solve, update v, threshold detection (Sec. 2);
//   B  back-substitution root to leaves, one level at a time, updating v.
// At the end of the chunk the group's spikes fan out through their NetCons into the event ring (the spike exchange
// of Sec. 2, here on one device).
#include <hip/hip_runtime.h>

#include "cn_internal.h"

namespace cn {

// ------------------------------------------------------------------------------------------------------------------
// Background events: Philox4x32-10 (Salmon, Moraes, Dror, Shaw, SC'11), ten rounds of two 32x32->64 multiplies
// that mix the counter under a key bumped by Weyl constants. The event of (synapse stream k, step n) is word n % 4
// of Philox(counter = (k lo, k hi, n/4 lo, n/4 hi), key = (seed lo, seed hi)) below the rate threshold, so one call
// serves four consecutive steps (bg_mask4 below).

// ------------------------------------------------------------------------------------------------------------------
// Mechanism kinetics. S is the state type: double on the FP64 path, float on the FP32-mechanism path (rates and
// exponentials in float with the hardware exp; voltage, currents, assembly and solve stay double).
template <typename S>
struct Math;
template <>
struct Math<double> {
  static __device__ __forceinline__ double ex(double x) { return exp(x); }
  // reciprocal: hardware estimate refined by two Newton steps (error within an ulp or two of 1/x)
  static __device__ __forceinline__ double rcp(double x) {
    double r = __builtin_amdgcn_rcp(x);
    double e = fma(-x, r, 1.0);
    r = fma(r, e, r);
    e = fma(-x, r, 1.0);
    return fma(r, e, r);
  }
  // 1 - exp(-z)
  static __device__ __forceinline__ double omx(double z) { return 1.0 - exp(-z); }
};
template <>
struct Math<float> {
  static __device__ __forceinline__ float ex(float x) { return __expf(x); }
  static __device__ __forceinline__ float rcp(float x) { return __builtin_amdgcn_rcpf(x); }
  // 1 - exp(-z) without the cancellation of the subtraction at small z (four-term series below 0.03)
  static __device__ __forceinline__ float omx(float z) {
    return z < 0.03f ? z * (1.0f - z * 0.5f * (1.0f - z * (1.0f / 3.0f) * (1.0f - 0.25f * z))) : 1.0f - __expf(-z);
  }
};

__device__ __forceinline__ double rcp64(double x) { return Math<double>::rcp(x); }

constexpr double E_NEG_1P5 = 0.22313016014842982893;  // exp(-1.5)
constexpr double E_POS_0P5 = 1.64872127070012814685;  // exp(0.5)

// Hodgkin-Huxley gates, exponential relaxation toward x_inf(v) over dt with v frozen.
template <typename S>
__device__ __forceinline__ void hh_advance(double vd, S q10dt, S &m, S &h, S &n) {
  using M = Math<S>;
  const S v = (S)vd;
  const S u = v + S(40);
  const S xm = -u * S(0.1);  // -(v+40)/10
  const S e40 = M::ex(xm);
  const S am = fabs(xm) < S(1e-6) ? S(1) * (S(1) - xm * S(0.5)) : S(0.1) * (-u) * M::rcp(e40 - S(1));
  const S xn = xm - S(1.5);  // -(v+55)/10
  const S en = e40 * S(E_NEG_1P5);
  const S an = fabs(xn) < S(1e-6) ? S(0.1) * (S(1) - xn * S(0.5)) : S(0.01) * (-(u + S(15))) * M::rcp(en - S(1));
  const S bh = M::rcp(e40 * S(E_POS_0P5) + S(1));
  const S w = v + S(65);
  const S bm = S(4) * M::ex(w * S(-1.0 / 18.0));
  const S e80 = M::ex(w * S(-1.0 / 80.0));
  const S e20 = (e80 * e80) * (e80 * e80);
  const S ah = S(0.07) * e20;
  const S bn = S(0.125) * e80;
  const S sm = am + bm, sh = ah + bh, sn = an + bn;
  m += M::omx(q10dt * sm) * (am * M::rcp(sm) - m);
  h += M::omx(q10dt * sh) * (ah * M::rcp(sh) - h);
  n += M::omx(q10dt * sn) * (an * M::rcp(sn) - n);
}

// slow K: n_inf = 1/(1+exp(-(v+35)/10)), tau = 400/(3.3 exp((v+35)/20) + exp(-(v+35)/20)) ms
template <typename S>
__device__ __forceinline__ void km_advance(double vd, S dt, S &n) {
  using M = Math<S>;
  const S u = (S)vd + S(35);
  const S e = M::ex(u * S(0.05));
  const S ei = M::rcp(e);
  const S ninf = M::rcp(S(1) + ei * ei);
  const S z = dt * S(1.0 / 400.0) * (S(3.3) * e + ei);
  n += M::omx(z) * (ninf - n);
}

// high-threshold Ca: m_inf = 1/(1+exp(-(v+20)/9)), tau_m 1 ms; shell calcium relaxing toward
// cai0 - k tau_r ica with ica taken at the new m.
template <typename S>
__device__ __forceinline__ void cahi_advance(double vd, S fm, S fr, S kk, S gca, S &m, S &cai) {
  using M = Math<S>;
  const S v = (S)vd;
  const S minf = M::rcp(S(1) + M::ex((v + S(20)) * S(-1.0 / 9.0)));
  m += fm * (minf - m);
  const S ica = gca * m * m * (v - S(120));
  cai += fr * (S(5e-5) - kk * ica - cai);
}

template <typename S>
__device__ __forceinline__ S ld(const void *p, int64_t i) {
  return static_cast<const S *>(p)[i];
}
template <typename S>
__device__ __forceinline__ void stv(void *p, int64_t i, S x) {
  static_cast<S *>(p)[i] = x;
}

__device__ __forceinline__ uint32_t ev_syn(uint64_t k) { return (uint32_t)(k >> EV_SYN_SHIFT) & EV_SYN_MASK; }

// background-event bits of synapse stream `key` for the four steps 4*blk .. 4*blk+3
__device__ __forceinline__ uint32_t bg_mask4(uint64_t seed, uint64_t key, uint64_t blk, uint64_t thresh) {
  uint32_t c0 = (uint32_t)key, c1 = (uint32_t)(key >> 32), c2 = (uint32_t)blk, c3 = (uint32_t)(blk >> 32);
  uint32_t k0 = (uint32_t)seed, k1 = (uint32_t)(seed >> 32);
#pragma unroll
  for (int r = 0; r < 10; ++r) {
    const uint32_t lo0 = 0xD2511F53u * c0, hi0 = __umulhi(0xD2511F53u, c0);
    const uint32_t lo1 = 0xCD9E8D57u * c2, hi1 = __umulhi(0xCD9E8D57u, c2);
    const uint32_t n0 = hi1 ^ c1 ^ k0, n2 = hi0 ^ c3 ^ k1;
    c0 = n0;
    c1 = lo1;
    c2 = n2;
    c3 = lo0;
    k0 += 0x9E3779B9u;
    k1 += 0xBB67AE85u;
  }
  return ((uint64_t)c0 < thresh ? 1u : 0u) | ((uint64_t)c1 < thresh ? 2u : 0u) | ((uint64_t)c2 < thresh ? 4u : 0u) |
         ((uint64_t)c3 < thresh ? 8u : 0u);
}

// one node of the elimination: gather the children's contributions, then publish this node's own
__device__ __forceinline__ void tri_node(int q, double a, double b, uint32_t ch, double *w_l, double *u_l, double *P_l,
                                         double *Q_l) {
  double d = w_l[q], rhs = u_l[q];
  const int c0 = (int)(ch & 0xFFFFu), cn = (int)(ch >> 16);
  for (int c = c0; c < c0 + cn; ++c) {
    d -= P_l[c];
    rhs -= Q_l[c];
  }
  const double ri = rcp64(d);
  const double w = ri * b, u = ri * rhs;
  w_l[q] = w;
  u_l[q] = u;
  P_l[q] = a * (w + 1.0);
  Q_l[q] = a * (u - Q_l[q]);
}

struct SolveNode {
  int q;
  uint32_t ch;
  double a, b;
};

// the node thread t handles at level L of the elimination (q >= the level's end when there is none)
__device__ __forceinline__ SolveNode solve_node(const KParams &p, int64_t nb, const int *lv, int L, int t) {
  SolveNode r{0x7FFFFFFF, 0u, 0.0, 0.0};
  if (L >= 1) {
    r.q = lv[L] + t;
    if (r.q < lv[L + 1]) {
      const NodeRec nr = p.nrec[nb + r.q];
      r.a = nr.a;
      r.b = nr.b;
      r.ch = p.nidx[nb + r.q].ch;
    }
  }
  return r;
}

// parent of the node thread t handles at level L of the substitution (0 when there is none)
__device__ __forceinline__ int par_of(const KParams &p, int64_t nb, const int *lv, int D, int L, int t) {
  if (L < D) {
    const int q = lv[L] + t;
    if (q < lv[L + 1]) return p.nidx[nb + q].par;
  }
  return 0;
}

// ------------------------------------------------------------------------------------------------------------------
// LDS: four rows of nmax doubles per group -
//   w_l  d (diagonal) after assembly, then w = b/d after elimination;
//   u_l  rhs after assembly, then u = rhs/d after elimination;
//   P_l  the node's contribution a(w + 1) to its parent's diagonal, later the solution x = Delta v;
//   Q_l  dv = v_parent - v after assembly (v itself at a root), then the contribution a(u - dv) to the parent's rhs.
// With these, elimination of node i reads d_i, rhs_i and its children's contributions, and back-substitution is
// x_i = u_i - w_i x_parent.
// The membrane potential stays in global memory, double-buffered across steps: step k of a chunk reads v_{k-1}
// from one buffer, adds the pending Delta v still held in P_l, and writes v_k to the other buffer, so a child reading
// its parent's potential never races the parent's own update. The chunk's last Delta v is applied at its end.
template <int T, typename S>
__global__ void __launch_bounds__(T, 4) cn_interval(const KParams p) {
  extern __shared__ __align__(16) unsigned char lds[];
  const int NMAX = p.nmax;
  double *w_l = reinterpret_cast<double *>(lds);
  double *u_l = w_l + NMAX;
  double *P_l = u_l + NMAX;
  double *Q_l = P_l + NMAX;
  uint64_t *ev = reinterpret_cast<uint64_t *>(lds + p.lds_ev_off);
  int *seg = reinterpret_cast<int *>(lds + p.lds_seg_off);
  int *lv = reinterpret_cast<int *>(lds + p.lds_lvl_off);
  uint8_t *bgm = reinterpret_cast<uint8_t *>(lds + p.lds_bg_off);
  int *misc = reinterpret_cast<int *>(lds + p.lds_misc_off);
  double *cst = reinterpret_cast<double *>(lds + p.lds_cst_off);

  const int G = blockIdx.x;
  const int t = threadIdx.x;
  const GroupDesc gd = p.groups[G];
  const int64_t n_begin = p.ctl[0];
  const int64_t n_target = p.ctl[1];
  const int M = p.M;
  const int64_t ival = n_begin / M;
  const int64_t n_end = min(n_target, (ival + 1) * (int64_t)M);
  if (n_end <= n_begin) return;
  const int slot = (int)(ival % p.ring);
  const int N = gd.n_nodes;
  const int D = gd.n_levels;
  const int n_syn = gd.n_syn;
  const int64_t nb = gd.node_base;
  const int64_t sb = gd.syn_base;

  // ---- prologue: level starts on chip, this interval's events sorted
  for (int L = t; L <= D; L += T) lv[L] = p.lvl_start[gd.lvl_base + L];
  if (t < N_PRM) cst[C_PRM + t] = p.prm_s[t];
  if (t == 0) {
    cst[C_Q10DT] = p.q10dt;
    cst[C_DT] = p.dt;
    cst[C_CA_FM] = p.ca_fm;
    cst[C_CA_FR] = p.ca_fr;
    cst[C_CA_K] = p.ca_k;
    int lo = gd.kick_base, hi = gd.kick_base + gd.n_kick;
    int a = lo, b = hi;  // first kick with step >= n_begin
    while (a < b) {
      const int mid = (a + b) >> 1;
      if (p.kick_step[mid] < n_begin) a = mid + 1; else b = mid;
    }
    int c = a, e = hi;  // first kick with step >= n_end
    while (c < e) {
      const int mid = (c + e) >> 1;
      if (p.kick_step[mid] < n_end) c = mid + 1; else e = mid;
    }
    int nbk = p.ev_cnt[(int64_t)slot * p.n_groups + G];
    if (nbk > p.ev_cap) {
      nbk = p.ev_cap;
      atomicOr(&p.flags[FLAG_EV_OVERFLOW], 1);
    }
    int nk = c - a;
    if (nbk + nk > p.ev_cap) {
      nk = p.ev_cap - nbk;
      atomicOr(&p.flags[FLAG_EV_OVERFLOW], 1);
    }
    misc[0] = nbk;
    misc[1] = 0;  // spikes of this chunk
    misc[2] = a;
    misc[3] = nk;
  }
  __syncthreads();
  const int nbk = misc[0], k0 = misc[2], nk = misc[3];
  const int n_ev = nbk + nk;
  int P = 1;
  while (P < n_ev) P <<= 1;
  {
    const uint64_t *bucket = p.ev_key + ((int64_t)slot * p.n_groups + G) * p.ev_cap;
    for (int i = t; i < P; i += T) {
      uint64_t key = ~0ull;
      if (i < nbk) {
        key = bucket[i];
      } else if (i < n_ev) {
        const int kq = k0 + (i - nbk);
        const uint64_t ss = (uint64_t)(p.kick_step[kq] - ival * M);
        key = (ss << EV_STEP_SHIFT) | ((uint64_t)(uint32_t)p.kick_lsyn[kq] << EV_SYN_SHIFT) | (uint32_t)p.kick_id[kq];
      }
      ev[i] = key;
    }
  }
  __syncthreads();
  for (int k = 2; k <= P; k <<= 1) {  // bitonic sort of the keys
    for (int j = k >> 1; j > 0; j >>= 1) {
      for (int i = t; i < P; i += T) {
        const int ixj = i ^ j;
        if (ixj > i) {
          const uint64_t x = ev[i], y = ev[ixj];
          const bool up = (i & k) == 0;
          if (up ? (x > y) : (x < y)) {
            ev[i] = y;
            ev[ixj] = x;
          }
        }
      }
      __syncthreads();
    }
  }
  for (int s = t; s <= M; s += T) {  // first event of each step
    const uint64_t target = (uint64_t)s << EV_STEP_SHIFT;
    int a = 0, b = n_ev;
    while (a < b) {
      const int mid = (a + b) >> 1;
      if (ev[mid] < target) a = mid + 1; else b = mid;
    }
    seg[s] = a;
  }
  __syncthreads();

  StRec<S> *st = static_cast<StRec<S> *>(p.st);
  const int64_t sst = p.n_nodes_total;
  const SynRec<S> *syn = static_cast<const SynRec<S> *>(p.syn) + sb;
  S *sg = static_cast<S *>(p.syn_g) + sb;
  double *const vbuf[2] = {p.v2 + nb, p.v + nb};  // step k writes vbuf[k & 1]; p.v holds v between chunks
  const int lv1 = lv[1];
  if (!p.has_bg)
    for (int i = t; i < n_syn; i += T) bgm[i] = 0;

  for (int64_t n = n_begin; n < n_end; ++n) {
    const int s = (int)(n - ival * M);
    // ---- background-event bits for a block of four steps (one Philox call gives four words)
    if (p.has_bg && (n == n_begin || (n & 3) == 0)) {
      const uint64_t blk = (uint64_t)n >> 2;
      for (int i = t; i < n_syn; i += T) bgm[i] = (uint8_t)bg_mask4(p.seed, syn[i].key, blk, p.bg_thresh);
    }
    // ---- A: delivery (Sec. 2, event-driven delivery step): one thread per synapse run, in key order
    const int e0 = seg[s], e1 = seg[s + 1];
    for (int e = e0 + t; e < e1; e += T) {
      const uint32_t ls = ev_syn(ev[e]);
      if (e == e0 || ev_syn(ev[e - 1]) != ls) {
        S g = sg[ls];
        for (int e2 = e; e2 < e1; ++e2) {
          const uint64_t key = ev[e2];
          if (ev_syn(key) != ls) break;
          const uint32_t id = (uint32_t)key & 0x7FFFFFFFu;
          g += ((uint32_t)key & EV_KIND_NETCON) ? ld<S>(p.nc_w, id) : ld<S>(p.kick_w, id);
        }
        sg[ls] = g;
      }
    }
    __syncthreads();
    // ---- C: states, currents, conductances and the compartment's own axial terms
    const bool pend = n > 0;
    const uint32_t bsh = (uint32_t)(n & 3);
    const int kk = (int)(n - n_begin);
    const bool first = kk == 0;
    const double *vr = first ? p.v + nb : vbuf[(kk - 1) & 1];  // v_{k-1} (pending Delta v in P_l unless first)
    double *vw = vbuf[kk & 1];
    const S q10dt = (S)cst[C_Q10DT];
    const S sdt = (S)cst[C_DT];
    const S ca_fm = (S)cst[C_CA_FM], ca_fr = (S)cst[C_CA_FR], ca_k = (S)cst[C_CA_K];
    // records and states of the thread's next compartment are loaded while the current one is computed
    NodeRec nr_n{};
    NodeIdx nx_n{};
    StRec<S> sr_n{};
    double v_n = 0.0;
    if (t < N) {
      nr_n = p.nrec[nb + t];
      nx_n = p.nidx[nb + t];
      sr_n = st[nb + t];
      v_n = vr[t];
    }
#pragma unroll 1
    for (int q = t; q < N; q += T) {
      const int64_t i = nb + q;
      const NodeRec nr = nr_n;
      const NodeIdx nx = nx_n;
      StRec<S> sr = sr_n;
      const double vpar_old = nx.par >= 0 ? vr[nx.par] : 0.0;
      const double v = first ? v_n : v_n + P_l[q];
      if (q + T < N) {
        nr_n = p.nrec[i + T];
        nx_n = p.nidx[i + T];
        sr_n = st[i + T];
        v_n = vr[q + T];
      }
      vw[q] = v;
      double rhs = 0.0, d = 0.0;
      const uint32_t mf = nx.pk >> 24;
      const bool has_st = (mf & (MF_HH | MF_KM | MF_CAHI)) != 0;
      if (pend && has_st) {
        if (mf & MF_HH) hh_advance<S>(v, q10dt, sr.m, sr.h, sr.n);
        if (mf & MF_KM) km_advance<S>(v, sdt, sr.kn);
        if (mf & MF_CAHI) {
          const S gca = (S)(p.prm ? p.prm[P_CA_G * sst + i] : cst[C_PRM + P_CA_G]);
          cahi_advance<S>(v, ca_fm, ca_fr, ca_k, gca, sr.cm, sr.cai);
        }
        st[i] = sr;
      }
      if (mf & MF_HH) {
        const double gnab = p.prm ? p.prm[P_HH_GNA * sst + i] : cst[C_PRM + P_HH_GNA];
        const double gkb = p.prm ? p.prm[P_HH_GK * sst + i] : cst[C_PRM + P_HH_GK];
        const double gl = p.prm ? p.prm[P_HH_GL * sst + i] : cst[C_PRM + P_HH_GL];
        const double el = p.prm ? p.prm[P_HH_EL * sst + i] : cst[C_PRM + P_HH_EL];
        const double gna = (double)((S)gnab * (sr.m * sr.m * sr.m * sr.h));
        const double gk = (double)((S)gkb * ((sr.n * sr.n) * (sr.n * sr.n)));
        rhs -= gna * (v - 50.0) + gk * (v + 77.0) + gl * (v - el);
        d += gna + gk + gl;
      }
      if (mf & MF_PAS) {
        const double g = p.prm ? p.prm[P_PAS_G * sst + i] : cst[C_PRM + P_PAS_G];
        const double e = p.prm ? p.prm[P_PAS_E * sst + i] : cst[C_PRM + P_PAS_E];
        rhs -= g * (v - e);
        d += g;
      }
      if (mf & MF_KM) {
        const double g = (double)((S)(p.prm ? p.prm[P_KM_G * sst + i] : cst[C_PRM + P_KM_G]) * sr.kn);
        rhs -= g * (v + 77.0);
        d += g;
      }
      if (mf & MF_CAHI) {
        const S gca = (S)(p.prm ? p.prm[P_CA_G * sst + i] : cst[C_PRM + P_CA_G]);
        const double g = (double)(gca * (sr.cm * sr.cm));
        rhs -= g * (v - 120.0);
        d += g;
      }
      const int n_icl = (int)((nx.pk >> 16) & 0xFFu);
      if (n_icl) {
        const IclRec *ic = p.icl + gd.icl_base + p.nd_icl0[i];
        for (int c = 0; c < n_icl; ++c)
          if (ic[c].on <= n && n < ic[c].off) rhs += ic[c].cur;
      }
      const int n_s = (int)(nx.pk & 0xFFFFu);
      for (int c = 0; c < n_s; ++c) {
        const int ls = nx.syn0 + c;
        const SynRec<S> sr = syn[ls];
        S g = sg[ls];
        if ((bgm[ls] >> bsh) & 1u) g += sr.wbg;
        const double gs = nr.sa * (double)g;
        rhs -= gs * (v - sr.e);
        d += gs;
        sg[ls] = g * sr.f;  // decay of this step, applied ahead of the next delivery
      }
      d += nr.k;
      double dvq = v;  // a root keeps its own potential here for threshold detection
      if (nx.par >= 0) {
        const double vpar = first ? vpar_old : vpar_old + P_l[nx.par];
        const double dv = vpar - v;
        rhs -= nr.b * dv;
        dvq = dv;
      }
      w_l[q] = d;
      u_l[q] = rhs;
      Q_l[q] = dvq;
    }
    __syncthreads();
    // ---- T: elimination, deepest level first, one thread per node of the level. Each thread's node records for
    // the next three levels are in flight while the current level is processed (they are loop invariant, but
    // too many to keep on chip for the whole chunk).
    const uint32_t root_ch = t < lv1 ? p.nidx[nb + t].ch : 0u;  // roots' children, used after the elimination
    {
      SolveNode c0n, c1n, c2n;
      int Lc = D - 1;
      c0n = solve_node(p, nb, lv, Lc, t);
      c1n = solve_node(p, nb, lv, Lc - 1, t);
      c2n = solve_node(p, nb, lv, Lc - 2, t);
      for (; Lc >= 1; --Lc) {
        const SolveNode cur = c0n;
        c0n = c1n;
        c1n = c2n;
        c2n = solve_node(p, nb, lv, Lc - 3, t);
        const int q = lv[Lc] + t, hi = lv[Lc + 1];
        if (q < hi) tri_node(q, cur.a, cur.b, cur.ch, w_l, u_l, P_l, Q_l);
        for (int q2 = q + T; q2 < hi; q2 += T) {  // levels wider than the group's threads
          const NodeRec r2 = p.nrec[nb + q2];
          tri_node(q2, r2.a, r2.b, p.nidx[nb + q2].ch, w_l, u_l, P_l, Q_l);
        }
        __syncthreads();
      }
    }
    // ---- R: roots (level 0 holds the group's cells in order): solve, v update, threshold detection
    for (int q = t; q < lv1; q += T) {
      const uint32_t ch = q == t ? root_ch : p.nidx[nb + q].ch;
      double d = w_l[q], rhs = u_l[q];
      const int c0 = (int)(ch & 0xFFFFu), cn = (int)(ch >> 16);
      for (int c = c0; c < c0 + cn; ++c) {
        d -= P_l[c];
        rhs -= Q_l[c];
      }
      const double x = rhs / d;
      const double vold = Q_l[q];
      const double vnew = vold + x;
      P_l[q] = x;
      const double th = p.cell_theta[gd.cell_base + q];
      if (vold < th && th <= vnew) {
        const int idx = atomicAdd(&misc[1], 1);
        p.gsp_pack[gd.spk_base + idx] = q | ((s + 1) << 16);
        p.gsp_frac[gd.spk_base + idx] = (th - vold) / (vnew - vold);
      }
      if (!isfinite(vnew)) atomicOr(&p.flags[FLAG_NONFINITE], 1);
    }
    __syncthreads();
    // ---- B: substitution, root to leaves: x = u - w x_parent (parents of the next three levels in flight)
    {
      int p0 = par_of(p, nb, lv, D, 1, t), p1 = par_of(p, nb, lv, D, 2, t), p2 = par_of(p, nb, lv, D, 3, t);
      for (int L = 1; L < D; ++L) {
        const int lo = lv[L], hi = lv[L + 1];
        const int q = lo + t, par = p0;
        p0 = p1;
        p1 = p2;
        p2 = par_of(p, nb, lv, D, L + 3, t);
        if (q < hi) {
          const double x = u_l[q] - w_l[q] * P_l[par];
          P_l[q] = x;
        }
        for (int q2 = q + T; q2 < hi; q2 += T) {
          const double x = u_l[q2] - w_l[q2] * P_l[p.nidx[nb + q2].par];
          P_l[q2] = x;
        }
        __syncthreads();
      }
    }
  }

  // ---- epilogue: apply the last step's Delta v; the chunk's spikes (count in gsp_cnt) are recorded and fanned
  // out by cn_fanout
  {
    const double *vl = vbuf[(int)(n_end - 1 - n_begin) & 1];
    for (int q = t; q < N; q += T) p.v[nb + q] = vl[q] + P_l[q];
  }
  if (t == 0) {
    p.gsp_cnt[G] = misc[1];
    if (n_end == (ival + 1) * (int64_t)M) p.ev_cnt[(int64_t)slot * p.n_groups + G] = 0;
  }
}

// Spike record and fan-out of one chunk (Sec. 2 spike exchange, on one device): each spike walks its source cell's
// NetCons and appends an event key to the ring slot of the interval it is due in. Slots of later intervals only, so
// it never touches the slot the chunk just consumed (every delay is at least one interval).
__global__ void __launch_bounds__(256) cn_fanout(const KParams p) {
  const int G = blockIdx.x;
  const int t = threadIdx.x;
  const int nsp = p.gsp_cnt[G];
  if (nsp == 0) return;
  const GroupDesc gd = p.groups[G];
  const int64_t n_begin = p.ctl[0];
  const int M = p.M;
  const int64_t ival = n_begin / M;
  for (int k = t; k < nsp; k += 256) {
    const int pk = p.gsp_pack[gd.spk_base + k];
    const int q = pk & 0xFFFF;
    const int64_t kstep = ival * M + (pk >> 16);
    const int r = atomicAdd(p.rec_cnt, 1);
    if (r < p.rec_cap) {
      p.rec_gid[r] = p.cell_gid[gd.cell_base + q];
      p.rec_step[r] = kstep;
      p.rec_t[r] = ((double)(kstep - 1) + p.gsp_frac[gd.spk_base + k]) * p.dt;
    } else {
      atomicOr(&p.flags[FLAG_REC_OVERFLOW], 1);
    }
  }
  for (int k = 0; k < nsp; ++k) {
    const int pk = p.gsp_pack[gd.spk_base + k];
    const int q = pk & 0xFFFF;
    const int64_t kstep = ival * M + (pk >> 16);
    const int gid = p.cell_gid[gd.cell_base + q];
    const int64_t o0 = p.out_off[gid], o1 = p.out_off[gid + 1];
    for (int64_t o = o0 + t; o < o1; o += 256) {
      const int nc = p.out_nc[o];
      const int64_t td = kstep + p.nc_D[nc];
      const int64_t it = td / M;
      const int sl = (int)(it % p.ring);
      const uint64_t ss = (uint64_t)(td - it * M);
      const int tg = p.nc_tgt_group[nc];
      const uint64_t key = (ss << EV_STEP_SHIFT) | ((uint64_t)(uint32_t)p.nc_tgt_lsyn[nc] << EV_SYN_SHIFT) |
                           EV_KIND_NETCON | (uint32_t)nc;
      const int64_t b = (int64_t)sl * p.n_groups + tg;
      const int pos = atomicAdd(&p.ev_cnt[b], 1);
      if (pos < p.ev_cap) p.ev_key[b * p.ev_cap + pos] = key;
      else atomicOr(&p.flags[FLAG_EV_OVERFLOW], 1);
    }
  }
}

// next chunk: up to the next interval boundary or the target
__global__ void cn_advance(int64_t *ctl, int32_t M) {
  if (threadIdx.x == 0 && blockIdx.x == 0) {
    const int64_t nb = ctl[0];
    const int64_t nxt = (nb / M + 1) * (int64_t)M;
    ctl[0] = nxt < ctl[1] ? nxt : ctl[1];
  }
}

__global__ void cn_set_ctl(int64_t *ctl, int64_t n_begin, int64_t n_target) {
  if (threadIdx.x == 0 && blockIdx.x == 0) {
    ctl[0] = n_begin;
    ctl[1] = n_target;
  }
}

__global__ void cn_fill_i32(int32_t *p, int64_t n, int32_t v) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    p[i] = v;
}

// mechanism state readout at the current step: states are stored one update behind (the update of the last step
// is applied at the start of the next), so apply it to a copy here.
template <typename S>
__global__ void cn_read_state(const KParams p, int64_t n_nodes, int64_t step, int type, int which, double *out) {
  const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (i >= n_nodes) return;
  const double v = p.v[i];
  const bool pend = step > 0;
  StRec<S> sr = static_cast<const StRec<S> *>(p.st)[i];
  const int64_t sst = p.n_nodes_total;
  if (type == 0) {
    if (pend) hh_advance<S>(v, (S)p.q10dt, sr.m, sr.h, sr.n);
    out[i] = which == 0 ? (double)sr.m : (which == 1 ? (double)sr.h : (double)sr.n);
  } else if (type == 2) {
    if (pend) km_advance<S>(v, (S)p.dt, sr.kn);
    out[i] = (double)sr.kn;
  } else if (type == 3) {
    const S gca = (S)(p.prm ? p.prm[P_CA_G * sst + i] : p.prm_s[P_CA_G]);
    if (pend) cahi_advance<S>(v, (S)p.ca_fm, (S)p.ca_fr, (S)p.ca_k, gca, sr.cm, sr.cai);
    out[i] = which == 0 ? (double)sr.cm : (double)sr.cai;
  }
}

// ------------------------------------------------------------------------------------------------------------------
// launch wrappers (host side)
using IntervalFn = void (*)(const KParams);

static IntervalFn interval_fn(bool fp32, int threads) {
  if (threads == 256) return fp32 ? cn_interval<256, float> : cn_interval<256, double>;
  if (threads == 512) return fp32 ? cn_interval<512, float> : cn_interval<512, double>;
  if (threads == 128) return fp32 ? cn_interval<128, float> : cn_interval<128, double>;
  return nullptr;
}

hipError_t set_interval_lds(bool fp32, int threads, int slots, int lds_bytes) {
  (void)slots;
  IntervalFn fn = interval_fn(fp32, threads);
  if (!fn) return hipErrorInvalidValue;
  return hipFuncSetAttribute(reinterpret_cast<const void *>(fn), hipFuncAttributeMaxDynamicSharedMemorySize,
                             lds_bytes);
}

hipError_t launch_interval(const KParams &p, bool fp32, int threads, int slots, int lds_bytes, hipStream_t st) {
  (void)slots;
  IntervalFn fn = interval_fn(fp32, threads);
  if (!fn) return hipErrorInvalidValue;
  hipLaunchKernelGGL(fn, dim3(p.n_groups), dim3(threads), lds_bytes, st, p);
  return hipGetLastError();
}

hipError_t launch_fanout(const KParams &p, hipStream_t st) {
  hipLaunchKernelGGL(cn_fanout, dim3(p.n_groups), dim3(256), 0, st, p);
  return hipGetLastError();
}

hipError_t launch_advance(int64_t *ctl, int32_t M, hipStream_t st) {
  hipLaunchKernelGGL(cn_advance, dim3(1), dim3(64), 0, st, ctl, M);
  return hipGetLastError();
}

hipError_t launch_set_ctl(int64_t *ctl, int64_t n_begin, int64_t n_target, hipStream_t st) {
  hipLaunchKernelGGL(cn_set_ctl, dim3(1), dim3(64), 0, st, ctl, n_begin, n_target);
  return hipGetLastError();
}

hipError_t launch_fill_i32(int32_t *ptr, int64_t n, int32_t v, hipStream_t st) {
  if (n <= 0) return hipSuccess;
  int64_t blocks = (n + 255) / 256;
  if (blocks > 4096) blocks = 4096;
  hipLaunchKernelGGL(cn_fill_i32, dim3((unsigned)blocks), dim3(256), 0, st, ptr, n, v);
  return hipGetLastError();
}

hipError_t launch_read_state(const KParams &p, bool fp32, int64_t n_nodes, int64_t step, int type, int which,
                             double *out, hipStream_t st) {
  if (n_nodes <= 0) return hipSuccess;
  const unsigned blocks = (unsigned)((n_nodes + 255) / 256);
  if (fp32) hipLaunchKernelGGL(cn_read_state<float>, dim3(blocks), dim3(256), 0, st, p, n_nodes, step, type, which, out);
  else hipLaunchKernelGGL(cn_read_state<double>, dim3(blocks), dim3(256), 0, st, p, n_nodes, step, type, which, out);
  return hipGetLastError();
}

}  // namespace cn
