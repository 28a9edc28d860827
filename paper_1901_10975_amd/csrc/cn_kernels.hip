// Device code of the cn library (gfx950).
//
// One launch of cn_interval advances every cell group through one chunk of a minimum-delay interval (at most M
// steps). Cells exchange spikes only once per interval because every NetCon delay is at least M steps (Sec. 2), so
// a workgroup can keep its group's voltages, synaptic conductances and the interval's events on chip for the whole
// chunk and loop the per-step operations of Sec. 2 itself:
//   A  deliver the events due at this step (sorted keys in LDS; one thread per synapse run, in key order);
//   θ  threshold detection at each cell's soma for the previous step (Sec. 2), whose potentials are still on chip;
//   S  per synapse: conductance and current at v_n staged in LDS;
//   C  per compartment: advance the channel states with v_n (the state update of the previous step, done here so
//      the states are read and written once per step), then the currents and analytic conductances at
//      (v_n, states_n) into d and rhs (Sec. 2 matrix assembly; Sec. 3.5 CONDUCTANCE), point processes, background
//      events drawn from a counter-based stream (Sec. 3.5, Random123), and the compartment's own axial terms;
//   T  elimination from the leaves, one tree level at a time: each node gathers its children's contributions from
//      LDS, then publishes its own (Sec. 2, Gaussian elimination of the tree; Sec. 4.4 constant-depth ordering);
//   R  the roots (each cell rooted at a tree centre): solve, update v;
//   B  back-substitution root to leaves, three levels per barrier, updating v.
// At the end of the chunk the group's spikes fan out through their NetCons into the event ring (the spike exchange
// of Sec. 2, here on one device).
#include <hip/hip_runtime.h>

#include <type_traits>

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
// the exp table lives in LDS; the explicit address space keeps its loads LDS reads after inlining
typedef const __attribute__((address_space(3))) double lds_table;
// exp in double by Tang's table-driven method (ACM TOMS 15(2), 1989): x = (64 m + j) ln2/64 + r with |r| <= ln2/128,
// exp(x) = 2^m 2^(j/64) exp(r), exp(r) - 1 by its Taylor series to r^5 (truncation below 4e-17 relative). The 64
// table values 2^(j/64) sit in LDS (exp_tab). Arguments here are bounded (|x| < 60); no overflow handling.
__device__ __forceinline__ double exp_tang(double x, const lds_table *exp_tab) {
  const double n = __builtin_rint(x * 92.33248261689366);  // 64 / ln 2
  const int ni = (int)n;
  // ln2/64 = hi + lo, hi with its low 12 mantissa bits clear so that n hi is exact
  const double r = fma(-n, 4.411764150473684e-15, fma(-n, 0.010830424696244734, x));
  const double c = fma(fma(fma(r, 1.0 / 120.0, 1.0 / 24.0), r, 1.0 / 6.0), r, 0.5);
  const double pr = fma(r * r, c, r);  // exp(r) - 1
  const double tj = exp_tab[ni & 63];
  return __builtin_ldexp(fma(tj, pr, tj), ni >> 6);
}

template <>
struct Math<double> {
  static __device__ __forceinline__ double ex(double x, const lds_table *et) { return exp_tang(x, et); }
  // reciprocal: the hardware estimate r (relative error eps below 2^-24) corrected to second order. With
  // e = 1 - x r = eps (exact by fma), 1/x = r (1 + e + e^2 + ...), and r (1 + e + e^2) is off by eps^3 before its
  // last rounding: the accuracy of two Newton steps in one operation fewer.
  static __device__ __forceinline__ double rcp(double x) {
    const double r = __builtin_amdgcn_rcp(x);
    const double e = fma(-x, r, 1.0);
    return fma(r, fma(e, e, e), r);
  }
  // 1 - exp(-z)
  static __device__ __forceinline__ double omx(double z, const lds_table *et) { return 1.0 - exp_tang(-z, et); }
  // vtrap(x, y) = y vser(u) near u = x/y = 0: the series 1 - u/2 below |u| = 1e-6 (reading R4)
  static __device__ __forceinline__ double vser(double u) { return 1.0 - u * 0.5; }
  static constexpr double VCUT = 1e-6;
};
template <>
struct Math<float> {
  static __device__ __forceinline__ float ex(float x, const lds_table *) { return __expf(x); }
  static __device__ __forceinline__ float rcp(float x) { return __builtin_amdgcn_rcpf(x); }
  // 1 - exp(-z). Below z = 1/64 the subtraction would cancel (a relative error of ulp(1)/z, the same sign every step
  // for slow gates such as km with z near 3e-4); there the series z (1 - z/2 + z^2/6), whose first omitted term is
  // below 3e-9 relative, is selected without a branch.
  static __device__ __forceinline__ float omx(float z, const lds_table *) {
    const float e = __expf(-z);
    return z < (1.0f / 64.0f) ? z * (1.0f - z * (0.5f - z * (1.0f / 6.0f))) : 1.0f - e;
  }
  // vtrap(x, y) = x / (exp(u) - 1) with u = x/y is y vser(u) near u = 0. In float, exp(u) - 1 loses ulp(1)/|u|
  // relative accuracy, so below |u| = 1/64 the series 1 - u/2 + u^2/12 (first omitted term u^4/720) is used.
  static __device__ __forceinline__ float vser(float u) { return 1.0f - u * (0.5f - u * (1.0f / 12.0f)); }
  static constexpr float VCUT = 1.0f / 64.0f;
};

// reciprocal of the tree solve: the FP64 kernels use Math<double>::rcp; the FP32-mechanism kernels keep two Newton
// steps after the hardware estimate (the same accuracy; measured faster in their instruction mix)
template <typename S>
__device__ __forceinline__ double rcp64(double x) {
  if (std::is_same<S, double>::value) return Math<double>::rcp(x);
  double r = __builtin_amdgcn_rcp(x);
  double e = fma(-x, r, 1.0);
  r = fma(r, e, r);
  e = fma(-x, r, 1.0);
  return fma(r, e, r);
}

constexpr double E_NEG_1P5 = 0.22313016014842982893;  // exp(-1.5)
constexpr double E_POS_0P5 = 1.64872127070012814685;  // exp(0.5)

// Hodgkin-Huxley gates, exponential relaxation toward x_inf(v) over dt with v frozen.
template <typename S>
__device__ __forceinline__ void hh_advance(double vd, S q10dt, S &m, S &h, S &n, const lds_table *et) {
  using M = Math<S>;
  const S v = (S)vd;
  const S u = v + S(40);
  const S xm = -u * S(0.1);  // -(v+40)/10
  const S e40 = M::ex(xm, et);
  // vtrap(x, y) = x / (exp(x/y) - 1), and its series near x = 0 (selected without a branch)
  const S am_s = S(1) * M::vser(xm);
  const S am_e = S(0.1) * (-u) * M::rcp(e40 - S(1));
  const S am = fabs(xm) < M::VCUT ? am_s : am_e;
  const S xn = xm - S(1.5);  // -(v+55)/10
  const S en = e40 * S(E_NEG_1P5);
  const S an_s = S(0.1) * M::vser(xn);
  const S an_e = S(0.01) * (-(u + S(15))) * M::rcp(en - S(1));
  const S an = fabs(xn) < M::VCUT ? an_s : an_e;
  const S bh = M::rcp(e40 * S(E_POS_0P5) + S(1));
  const S w = v + S(65);
  const S bm = S(4) * M::ex(w * S(-1.0 / 18.0), et);
  const S e80 = M::ex(w * S(-1.0 / 80.0), et);
  const S e20 = (e80 * e80) * (e80 * e80);
  const S ah = S(0.07) * e20;
  const S bn = S(0.125) * e80;
  const S sm = am + bm, sh = ah + bh, sn = an + bn;
  m += M::omx(q10dt * sm, et) * (am * M::rcp(sm) - m);
  h += M::omx(q10dt * sh, et) * (ah * M::rcp(sh) - h);
  n += M::omx(q10dt * sn, et) * (an * M::rcp(sn) - n);
}

// slow K: n_inf = 1/(1+exp(-(v+35)/10)), tau = 400/(3.3 exp((v+35)/20) + exp(-(v+35)/20)) ms
template <typename S>
__device__ __forceinline__ void km_advance(double vd, S dt, S &n, const lds_table *et) {
  using M = Math<S>;
  const S u = (S)vd + S(35);
  const S e = M::ex(u * S(0.05), et);
  const S ei = M::rcp(e);
  const S ninf = M::rcp(S(1) + ei * ei);
  const S z = dt * S(1.0 / 400.0) * (S(3.3) * e + ei);
  n += M::omx(z, et) * (ninf - n);
}

// high-threshold Ca: m_inf = 1/(1+exp(-(v+20)/9)), tau_m 1 ms; shell calcium relaxing toward
// cai0 - k tau_r ica with ica taken at the new m.
template <typename S>
__device__ __forceinline__ void cahi_advance(double vd, S fm, S fr, S kk, S gca, S &m, S &cai, const lds_table *et) {
  using M = Math<S>;
  const S v = (S)vd;
  const S minf = M::rcp(S(1) + M::ex((v + S(20)) * S(-1.0 / 9.0), et));
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

// Channel states of one compartment advanced with v (the update pending from the previous step, when `pend`), then
// the currents and analytic conductances of its density mechanisms and IClamps at (v, states): rhs -= i, d += G
// (Sec. 2, matrix assembly; Sec. 3.5, CONDUCTANCE). mf: the compartment's mechanism flags; pk: its counts word;
// prm(col): one of its mechanism parameters; icl_of(): its first IClamp record.
template <typename S, bool UNI, typename Prm, typename Icl>
__device__ __forceinline__ void mech_terms(const KParams &p, uint32_t mf, uint32_t pk, Icl icl_of, int64_t n, double v,
                                           bool pend, S q10dt, S sdt, S ca_fm, S ca_fr, S ca_k, StRec<S> &sr,
                                           const lds_table *et, Prm prm, double &rhs, double &d) {
  if (pend) {
    if (mf & MF_HH) hh_advance<S>(v, q10dt, sr.m, sr.h, sr.n, et);
    if (mf & MF_KM) km_advance<S>(v, sdt, sr.kn, et);
    if (mf & MF_CAHI) cahi_advance<S>(v, ca_fm, ca_fr, ca_k, (S)prm(P_CA_G), sr.cm, sr.cai, et);
  }
  if (mf & MF_HH) {
    const double gnab = prm(P_HH_GNA), gkb = prm(P_HH_GK), gl = prm(P_HH_GL), el = prm(P_HH_EL);
    const double gna = (double)((S)gnab * (sr.m * sr.m * sr.m * sr.h));
    const double gk = (double)((S)gkb * ((sr.n * sr.n) * (sr.n * sr.n)));
    rhs -= gna * (v - 50.0) + gk * (v + 77.0) + gl * (v - el);
    d += gna + gk + gl;
  }
  if (mf & MF_PAS) {
    const double g = prm(P_PAS_G), e = prm(P_PAS_E);
    rhs -= g * (v - e);
    d += g;
  }
  if (mf & MF_KM) {
    const double g = (double)((S)prm(P_KM_G) * sr.kn);
    rhs -= g * (v + 77.0);
    d += g;
  }
  if (mf & MF_CAHI) {
    const double g = (double)((S)prm(P_CA_G) * (sr.cm * sr.cm));
    rhs -= g * (v - 120.0);
    d += g;
  }
  const int n_icl = (!UNI || p.has_icl) ? (int)((pk >> 16) & 0xFFu) : 0;
  if (n_icl) {
    const IclRec *ic = icl_of();
    for (int c = 0; c < n_icl; ++c)
      if (ic[c].on <= n && n < ic[c].off) rhs += ic[c].cur;
  }
}

// The chunk's events on chip (Sec. 2, event delivery): the keys of this group's ring bucket for the interval and the
// kicks due in the chunk, bitonic-sorted in LDS (key order is the delivery order), and in seg the first key of each
// step of the interval. Called by all T threads of the group; ev, seg and misc are read only after a later barrier.
// misc: [0] bucket keys, [1] the chunk's spike count (set to 0), [2] first kick, [3] kick count.
template <int T>
__device__ __forceinline__ void stage_events(const KParams &p, const GroupDesc &gd, int G, int t, int slot,
                                             int64_t ival, int64_t n_begin, int64_t n_end, uint64_t *ev, int *seg,
                                             int *misc) {
  const int M = p.M;
  if (t == 0) {
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
}

// a node's own inputs to the elimination: a, b, children, and from the assembly d, rhs and dv (v at a root)
struct TriIn {
  double a, b, d, r, dv;
  uint32_t ch;
};

// Subtract the children's contributions from d and rhs, in child order. `ch` holds the byte offset of the first
// child (its position times 8) in the low 16 bits and the child count in the high 16; `zero8` is the byte offset of
// the rows' zero entry. The first four children are read unconditionally, an absent one from the zero entry (x - 0
// is x exactly), so one LDS round trip serves most nodes. Child k is read at base + 8k, with base the first child's
// offset or zero8 - 8k when absent: 8k stays the instruction's immediate offset.
__device__ __forceinline__ double lds_at(const double *row, int byte_off) {
  return *reinterpret_cast<const double *>(reinterpret_cast<const char *>(row) + byte_off);
}
__device__ __forceinline__ void gather_children(uint32_t ch, int zero8, const double *P_l, const double *Q_l,
                                                double &d, double &rhs) {
  const int c0 = (int)(ch & 0xFFFFu), cn = (int)(ch >> 16);
  int b0 = cn > 0 ? c0 : zero8, b1 = cn > 1 ? c0 : zero8 - 8, b2 = cn > 2 ? c0 : zero8 - 16,
      b3 = cn > 3 ? c0 : zero8 - 24;
  asm volatile("" : "+v"(b1), "+v"(b2), "+v"(b3));  // keep the selects on the bases
  const double p0 = lds_at(P_l, b0), p1 = lds_at(P_l, b1 + 8), p2 = lds_at(P_l, b2 + 16), p3 = lds_at(P_l, b3 + 24);
  const double q0 = lds_at(Q_l, b0), q1 = lds_at(Q_l, b1 + 8), q2 = lds_at(Q_l, b2 + 16), q3 = lds_at(Q_l, b3 + 24);
  d -= p0;
  rhs -= q0;
  d -= p1;
  rhs -= q1;
  d -= p2;
  rhs -= q2;
  d -= p3;
  rhs -= q3;
  for (int c = c0 + 32; c < c0 + 8 * cn; c += 8) {
    d -= lds_at(P_l, c);
    rhs -= lds_at(Q_l, c);
  }
}

// one node of the elimination: gather the children's contributions, then publish this node's own
template <typename S>
__device__ __forceinline__ void tri_node(int q, const TriIn &x, int zero8, double *w_l, double *u_l, double *P_l,
                                         double *Q_l) {
  double d = x.d, rhs = x.r;
  gather_children(x.ch, zero8, P_l, Q_l, d, rhs);
  const double adv = x.a * x.dv;  // off the dependency chain
  const double ri = rcp64<S>(d);
  const double w = ri * x.b, u = ri * rhs;
  w_l[q] = w;
  u_l[q] = u;
  P_l[q] = fma(x.a, w, x.a);  // a (w + 1)
  Q_l[q] = fma(x.a, u, -adv);  // a (u - dv)
}

// ------------------------------------------------------------------------------------------------------------------
// LDS rows of NMAX = T K entries (the group capacity) and one more, in the order w, P, u, Q, V -
//   w_l  d (diagonal) after assembly, then w = b/d after elimination;
//   P_l  the node's contribution a(w + 1) to its parent's diagonal, later the solution x = Delta v;
//   u_l  rhs after assembly, then u = rhs/d after elimination;
//   Q_l  dv = v_parent - v after assembly (v itself at a root), then the contribution a(u - dv) to the parent's rhs;
//   V_l  the membrane potential v, updated in place by the substitution.
// Entry NMAX of the P and Q rows is zero: the children gather reads it for absent children. While the compartments
// assemble, the rows w and P together hold each synapse's conductance sa g and the rows u and Q its current
// sa g (v - e), for up to 2 NMAX synapses (short of the zero entries); the assembly keeps its results in registers
// until all threads have read them. For groups of up to 2048 nodes, further rows hold the chunk's per-node
// constants: parent and children (32-bit), a, b, k.
// With these, elimination of node i reads d_i, rhs_i and its children's contributions, and back-substitution is
// x_i = u_i - w_i x_parent. Each thread keeps the channel states of its compartments (node q = j T + t in register
// slot j) in registers for the whole chunk; states and potentials cross global memory once per chunk.
constexpr bool const_in_lds(int nmax) { return nmax <= 2048; }
// bytes of the node rows: two 32-bit rows of nmax and eight double rows of nmax + 1 entries, or five double rows
constexpr int lds_row_bytes(int nmax) { return const_in_lds(nmax) ? 8 * nmax + 64 * (nmax + 1) : 40 * (nmax + 1); }
// Waves per SIMD the register budget is sized for: more register slots per thread keep more compartments on chip.
// A group of 512 threads puts two waves on every SIMD, so two co-resident groups need four. The general 512 x 2
// kernels are held to four (a few registers spill); the uniform ones fit in 128 registers under a bound of three,
// whose schedule is measured 7-10 % faster than the one compiled for four. cn_model_info reports the groups that
// are co-resident on a CU, so a kernel that outgrows 128 registers shows up there. A group of 1024 threads puts four
// waves on every SIMD by itself.
constexpr int waves_for_shape(int T, int K, bool uni) {
  return T >= 1024 ? 4 : (K <= 1 ? 4 : (K == 2 ? (T >= 512 && !uni ? 4 : 3) : (K == 4 ? 2 : 1)));
}

// Phase clocks (profiling builds only, compiled with CN_PHASE_CLOCKS): each thread adds the shader clock between
// consecutive marks to a per-phase sum; the marks sit right after the barriers that close a phase, so the first
// wave's sums are the group's time per phase. Thread 0 adds them to p.phase_clk at the end.
#ifdef CN_PHASE_CLOCKS
#define CN_PHASE_MARK(k)                   \
  do {                                     \
    const uint64_t now_ = clock64();       \
    ph_clk[k] += now_ - ph_t0;             \
    ph_t0 = now_;                          \
  } while (0)
#else
#define CN_PHASE_MARK(k) \
  do {                   \
  } while (0)
#endif

// UNI: every compartment carries the same density mechanisms (flags in mf_uni) and every parameter is uniform
// (read from the LDS constants, not the per-node table)
template <int T, int K, typename S, bool UNI>
__global__ void __launch_bounds__(T, waves_for_shape(T, K, UNI)) cn_interval(const KParams p) {
  extern __shared__ __align__(16) unsigned char lds[];
  constexpr int NMAX = T * K;
  constexpr bool CL = const_in_lds(NMAX);
  // fixed row offsets: they become immediate offsets of the LDS instructions
  int *par_l = reinterpret_cast<int *>(lds);
  uint32_t *ch_l = reinterpret_cast<uint32_t *>(par_l + NMAX);
  constexpr int RS = NMAX + 1;  // double row stride; entry NMAX of P and Q is the zero entry
  double *w_l = reinterpret_cast<double *>(lds + (CL ? 8 * NMAX : 0));
  double *P_l = w_l + RS;
  double *u_l = P_l + RS;
  double *Q_l = u_l + RS;
  double *V_l = Q_l + RS;
  double *GS_l = w_l;  // synapse conductances (2 NMAX entries)
  double *IS_l = u_l;  // synapse currents (2 NMAX entries)
  double *a_l = V_l + RS;
  double *b_l = a_l + RS;
  double *k_l = b_l + RS;
  uint64_t *ev = reinterpret_cast<uint64_t *>(lds + p.lds_ev_off);
  int *seg = reinterpret_cast<int *>(lds + p.lds_seg_off);
  int *lv = reinterpret_cast<int *>(lds + p.lds_lvl_off);
  uint8_t *bgm = reinterpret_cast<uint8_t *>(lds + p.lds_bg_off);
  int *misc = reinterpret_cast<int *>(lds + p.lds_misc_off);
  double *cst = reinterpret_cast<double *>(lds + p.lds_cst_off);
  double *etab = reinterpret_cast<double *>(lds + p.lds_exp_off);
  const lds_table *etab3 = (const lds_table *)etab;

  const int G = blockIdx.x;
  const int t = threadIdx.x;
#ifdef CN_PHASE_CLOCKS
  uint64_t ph_clk[PH_COUNT] = {};
  uint64_t ph_t0 = clock64();
#endif
  const GroupDesc gd = p.groups[G];
  const int64_t n_begin = p.ctl[0];
  const int64_t n_target = p.ctl[1];
  // the chunk's first step carries no pending state update when it is step 0 or the step of a restart (ctl[2])
  const bool pend0 = n_begin > p.ctl[2];
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
  if (t < 64) etab[t] = p.exp_tab[t];
  if (t == 0) {
    cst[C_Q10DT] = p.q10dt;
    cst[C_DT] = p.dt;
    cst[C_CA_FM] = p.ca_fm;
    cst[C_CA_FR] = p.ca_fr;
    cst[C_CA_K] = p.ca_k;
    reinterpret_cast<uint64_t *>(cst)[C_SEED] = (uint64_t)p.ctl[3];  // key of the background streams
  }
  stage_events<T>(p, gd, G, t, slot, ival, n_begin, n_end, ev, seg, misc);

  auto c_a = [&](int q) { return CL ? a_l[q] : p.nrec[nb + q].a; };
  auto c_b = [&](int q) { return CL ? b_l[q] : p.nrec[nb + q].b; };
  auto c_k = [&](int q) { return CL ? k_l[q] : p.nrec[nb + q].k; };
  // the parent row packs the parent (12 bits, 4095 at a root) and the node's first synapse (20 bits)
  auto c_par = [&](int q) {
    if (!CL) return p.nidx[nb + q].par;
    const int pw = par_l[q] & 0xFFF;
    return pw == 0xFFF ? -1 : pw;
  };
  // children: first child as a byte offset (position times 8) | count << 16
  auto c_ch = [&](int q) {
    if (CL) return ch_l[q];
    const uint32_t c = p.nidx[nb + q].ch;
    return ((c & 0xFFFFu) << 3) | (c & 0xFFFF0000u);
  };
  auto tri_in = [&](int q) { return TriIn{c_a(q), c_b(q), w_l[q], u_l[q], Q_l[q], c_ch(q)}; };
  // uniform mechanism constants: FP32-mechanism kernels (registers to spare) take them straight from the kernel
  // arguments, FP64 kernels from the LDS copy
  constexpr bool KARG = std::is_same<S, float>::value;
  auto prm = [&](int col, int64_t i) -> double {
    if (UNI) return KARG ? p.prm_s[col] : cst[C_PRM + col];
    return p.prm ? p.prm[col * p.n_nodes_total + i] : cst[C_PRM + col];  // a column that varies: the table
  };
  StRec<S> *st = static_cast<StRec<S> *>(p.st);
  const SynRec<S> *syn = static_cast<const SynRec<S> *>(p.syn) + sb;
  S *sg = static_cast<S *>(p.syn_g) + sb;
  for (int q = t; q < N; q += T) {
    V_l[q] = p.v[nb + q];
    if (CL) {
      const NodeRec nr = p.nrec[nb + q];
      const NodeIdx nx = p.nidx[nb + q];
      a_l[q] = nr.a;
      b_l[q] = nr.b;
      k_l[q] = nr.k;
      par_l[q] = (nx.par < 0 ? 0xFFF : nx.par) | (int)((uint32_t)nx.syn0 << 12);
      ch_l[q] = ((nx.ch & 0xFFFFu) << 3) | (nx.ch & 0xFFFF0000u);
    }
  }
  // per-slot registers for the whole chunk: channel states, counts-and-flags
  StRec<S> rs[K];
  uint32_t rpk[K];
#pragma unroll
  for (int j = 0; j < K; ++j) {
    const int q = j * T + t;
    rs[j] = StRec<S>{};
    rpk[j] = 0u;
    if (q < N) {
      const NodeIdx nx = p.nidx[nb + q];
      rpk[j] = nx.pk;
      rs[j] = st[nb + q];
    }
  }
  if (!p.has_bg)
    for (int i = t; i < n_syn; i += T) bgm[i] = 0;
  // per cell of the group, on chip: threshold, soma potential before the step, soma position
  const int NC = gd.n_cells;
  double *theta_l = reinterpret_cast<double *>(lds + p.lds_cell_off);
  double *vold_l = theta_l + NC;
  int *soma_l = reinterpret_cast<int *>(vold_l + NC);
  for (int c = t; c < NC; c += T) {
    theta_l[c] = p.cell_theta[gd.cell_base + c];
    soma_l[c] = p.cell_soma[gd.cell_base + c];
  }
  if (t == 0) {
    P_l[NMAX] = 0.0;
    Q_l[NMAX] = 0.0;
  }
  // level starts, lane L of every wave holding lv[L]: read back with a lane read instead of an LDS round trip
  const int lvr = (t & 63) <= D ? lv[t & 63] : 0;
  // the deepest level holds leaves only: their elimination needs nothing from other nodes, so the assembly's
  // write-back does it and the sweeps start one level up (E levels left to them: all of them when D == 1)
  const int deep0 = D >= 2 ? lv[D - 1] : N;
  const int E = D >= 2 ? D - 1 : D;
  // synapse terms are staged on chip when the group's synapses fit the rows
  const bool staged = n_syn <= 2 * NMAX;
  __syncthreads();
  // everything but the compartments' assembly is latency-bound and runs at the higher wave priority
  __builtin_amdgcn_s_setprio(2);

  // ---- background-event bits and delivery for step n, by threads tid0, tid0 + stride, ...
  auto bg_and_deliver = [&](int64_t n, int tid0, int stride) {
    // background-event bits for a block of four steps (one Philox call gives four words)
    if (p.has_bg && (n == n_begin || (n & 3) == 0)) {
      const uint64_t blk = (uint64_t)n >> 2;
      // the background key: from the control block in the FP64 kernels (a scalar load), from its LDS copy in the
      // FP32-mechanism kernels, whose scalar registers are the scarcer resource
      const uint64_t seed = KARG ? reinterpret_cast<const uint64_t *>(cst)[C_SEED] : (uint64_t)p.ctl[3];
      for (int i = tid0; i < n_syn; i += stride) bgm[i] = (uint8_t)bg_mask4(seed, syn[i].key, blk, p.bg_thresh);
    }
    // A: delivery (Sec. 2, event-driven delivery step): one thread per synapse run, in key order
    const int sn = (int)(n - ival * M);
    const int e0 = seg[sn], e1 = seg[sn + 1];
    for (int e = e0 + tid0; e < e1; e += stride) {
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
  };
  // These depend only on the previous step's synapse staging. With the FP32 mechanisms (whose register budget has
  // room for it) they run, for every step but a chunk's first, during the previous step's elimination on the upper
  // half of the threads, which the narrow deep levels leave idle.
  constexpr bool EARLY = std::is_same<S, float>::value;
  if (EARLY) {
    bg_and_deliver(n_begin, t, T);
    __syncthreads();
  }

  // ---- threshold detection at each cell's soma (Sec. 2): an upward crossing between the potential before and
  // after a step. The soma potential a step produces stays in V_l until the next step's substitution, so the test
  // of step n runs at the top of step n + 1 (for a chunk's last step, after the loop), on the highest threads, which
  // the synapse staging leaves idle in most groups; the potential is then kept as the next step's old one. `sn` is
  // the step inside the interval whose potentials V_l holds.
  auto detect = [&](int sn, bool test) {
    for (int c = T - 1 - t; c < NC; c += T) {
      const double vnew = V_l[soma_l[c]];
      if (test) {
        const double vold = vold_l[c], th = theta_l[c];
        if (vold < th && th <= vnew) {
          const int idx = atomicAdd(&misc[1], 1);
          p.gsp_pack[gd.spk_base + idx] = c | (sn << 16);
          p.gsp_frac[gd.spk_base + idx] = (th - vold) / (vnew - vold);
        }
      }
      vold_l[c] = vnew;
    }
  };

  CN_PHASE_MARK(PH_CHUNK);
  for (int64_t n = n_begin; n < n_end; ++n) {
    const int s = (int)(n - ival * M);
    if (!EARLY) {
      bg_and_deliver(n, t, T);
      __syncthreads();
    }
    detect(s, n > n_begin);
    const uint32_t bsh = (uint32_t)(n & 3);
    // ---- S: synapses, one thread per synapse over contiguous records: conductance gs = sa g (with this step's
    // background event) and current gs (v - e) to LDS; the step's decay is applied to g ahead of the next delivery
    if (staged) {
      for (int ls = t; ls < n_syn; ls += T) {
        const SynRec<S> sy = syn[ls];
        S g = sg[ls];
        if ((bgm[ls] >> bsh) & 1u) g += sy.wbg;
        const double gs = sy.sa * (double)g;
        GS_l[ls] = gs;
        IS_l[ls] = gs * (V_l[sy.q] - sy.e);
        sg[ls] = g * sy.f;
      }
      __syncthreads();
    }
    CN_PHASE_MARK(PH_EVENTS);
    // ---- C: states, currents, conductances and the compartment's own axial terms. Throughput work: it runs at
    // the lower wave priority, so that a co-resident group's latency-bound sweeps issue ahead of it.
    __builtin_amdgcn_s_setprio(0);
    const bool pend = n > n_begin || pend0;
    const S q10dt = (S)(KARG ? p.q10dt : cst[C_Q10DT]);
    const S sdt = (S)(KARG ? p.dt : cst[C_DT]);
    const S ca_fm = (S)(KARG ? p.ca_fm : cst[C_CA_FM]), ca_fr = (S)(KARG ? p.ca_fr : cst[C_CA_FR]),
            ca_k = (S)(KARG ? p.ca_k : cst[C_CA_K]);
    double od[K], orhs[K], odv[K];  // assembly results, written once every thread has read the staged synapses
#pragma unroll
    for (int j = 0; j < K; ++j) {
      const int q = j * T + t;
      od[j] = orhs[j] = odv[j] = 0.0;
      if (q < N) {
        const int64_t i = nb + q;
        const int par = c_par(q);
        const uint32_t pk = rpk[j];
        const double v = V_l[q];
        double rhs = 0.0, d = 0.0;
        // with one mechanism set on every compartment the flags are a kernel argument: uniform branches
        const uint32_t mf = UNI ? p.mf_uni : (pk >> 24) & 0xFu;
        mech_terms<S, UNI>(
            p, mf, pk, [&]() { return p.icl + gd.icl_base + p.nd_icl0[i]; }, n, v, pend, q10dt, sdt, ca_fm, ca_fr,
            ca_k, rs[j], etab3, [&](int col) { return prm(col, i); }, rhs, d);
        const int n_s = (int)(pk & 0xFFFFu);
        {
          if (staged) {
            const int syn0 = CL ? (int)((uint32_t)par_l[q] >> 12) : p.nidx[i].syn0;
            // the first two synapses unconditionally, an absent one from the rows' zero entry (index 2 NMAX + 1
            // of the staged span is the P and Q rows' zero entry, which staging leaves alone): adding zero leaves
            // the sums exact, in the same order
            const int z = 2 * NMAX + 1, c0 = n_s > 0 ? syn0 : z, c1 = n_s > 1 ? syn0 + 1 : z;
            rhs -= IS_l[c0];
            d += GS_l[c0];
            rhs -= IS_l[c1];
            d += GS_l[c1];
            for (int c = syn0 + 2; c < syn0 + n_s; ++c) {
              rhs -= IS_l[c];
              d += GS_l[c];
            }
          } else if (n_s) {  // groups with more synapses than a row holds: the same terms, computed here
            const int syn0 = p.nidx[i].syn0;
            for (int ls = syn0; ls < syn0 + n_s; ++ls) {
              const SynRec<S> sy = syn[ls];
              S g = sg[ls];
              if ((bgm[ls] >> bsh) & 1u) g += sy.wbg;
              const double gs = sy.sa * (double)g;
              rhs -= gs * (v - sy.e);
              d += gs;
              sg[ls] = g * sy.f;
            }
          }
        }
        // half-gap junctions (reading R13): the partner's potential from the start of the step, still in V_l (a
        // model with junctions runs the general kernels: the uniform ones keep their registers for the rest)
        const int n_gap = UNI ? 0 : (int)(pk >> 28);
        if (n_gap) {
          const GapRec *gr = p.gap + gd.gap_base + p.nd_gap0[i];
          for (int c = 0; c < n_gap; ++c) {
            rhs -= gr[c].gs * (v - V_l[gr[c].q]);
            d += gr[c].gs;
          }
        }
        d += c_k(q);
        double dvq = v;  // a root carries its own potential: the root solve adds its x to it
        if (par >= 0) {
          dvq = V_l[par] - v;
          rhs -= c_b(q) * dvq;
        }
        od[j] = d;
        orhs[j] = rhs;
        odv[j] = dvq;
      }
      __builtin_amdgcn_sched_barrier(0);
    }
    __syncthreads();
#pragma unroll
    for (int j = 0; j < K; ++j) {
      const int q = j * T + t;
      if (q < N) {
        if (q < deep0) {
          w_l[q] = od[j];
          u_l[q] = orhs[j];
          Q_l[q] = odv[j];
        } else {  // a leaf of the deepest level: the elimination of tri_node with no child to gather
          const double a = c_a(q), adv = a * odv[j];
          const double ri = rcp64<S>(od[j]);
          const double w = ri * c_b(q), u = ri * orhs[j];
          w_l[q] = w;
          u_l[q] = u;
          P_l[q] = fma(a, w, a);
          Q_l[q] = fma(a, u, -adv);
        }
      }
    }
    __syncthreads();
    __builtin_amdgcn_s_setprio(2);
    CN_PHASE_MARK(PH_MECH);
    // the next step's background bits and delivery (FP32 mechanisms), on the upper half of the threads; the
    // elimination's first barrier waits for them
    if (EARLY && n + 1 < n_end && t >= T / 2) bg_and_deliver(n + 1, t - T / 2, T / 2);
    // the sweeps; level starts are read from lane registers when the group has fewer than 64 levels
    auto sweeps = [&]() {
      auto LVB = [&](int L) -> int { return __builtin_amdgcn_readlane(lvr, L); };
      // ---- T: elimination from the level above the deepest (done in the assembly's write-back) up, one thread per
      // node of the level. A level's own inputs are final before it starts, so each thread loads them one level
      // ahead; after a barrier only the children's contributions remain to be read.
      int hi = LVB(E), lo = LVB(E - 1), lo_n = E >= 2 ? LVB(E - 2) : 0;
      int q = lo + t;
      TriIn cur{};
      if (q < hi) cur = tri_in(q);
      for (int L = E - 1; L >= 1; --L) {  // level L is [lo, hi), level L - 1 is [lo_n, lo)
        const int lo_nn = L >= 2 ? LVB(L - 2) : 0;
        const int nq = lo_n + t;
        const TriIn nxt = tri_in(min(nq, N - 1));  // lanes past the level read the group's last node and ignore it
        if (q < hi) tri_node<S>(q, cur, NMAX * 8, w_l, u_l, P_l, Q_l);
        for (int q2 = q + T; q2 < hi; q2 += T) tri_node<S>(q2, tri_in(q2), NMAX * 8, w_l, u_l, P_l, Q_l);  // wide levels
        __syncthreads();
        hi = lo;
        lo = lo_n;
        lo_n = lo_nn;
        q = nq;
        cur = nxt;
      }
      CN_PHASE_MARK(PH_ELIM);
      // ---- R: roots (level 0 holds the group's cells in order): solve and v update
      for (; q < hi; q += T) {
        const TriIn x = q == t ? cur : tri_in(q);
        double d = x.d, rhs = x.r;
        gather_children(x.ch, NMAX * 8, P_l, Q_l, d, rhs);
        const double xs = rhs * rcp64<S>(d);
        const double vnew = x.dv + xs;
        P_l[q] = xs;
        V_l[q] = vnew;
        if (!isfinite(vnew)) atomicOr(&p.flags[FLAG_NONFINITE], 1);
      }
      __syncthreads();
      CN_PHASE_MARK(PH_ROOT);
      // ---- B: substitution, root to leaves, v += x, BL levels per barrier. A node of the first level of a pass reads
      // its parent's x: x = u - w x_p. A node j levels deeper folds the steps of its j nearest ancestors into its
      // coefficients, x = cu - cw x_a with a its (j+1)-th ancestor (cu <- cu - cw u_p, cw <- -cw w_p, p <- parent of
      // p), and reads x_a, which a previous pass computed. Every term but that x is final once the elimination is
      // done, so each thread loads and folds them one pass ahead.
      if (D > 1) {
        constexpr int BL = 3;
        // inputs of node q in a pass whose deeper levels start at m1, m2: x = cu - cw x[cs] (v, read after the
        // barrier in the same round trip as x[cs], gets v + x)
        auto pass_in = [&](int q, int m1, int m2, double &cu, double &cw, int &cs) {
          cu = u_l[q];
          cw = w_l[q];
          cs = c_par(q);
          const int j = (q >= m1) + (q >= m2);
          for (int i = 0; i < j; ++i) {
            const double up = u_l[cs], wp = w_l[cs];
            cs = c_par(cs);
            cu = fma(-cw, up, cu);
            cw = -(cw * wp);
          }
        };
        int bm1 = LVB(min(2, D)), bm2 = LVB(min(3, D)), bend = LVB(min(1 + BL, D));
        int bq = LVB(1) + t;
        double cu = 0.0, cw = 0.0;
        int cs = 0;
        if (bq < bend) pass_in(bq, bm1, bm2, cu, cw, cs);
        for (int L0 = 1; L0 < D; L0 += BL) {  // this pass: levels L0 .. L0 + BL - 1, nodes [bq - t, bend)
          const int L1 = L0 + BL;
          int nm1 = 0, nm2 = 0, nend = 0;
          if (L1 < D) {
            nm1 = LVB(min(L1 + 1, D));
            nm2 = LVB(min(L1 + 2, D));
            nend = LVB(min(L1 + BL, D));
          }
          const int nq = bend + t;
          double nu = 0.0, nw = 0.0;
          int ns = 0;
          if (nq < nend) pass_in(nq, nm1, nm2, nu, nw, ns);
          if (bq < bend) {
            const double x = cu - cw * P_l[cs];
            P_l[bq] = x;
            V_l[bq] += x;
          }
          for (int q2 = bq + T; q2 < bend; q2 += T) {  // passes wider than the group's threads
            double u2, w2;
            int s2;
            pass_in(q2, bm1, bm2, u2, w2, s2);
            const double x = u2 - w2 * P_l[s2];
            P_l[q2] = x;
            V_l[q2] += x;
          }
          __syncthreads();
          bq = nq;
          bm1 = nm1;
          bm2 = nm2;
          bend = nend;
          cu = nu;
          cw = nw;
          cs = ns;
        }
      }
      CN_PHASE_MARK(PH_SUBST);
    };
    // the same sweeps without the look-ahead, for groups of 64 or more levels (level starts from LDS)
    auto plain_sweeps = [&]() {
      for (int L = E - 1; L >= 1; --L) {
        for (int q = lv[L] + t; q < lv[L + 1]; q += T) tri_node<S>(q, tri_in(q), NMAX * 8, w_l, u_l, P_l, Q_l);
        __syncthreads();
      }
      CN_PHASE_MARK(PH_ELIM);
      for (int q = t; q < lv[1]; q += T) {
        const TriIn x = tri_in(q);
        double d = x.d, rhs = x.r;
        gather_children(x.ch, NMAX * 8, P_l, Q_l, d, rhs);
        const double xs = rhs * rcp64<S>(d);
        const double vnew = x.dv + xs;
        P_l[q] = xs;
        V_l[q] = vnew;
        if (!isfinite(vnew)) atomicOr(&p.flags[FLAG_NONFINITE], 1);
      }
      __syncthreads();
      CN_PHASE_MARK(PH_ROOT);
      for (int L = 1; L < D; ++L) {
        for (int q = lv[L] + t; q < lv[L + 1]; q += T) {
          const double x = u_l[q] - w_l[q] * P_l[c_par(q)];
          P_l[q] = x;
          V_l[q] += x;
        }
        __syncthreads();
      }
      CN_PHASE_MARK(PH_SUBST);
    };
    if (D < 64) sweeps();
    else plain_sweeps();
  }
  if (n_end > n_begin) detect((int)(n_end - ival * M), true);

  // ---- epilogue: potentials and states back to global memory; the chunk's spikes (count in gsp_cnt) are recorded
  // and fanned out by cn_fanout
  for (int q = t; q < N; q += T) p.v[nb + q] = V_l[q];
#pragma unroll
  for (int j = 0; j < K; ++j) {
    const int q = j * T + t;
    if (q < N) st[nb + q] = rs[j];
  }
  __syncthreads();  // every detection's count is in
  if (t == 0) {
    p.gsp_cnt[G] = misc[1];
    if (n_end == (ival + 1) * (int64_t)M) p.ev_cnt[(int64_t)slot * p.n_groups + G] = 0;
  }
#ifdef CN_PHASE_CLOCKS
  CN_PHASE_MARK(PH_CHUNK);
  if (t == 0)
    for (int k = 0; k < PH_COUNT; ++k) atomicAdd(reinterpret_cast<unsigned long long *>(p.phase_clk + k), ph_clk[k]);
#endif
}

// ------------------------------------------------------------------------------------------------------------------
// Interleaved layout, one lane per cell (the paper's one-cell-per-thread GPU ordering, Sec. 4.4): a group is up to 64
// cells, one per lane of a single wave, whose compartments are interleaved in global memory: compartment k of lane j
// sits at node_base + 64 k + j, in the caller's order (root first, parent before child), the group padded to its
// largest cell with inert compartments (d = 1, no terms, parent the root). Each lane advances its own cell through
// the chunk with no barrier: delivery and background events of its synapses, then one pass over its compartments
// from the last to the root doing each one's states, currents, assembly and elimination (Sec. 2, Gaussian
// elimination in the Hines order), then the substitution back. Accesses are coalesced across the wave when the 64
// cells share the parent index of a compartment (identical cells), strided otherwise: the effect the paper measures.
// The tree work arrays (the elimination's accumulators, later w and u; the solution x) live in global memory.
// Threshold detection at the root, compacted in cell order with a wave ballot.
template <typename S, bool UNI>
__global__ void __launch_bounds__(64) cn_lpc(const KParams p) {
  extern __shared__ __align__(16) unsigned char lds[];
  uint64_t *ev = reinterpret_cast<uint64_t *>(lds + p.lds_ev_off);
  int *seg = reinterpret_cast<int *>(lds + p.lds_seg_off);
  uint8_t *bgm = reinterpret_cast<uint8_t *>(lds + p.lds_bg_off);
  int *misc = reinterpret_cast<int *>(lds + p.lds_misc_off);
  double *etab = reinterpret_cast<double *>(lds + p.lds_exp_off);
  const lds_table *etab3 = (const lds_table *)etab;
  const int G = blockIdx.x;
  const int lane = threadIdx.x;
  const GroupDesc gd = p.groups[G];
  const int64_t n_begin = p.ctl[0];
  const int64_t n_target = p.ctl[1];
  const int64_t n_fresh = p.ctl[2];
  const uint64_t seed = (uint64_t)p.ctl[3];
  const int M = p.M;
  const int64_t ival = n_begin / M;
  const int64_t n_end = min(n_target, (ival + 1) * (int64_t)M);
  if (n_end <= n_begin) return;
  const int slot = (int)(ival % p.ring);
  etab[lane] = p.exp_tab[lane];
  stage_events<64>(p, gd, G, lane, slot, ival, n_begin, n_end, ev, seg, misc);
  __syncthreads();

  const bool act = lane < gd.n_cells;
  const int KN = gd.n_levels;  // compartment slots per lane
  const int64_t nb = gd.node_base + lane;
  const int cb = gd.cell_base + lane;
  const double theta = act ? p.cell_theta[cb] : 0.0;
  StRec<S> *st = static_cast<StRec<S> *>(p.st);
  const SynRec<S> *syn = static_cast<const SynRec<S> *>(p.syn) + gd.syn_base;
  S *sg = static_cast<S *>(p.syn_g) + gd.syn_base;
  double *V = p.v, *Dw = p.lw_d, *Rw = p.lw_r, *DVw = p.lw_dv;
  auto prm = [&](int col, int64_t i) -> double {
    return (UNI || !p.prm) ? p.prm_s[col] : p.prm[col * p.n_nodes_total + i];
  };
  const S q10dt = (S)p.q10dt, sdt = (S)p.dt, ca_fm = (S)p.ca_fm, ca_fr = (S)p.ca_fr, ca_k = (S)p.ca_k;
  double vold = act ? V[nb] : 0.0;
  int nspk = 0;  // spikes of the chunk so far (uniform across the wave)
  for (int64_t n = n_begin; n < n_end; ++n) {
    const int s = (int)(n - ival * M);
    const uint32_t bsh = (uint32_t)(n & 3);
    // delivery: this cell's events of step n (a synapse belongs to the lane of its compartment), in key order
    for (int e = seg[s]; e < seg[s + 1]; ++e) {
      const uint64_t key = ev[e];
      const int ls = (int)ev_syn(key);
      if ((syn[ls].q & 63) != lane) continue;
      const uint32_t id = (uint32_t)key & 0x7FFFFFFFu;
      sg[ls] += (key & EV_KIND_NETCON) ? ld<S>(p.nc_w, id) : ld<S>(p.kick_w, id);
    }
    // background-event bits of the cell's synapses are drawn for a block of four steps
    const bool draw = p.has_bg && (n == n_begin || (n & 3) == 0);
    // One pass over the compartments, last first: each compartment's states, currents and conductances, synapses
    // and own matrix terms, then its elimination, since its children (higher indices) are done. A child passes
    // a (w + 1) and a (u - dv) to its parent through the accumulators Dw, Rw (the parent's axial terms folded in),
    // which the substitution leaves at zero for the next step; the compartment's w, u take their place.
    const bool pend = n > n_fresh;
    double vnew = 0.0;
    for (int k = KN - 1; k >= 0; --k) {
      const int64_t i = nb + 64 * (int64_t)k;
      const NodeIdx nx = p.nidx[i];
      const NodeRec nr = p.nrec[i];
      const double v = V[i];
      const uint32_t mf = UNI ? p.mf_uni : (nx.pk >> 24) & 0xFu;
      double rhs = 0.0, d = 0.0;
      if (mf & (MF_HH | MF_KM | MF_CAHI)) {
        StRec<S> sr = st[i];
        mech_terms<S, UNI>(
            p, mf, nx.pk, [&]() { return p.icl + gd.icl_base + p.nd_icl0[i]; }, n, v, pend, q10dt, sdt, ca_fm, ca_fr,
            ca_k, sr, etab3, [&](int col) { return prm(col, i); }, rhs, d);
        st[i] = sr;
      } else {
        StRec<S> none{};
        mech_terms<S, UNI>(
            p, mf, nx.pk, [&]() { return p.icl + gd.icl_base + p.nd_icl0[i]; }, n, v, false, q10dt, sdt, ca_fm, ca_fr,
            ca_k, none, etab3, [&](int col) { return prm(col, i); }, rhs, d);
      }
      const int n_s = (int)(nx.pk & 0xFFFFu);
      for (int ls = nx.syn0; ls < nx.syn0 + n_s; ++ls) {
        const SynRec<S> sy = syn[ls];
        if (draw) bgm[ls] = (uint8_t)bg_mask4(seed, sy.key, (uint64_t)n >> 2, p.bg_thresh);
        S g = sg[ls];
        if (p.has_bg && ((bgm[ls] >> bsh) & 1u)) g += sy.wbg;
        const double gs = sy.sa * (double)g;
        rhs -= gs * (v - sy.e);
        d += gs;
        sg[ls] = g * sy.f;
      }
      // half-gap junctions: the partner is a compartment of this wave's cells, whose potential is still the one at
      // the start of the step (every lane updates potentials only in the substitution below)
      const int n_gap = UNI ? 0 : (int)(nx.pk >> 28);
      if (n_gap) {
        const GapRec *gr = p.gap + gd.gap_base + p.nd_gap0[i];
        for (int c = 0; c < n_gap; ++c) {
          rhs -= gr[c].gs * (v - V[gd.node_base + gr[c].q]);
          d += gr[c].gs;
        }
      }
      d += nr.k;
      double dv = v;  // the root carries its own potential
      if (k > 0) {
        dv = V[nb + 64 * (int64_t)nx.par] - v;
        rhs -= nr.b * dv;
      }
      d += Dw[i];  // the children's contributions (zero for a leaf)
      rhs += Rw[i];
      if (k > 0) {
        const int64_t ip = nb + 64 * (int64_t)nx.par;
        const double ri = rcp64<S>(d);
        const double w = ri * nr.b, u = ri * rhs;
        Dw[i] = w;
        Rw[i] = u;
        Dw[ip] -= fma(nr.a, w, nr.a);
        Rw[ip] -= fma(nr.a, u, -(nr.a * dv));
      } else {  // the root (compartment 0 of the lane's cell): solve, v update, threshold detection below
        const double xs = rhs * rcp64<S>(d);
        vnew = dv + xs;
        DVw[nb] = xs;
        V[nb] = vnew;
        Dw[nb] = 0.0;
        Rw[nb] = 0.0;
        if (act && !isfinite(vnew)) atomicOr(&p.flags[FLAG_NONFINITE], 1);
      }
    }
    // the substitution: x = u - w x_parent, v += x; the accumulators return to zero
    for (int k = 1; k < KN; ++k) {
      const int64_t i = nb + 64 * (int64_t)k;
      const double x = Rw[i] - Dw[i] * DVw[nb + 64 * (int64_t)p.nidx[i].par];
      DVw[i] = x;
      V[i] += x;
      Dw[i] = 0.0;
      Rw[i] = 0.0;
    }
    const bool spk = act && vold < theta && theta <= vnew;
    const uint64_t mask = __ballot(spk);
    if (spk) {
      const int idx = nspk + __popcll(mask & ((1ull << lane) - 1ull));
      p.gsp_pack[gd.spk_base + idx] = lane | ((s + 1) << 16);
      p.gsp_frac[gd.spk_base + idx] = (theta - vold) / (vnew - vold);
    }
    nspk += __popcll(mask);
    vold = vnew;
  }
  if (lane == 0) {
    p.gsp_cnt[G] = nspk;
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

// control block of a run: first step, target step, the step whose states are fresh, background key
__global__ void cn_set_ctl(int64_t *ctl, int64_t n_begin, int64_t n_target, int64_t n_fresh, uint64_t seed) {
  if (threadIdx.x == 0 && blockIdx.x == 0) {
    ctl[0] = n_begin;
    ctl[1] = n_target;
    ctl[2] = n_fresh;
    ctl[3] = (int64_t)seed;
  }
}

// events rebuilt by a restart: key k goes to ring bucket bucket[k] (the interval kernel sorts each bucket's keys, so
// the order of arrival does not matter)
__global__ void cn_insert_events(int32_t *ev_cnt, uint64_t *ev_key, int32_t cap, int64_t n, const int64_t *bucket,
                                 const uint64_t *key, int32_t *flags) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
    const int64_t b = bucket[i];
    const int pos = atomicAdd(&ev_cnt[b], 1);
    if (pos < cap) ev_key[b * cap + pos] = key[i];
    else atomicOr(&flags[FLAG_EV_OVERFLOW], 1);
  }
}

__global__ void cn_fill_i32(int32_t *p, int64_t n, int32_t v) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    p[i] = v;
}

// Mechanism state readout at the current step, in the caller's instance order: instance k sits at device node (or,
// for ExpSyn, device synapse) inst_dev[k]. Channel states are stored one update behind (the update of the last step is
// applied at the start of the next), so the pending update is applied to a copy here.
template <typename S>
__global__ void cn_gather_state(const KParams p, const int32_t *inst_dev, int64_t n, int64_t step, int64_t n_fresh,
                                int type, int which, double *out) {
  __shared__ double tab[64];
  if (threadIdx.x < 64) tab[threadIdx.x] = p.exp_tab[threadIdx.x];
  __syncthreads();
  const lds_table *et = (const lds_table *)tab;
  const int64_t k = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (k >= n) return;
  const int64_t i = inst_dev[k];
  if (type == 4) {
    out[k] = (double)static_cast<const S *>(p.syn_g)[i];
    return;
  }
  const double v = p.v[i];
  const bool pend = step > n_fresh;
  StRec<S> sr = static_cast<const StRec<S> *>(p.st)[i];
  if (type == 0) {
    if (pend) hh_advance<S>(v, (S)p.q10dt, sr.m, sr.h, sr.n, et);
    out[k] = which == 0 ? (double)sr.m : (which == 1 ? (double)sr.h : (double)sr.n);
  } else if (type == 2) {
    if (pend) km_advance<S>(v, (S)p.dt, sr.kn, et);
    out[k] = (double)sr.kn;
  } else if (type == 3) {
    const S gca = (S)(p.prm ? p.prm[P_CA_G * p.n_nodes_total + i] : p.prm_s[P_CA_G]);
    if (pend) cahi_advance<S>(v, (S)p.ca_fm, (S)p.ca_fr, (S)p.ca_k, gca, sr.cm, sr.cai, et);
    out[k] = which == 0 ? (double)sr.cm : (double)sr.cai;
  }
}

// ------------------------------------------------------------------------------------------------------------------
// launch wrappers (host side)
using IntervalFn = void (*)(const KParams);

template <typename S, bool UNI>
static IntervalFn interval_fn_s(int threads, int slots) {
  if (threads == 256) {
    switch (slots) {
      case 1: return cn_interval<256, 1, S, UNI>;
      case 2: return cn_interval<256, 2, S, UNI>;
      case 4: return cn_interval<256, 4, S, UNI>;
      default: break;
    }
  } else if (threads == 512) {
    switch (slots) {
      case 2: return cn_interval<512, 2, S, UNI>;
      case 4: return cn_interval<512, 4, S, UNI>;
      case 8: return cn_interval<512, 8, S, UNI>;
      default: break;
    }
  } else if (threads == 1024) {
    if (slots == 2) return cn_interval<1024, 2, S, UNI>;
  } else if (threads == 128) {
    switch (slots) {
      case 2: return cn_interval<128, 2, S, UNI>;
      case 4: return cn_interval<128, 4, S, UNI>;
      case 8: return cn_interval<128, 8, S, UNI>;
      default: break;
    }
  }
  return nullptr;
}

static IntervalFn interval_fn(bool fp32, int threads, int slots, bool uni) {
  if (uni) return fp32 ? interval_fn_s<float, true>(threads, slots) : interval_fn_s<double, true>(threads, slots);
  return fp32 ? interval_fn_s<float, false>(threads, slots) : interval_fn_s<double, false>(threads, slots);
}

static IntervalFn lpc_fn(bool fp32, bool uni) {
  if (uni) return fp32 ? cn_lpc<float, true> : cn_lpc<double, true>;
  return fp32 ? cn_lpc<float, false> : cn_lpc<double, false>;
}

hipError_t set_lpc_lds(bool fp32, bool uni, int lds_bytes) {
  return hipFuncSetAttribute(reinterpret_cast<const void *>(lpc_fn(fp32, uni)),
                             hipFuncAttributeMaxDynamicSharedMemorySize, lds_bytes);
}

hipError_t launch_lpc(const KParams &p, bool fp32, int lds_bytes, hipStream_t st) {
  hipLaunchKernelGGL(lpc_fn(fp32, p.uni != 0), dim3(p.n_groups), dim3(64), lds_bytes, st, p);
  return hipGetLastError();
}

int interval_row_bytes(int nmax) { return lds_row_bytes(nmax); }

hipError_t set_interval_lds(bool fp32, int threads, int slots, bool uni, int lds_bytes) {
  IntervalFn fn = interval_fn(fp32, threads, slots, uni);
  if (!fn) return hipErrorInvalidValue;
  return hipFuncSetAttribute(reinterpret_cast<const void *>(fn), hipFuncAttributeMaxDynamicSharedMemorySize,
                             lds_bytes);
}

// work-groups of the kernel that fit on one CU at once with this much dynamic LDS (registers, LDS and waves)
hipError_t interval_groups_per_cu(bool fp32, int threads, int slots, bool uni, int lds_bytes, int *n) {
  IntervalFn fn = interval_fn(fp32, threads, slots, uni);
  if (!fn) return hipErrorInvalidValue;
  return hipOccupancyMaxActiveBlocksPerMultiprocessor(n, reinterpret_cast<const void *>(fn), threads, lds_bytes);
}

hipError_t lpc_groups_per_cu(bool fp32, bool uni, int lds_bytes, int *n) {
  return hipOccupancyMaxActiveBlocksPerMultiprocessor(n, reinterpret_cast<const void *>(lpc_fn(fp32, uni)), 64,
                                                      lds_bytes);
}

hipError_t launch_interval(const KParams &p, bool fp32, int threads, int slots, int lds_bytes, hipStream_t st) {
  IntervalFn fn = interval_fn(fp32, threads, slots, p.uni != 0);
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

hipError_t launch_set_ctl(int64_t *ctl, int64_t n_begin, int64_t n_target, int64_t n_fresh, uint64_t seed,
                          hipStream_t st) {
  hipLaunchKernelGGL(cn_set_ctl, dim3(1), dim3(64), 0, st, ctl, n_begin, n_target, n_fresh, seed);
  return hipGetLastError();
}

hipError_t launch_insert_events(int32_t *ev_cnt, uint64_t *ev_key, int32_t cap, int64_t n, const int64_t *bucket,
                                const uint64_t *key, int32_t *flags, hipStream_t st) {
  if (n <= 0) return hipSuccess;
  int64_t blocks = (n + 255) / 256;
  if (blocks > 4096) blocks = 4096;
  hipLaunchKernelGGL(cn_insert_events, dim3((unsigned)blocks), dim3(256), 0, st, ev_cnt, ev_key, cap, n, bucket, key,
                     flags);
  return hipGetLastError();
}

hipError_t launch_fill_i32(int32_t *ptr, int64_t n, int32_t v, hipStream_t st) {
  if (n <= 0) return hipSuccess;
  int64_t blocks = (n + 255) / 256;
  if (blocks > 4096) blocks = 4096;
  hipLaunchKernelGGL(cn_fill_i32, dim3((unsigned)blocks), dim3(256), 0, st, ptr, n, v);
  return hipGetLastError();
}

hipError_t launch_gather_state(const KParams &p, bool fp32, const int32_t *inst_dev, int64_t n, int64_t step,
                               int64_t n_fresh, int type, int which, double *out, hipStream_t st) {
  if (n <= 0) return hipSuccess;
  const unsigned blocks = (unsigned)((n + 255) / 256);
  if (fp32)
    hipLaunchKernelGGL(cn_gather_state<float>, dim3(blocks), dim3(256), 0, st, p, inst_dev, n, step, n_fresh, type,
                       which, out);
  else
    hipLaunchKernelGGL(cn_gather_state<double>, dim3(blocks), dim3(256), 0, st, p, inst_dev, n, step, n_fresh, type,
                       which, out);
  return hipGetLastError();
}

}  // namespace cn
