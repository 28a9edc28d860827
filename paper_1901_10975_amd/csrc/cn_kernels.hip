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
// Philox4x32-10 (Salmon, Moraes, Dror, Shaw, SC'11): ten rounds of two 32x32->64 multiplies that mix the counter
// under a key bumped by Weyl constants. Background event for (synapse s, step n): word n % 4 of
// Philox(counter = (s lo, s hi, n/4 lo, n/4 hi), key = (seed lo, seed hi)) below the rate threshold.
__device__ __forceinline__ uint32_t bg_word(uint64_t seed, uint64_t syn, uint64_t step) {
  const uint64_t blk = step >> 2;
  uint32_t c0 = (uint32_t)syn, c1 = (uint32_t)(syn >> 32), c2 = (uint32_t)blk, c3 = (uint32_t)(blk >> 32);
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
  const int w = (int)(step & 3);
  return w == 0 ? c0 : (w == 1 ? c1 : (w == 2 ? c2 : c3));
}

// ------------------------------------------------------------------------------------------------------------------
// Mechanism kinetics. S is the state type: double on the FP64 path, float on the FP32-mechanism path (rates and
// exponentials in float with the hardware exp; voltage, currents, assembly and solve stay double).
template <typename S>
struct Math;
template <>
struct Math<double> {
  static __device__ __forceinline__ double ex(double x) { return exp(x); }
  static __device__ __forceinline__ double rcp(double x) { return 1.0 / x; }
  // 1 - exp(-z)
  static __device__ __forceinline__ double omx(double z) { return 1.0 - exp(-z); }
};
template <>
struct Math<float> {
  static __device__ __forceinline__ float ex(float x) { return __expf(x); }
  static __device__ __forceinline__ float rcp(float x) { return __fdividef(1.0f, x); }
  // 1 - exp(-z) without the cancellation of the subtraction at small z (four-term series below 0.03)
  static __device__ __forceinline__ float omx(float z) {
    return z < 0.03f ? z * (1.0f - z * 0.5f * (1.0f - z * (1.0f / 3.0f) * (1.0f - 0.25f * z))) : 1.0f - __expf(-z);
  }
};

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

// ------------------------------------------------------------------------------------------------------------------
template <int T, int K, typename S>
__global__ void __launch_bounds__(T) cn_interval(const KParams p) {
  extern __shared__ __align__(16) unsigned char lds[];
  constexpr int NMAX = T * K;
  double *v_l = reinterpret_cast<double *>(lds);
  double *s1 = v_l + NMAX;
  double *s2 = s1 + NMAX;
  S *g_l = reinterpret_cast<S *>(lds + p.lds_syn_off);
  uint64_t *ev = reinterpret_cast<uint64_t *>(lds + p.lds_ev_off);
  int *seg = reinterpret_cast<int *>(lds + p.lds_seg_off);
  int *misc = reinterpret_cast<int *>(lds + p.lds_misc_off);

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
  const int64_t nb = gd.node_base;
  const int64_t sb = gd.syn_base;
  const int32_t *lvl = p.lvl_start + gd.lvl_base;
  const int D = gd.n_levels;
  const int s_begin = (int)(n_begin - ival * M), s_end = (int)(n_end - ival * M);

  // ---- prologue: voltages and conductances on chip, this interval's events sorted
  for (int q = t; q < N; q += T) v_l[q] = p.v[nb + q];
  for (int s = t; s < gd.n_syn; s += T) g_l[s] = ld<S>(p.syn_g, sb + s);
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
  // per-node constants of the tree solve, in registers for the whole chunk
  double ra[K], rb[K], rd[K], rr[K], rdv[K];
  int rpar[K];
  uint32_t rch[K];
#pragma unroll
  for (int j = 0; j < K; ++j) {
    const int q = j * T + t;
    if (q < N) {
      ra[j] = p.nd_a[nb + q];
      rb[j] = p.nd_b[nb + q];
      rpar[j] = p.nd_par[nb + q];
      rch[j] = p.nd_ch[nb + q];
    } else {
      ra[j] = rb[j] = 0.0;
      rpar[j] = -1;
      rch[j] = 0;
    }
    rd[j] = 1.0;
    rr[j] = rdv[j] = 0.0;
  }
  __syncthreads();

  const S q10dt = (S)p.q10dt;
  const S sdt = (S)p.dt;
  const S ca_fm = (S)p.ca_fm, ca_fr = (S)p.ca_fr, ca_k = (S)p.ca_k;
  const bool has_hh_arr = p.hh_gna != nullptr;
  const bool has_pas_arr = p.pas_g != nullptr;

  for (int64_t n = n_begin; n < n_end; ++n) {
    const int s = (int)(n - ival * M);
    // ---- A: delivery (Sec. 2, event-driven delivery step)
    const int e0 = seg[s], e1 = seg[s + 1];
    if (e1 > e0) {
      for (int e = e0 + t; e < e1; e += T) {
        const uint32_t ls = ev_syn(ev[e]);
        if (e == e0 || ev_syn(ev[e - 1]) != ls) {
          S g = g_l[ls];
          for (int e2 = e; e2 < e1; ++e2) {
            const uint64_t key = ev[e2];
            if (ev_syn(key) != ls) break;
            const uint32_t id = (uint32_t)key & 0x7FFFFFFFu;
            g += ((uint32_t)key & EV_KIND_NETCON) ? ld<S>(p.nc_w, id) : ld<S>(p.kick_w, id);
          }
          g_l[ls] = g;
        }
      }
      __syncthreads();
    }
    // ---- C: states, currents, conductances and the compartment's own axial terms
    const bool pend = n > 0;
#pragma unroll
    for (int j = 0; j < K; ++j) {
      const int q = j * T + t;
      if (q < N) {
        const int64_t i = nb + q;
        const double v = v_l[q];
        double rhs = 0.0, d = 0.0;
        const uint32_t mf = p.nd_mf[i];
        if (mf & MF_HH) {
          S m = ld<S>(p.st[0], i), h = ld<S>(p.st[1], i), nn = ld<S>(p.st[2], i);
          if (pend) {
            hh_advance<S>(v, q10dt, m, h, nn);
            stv<S>(p.st[0], i, m);
            stv<S>(p.st[1], i, h);
            stv<S>(p.st[2], i, nn);
          }
          const double gnab = has_hh_arr ? p.hh_gna[i] : p.hh_gna_s;
          const double gkb = has_hh_arr ? p.hh_gk[i] : p.hh_gk_s;
          const double gl = has_hh_arr ? p.hh_gl[i] : p.hh_gl_s;
          const double el = has_hh_arr ? p.hh_el[i] : p.hh_el_s;
          const double gna = (double)((S)gnab * (m * m * m * h));
          const double gk = (double)((S)gkb * ((nn * nn) * (nn * nn)));
          rhs -= gna * (v - 50.0) + gk * (v + 77.0) + gl * (v - el);
          d += gna + gk + gl;
        }
        if (mf & MF_PAS) {
          const double g = has_pas_arr ? p.pas_g[i] : p.pas_g_s;
          const double e = has_pas_arr ? p.pas_e[i] : p.pas_e_s;
          rhs -= g * (v - e);
          d += g;
        }
        if (mf & MF_KM) {
          S nk = ld<S>(p.st[3], i);
          if (pend) {
            km_advance<S>(v, sdt, nk);
            stv<S>(p.st[3], i, nk);
          }
          const double g = (double)((S)(p.km_g ? p.km_g[i] : p.km_g_s) * nk);
          rhs -= g * (v + 77.0);
          d += g;
        }
        if (mf & MF_CAHI) {
          const S gca = (S)(p.ca_g ? p.ca_g[i] : p.ca_g_s);
          S mc = ld<S>(p.st[4], i);
          if (pend) {
            S cai = ld<S>(p.st[5], i);
            cahi_advance<S>(v, ca_fm, ca_fr, ca_k, gca, mc, cai);
            stv<S>(p.st[4], i, mc);
            stv<S>(p.st[5], i, cai);
          }
          const double g = (double)(gca * (mc * mc));
          rhs -= g * (v - 120.0);
          d += g;
        }
        const int2 ic = p.nd_icl[i];
        for (int c = 0; c < ic.y; ++c) {
          const int64_t k = gd.icl_base + ic.x + c;
          if (p.icl_on[k] <= n && n < p.icl_off[k]) rhs += p.icl_cur[k];
        }
        const int2 sy = p.nd_syn[i];
        if (sy.y > 0) {
          const double sa = p.nd_sa[i];
          for (int c = 0; c < sy.y; ++c) {
            const int ls = sy.x + c;
            const int64_t k = sb + ls;
            S g = g_l[ls];
            if (p.has_bg && (uint64_t)bg_word(p.seed, (uint64_t)p.syn_id[k], (uint64_t)n) < p.bg_thresh)
              g += ld<S>(p.syn_wbg, k);
            const double e = p.syn_e ? p.syn_e[k] : p.syn_e_s;
            const double gs = sa * (double)g;
            rhs -= gs * (v - e);
            d += gs;
            const S f = p.syn_f ? ld<S>(p.syn_f, k) : (S)p.syn_f_s;
            g_l[ls] = g * f;  // decay of this step, applied ahead of the next delivery
          }
        }
        d += p.nd_k[i];
        double dv = 0.0;
        if (rpar[j] >= 0) {
          dv = v_l[rpar[j]] - v;
          rhs -= rb[j] * dv;
        }
        rd[j] = d;
        rr[j] = rhs;
        rdv[j] = dv;
      }
    }
    // ---- T: elimination, deepest level first. A node's children publish cb = f b + a and cr = f rhs - a dv,
    // which fold the axial assembly terms of the parent's row into the elimination update.
    for (int L = D - 1; L >= 1; --L) {
      const int lo = lvl[L], hi = lvl[L + 1];
#pragma unroll
      for (int j = 0; j < K; ++j) {
        if (j * T < hi && j * T + T > lo) {
          const int q = j * T + t;
          if (q >= lo && q < hi) {
            double dd = rd[j], rr_ = rr[j];
            const int c0 = (int)(rch[j] & 0xFFFFu), cn = (int)(rch[j] >> 16);
            for (int c = c0; c < c0 + cn; ++c) {
              dd -= s1[c];
              rr_ -= s2[c];
            }
            const double r = 1.0 / dd;
            const double f = ra[j] * r;
            s1[q] = f * rb[j] + ra[j];
            s2[q] = f * rr_ - ra[j] * rdv[j];
            rd[j] = r;  // keep 1/d for the substitution
            rr[j] = rr_;
          }
        }
      }
      __syncthreads();
    }
    // ---- R: roots (level 0 holds the group's cells in order)
    {
      const int hi = lvl[1];
#pragma unroll
      for (int j = 0; j < K; ++j) {
        if (j * T < hi) {
          const int q = j * T + t;
          if (q < hi) {
            double dd = rd[j], rr_ = rr[j];
            const int c0 = (int)(rch[j] & 0xFFFFu), cn = (int)(rch[j] >> 16);
            for (int c = c0; c < c0 + cn; ++c) {
              dd -= s1[c];
              rr_ -= s2[c];
            }
            const double x = rr_ / dd;
            const double vold = v_l[q];
            const double vnew = vold + x;
            v_l[q] = vnew;
            s1[q] = x;
            const double th = p.cell_theta[gd.cell_base + q];
            if (vold < th && th <= vnew) {
              const int idx = atomicAdd(&misc[1], 1);
              p.gsp_pack[gd.spk_base + idx] = q | ((s + 1) << 16);
              p.gsp_frac[gd.spk_base + idx] = (th - vold) / (vnew - vold);
            }
            if (!isfinite(vnew)) atomicOr(&p.flags[FLAG_NONFINITE], 1);
          }
        }
      }
      __syncthreads();
    }
    // ---- B: substitution, root to leaves
    for (int L = 1; L < D; ++L) {
      const int lo = lvl[L], hi = lvl[L + 1];
#pragma unroll
      for (int j = 0; j < K; ++j) {
        if (j * T < hi && j * T + T > lo) {
          const int q = j * T + t;
          if (q >= lo && q < hi) {
            const double x = (rr[j] - rb[j] * s1[rpar[j]]) * rd[j];
            s1[q] = x;
            v_l[q] += x;
          }
        }
      }
      __syncthreads();
    }
  }

  // ---- epilogue: write back, record spikes, fan out through NetCons into the event ring
  for (int q = t; q < N; q += T) p.v[nb + q] = v_l[q];
  for (int s = t; s < gd.n_syn; s += T) stv<S>(p.syn_g, sb + s, g_l[s]);
  const int nsp = misc[1];
  for (int k = t; k < nsp; k += T) {
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
    for (int64_t o = o0 + t; o < o1; o += T) {
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
  if (t == 0 && n_end == (ival + 1) * (int64_t)M) p.ev_cnt[(int64_t)slot * p.n_groups + G] = 0;
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
  if (type == 0) {
    S m = ld<S>(p.st[0], i), h = ld<S>(p.st[1], i), nn = ld<S>(p.st[2], i);
    if (pend) hh_advance<S>(v, (S)p.q10dt, m, h, nn);
    out[i] = which == 0 ? (double)m : (which == 1 ? (double)h : (double)nn);
  } else if (type == 2) {
    S nk = ld<S>(p.st[3], i);
    if (pend) km_advance<S>(v, (S)p.dt, nk);
    out[i] = (double)nk;
  } else if (type == 3) {
    S mc = ld<S>(p.st[4], i), cai = ld<S>(p.st[5], i);
    if (pend) cahi_advance<S>(v, (S)p.ca_fm, (S)p.ca_fr, (S)p.ca_k, (S)(p.ca_g ? p.ca_g[i] : p.ca_g_s), mc, cai);
    out[i] = which == 0 ? (double)mc : (double)cai;
  }
}

// ------------------------------------------------------------------------------------------------------------------
// launch wrappers (host side)
using IntervalFn = void (*)(const KParams);

template <typename S>
static IntervalFn interval_fn_s(int threads, int slots) {
  if (threads == 256) {
    switch (slots) {
      case 1: return cn_interval<256, 1, S>;
      case 2: return cn_interval<256, 2, S>;
      case 4: return cn_interval<256, 4, S>;
      case 8: return cn_interval<256, 8, S>;
      default: break;
    }
  } else if (threads == 512) {
    switch (slots) {
      case 1: return cn_interval<512, 1, S>;
      case 2: return cn_interval<512, 2, S>;
      case 4: return cn_interval<512, 4, S>;
      default: break;
    }
  } else if (threads == 128) {
    switch (slots) {
      case 1: return cn_interval<128, 1, S>;
      case 2: return cn_interval<128, 2, S>;
      case 4: return cn_interval<128, 4, S>;
      case 8: return cn_interval<128, 8, S>;
      default: break;
    }
  }
  return nullptr;
}

static IntervalFn interval_fn(bool fp32, int threads, int slots) {
  return fp32 ? interval_fn_s<float>(threads, slots) : interval_fn_s<double>(threads, slots);
}

hipError_t set_interval_lds(bool fp32, int threads, int slots, int lds_bytes) {
  IntervalFn fn = interval_fn(fp32, threads, slots);
  if (!fn) return hipErrorInvalidValue;
  return hipFuncSetAttribute(reinterpret_cast<const void *>(fn), hipFuncAttributeMaxDynamicSharedMemorySize,
                             lds_bytes);
}

hipError_t launch_interval(const KParams &p, bool fp32, int threads, int slots, int lds_bytes, hipStream_t st) {
  IntervalFn fn = interval_fn(fp32, threads, slots);
  if (!fn) return hipErrorInvalidValue;
  hipLaunchKernelGGL(fn, dim3(p.n_groups), dim3(threads), lds_bytes, st, p);
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
