/*
 * Oracle: plain FP64 CPU simulator of the fixed-step cable-equation engine (CoreNEURON, arXiv 1901.10975).
 *
 * TEST INFRASTRUCTURE ONLY: loaded by the tests, the smoke check and the benchmark's CPU-baseline leg; never by the
 * product path, with which it shares no code. It is written to be checked by eye against the paper, not to be fast:
 * every step is done the obvious way, in the order the paper lists, in double precision, with no blocking, fusion or
 * reordering. Built with -ffp-contract=off so that each expression rounds as written.
 *
 * One step n -> n+1 (Sec. 2, the list of per-step operations):
 *   1. deliver the events due at step n (g += w per event), then the background events of step n;
 *   2. assemble the matrix: ionic and synaptic currents and their conductances at (v_n, states_n), the capacitive
 *      term and the axial coupling along the tree;
 *   3. solve it by Gaussian elimination from the leaves to the root and back (Hines), giving Delta-v;
 *   4. v += Delta-v, then advance the channel and synapse states with the new voltage;
 *   5. threshold detection at each cell's root; a spike's NetCon events are queued for step k + D.
 * Spikes are exchanged once per minimum-delay interval (Sec. 2): with batch_steps = M the queued events of an
 * interval's spikes are inserted only at the interval's end, which gives the same result because every NetCon delay
 * D is at least M.
 *
 * Readings of what the paper leaves open (each also listed in the design notes):
 *   R1 time scheme: first-order backward Euler in v with currents linearised at v_n (Sec. 2 "implicit integration";
 *      Sec. 3.5 "fixed time step"); states are staggered, advanced after the solve with v_{n+1}.
 *   R2 dI/dv: analytic conductance G of each current, which is linear in v at fixed states (Sec. 3.5, CONDUCTANCE).
 *   R3 gate update: x += (1 - exp(-dt/tau)) (xinf - x) with v frozen over the step.
 *   R4 hh: the Hodgkin-Huxley 1952 squid-axon rates in the modern sign convention (rest near -65 mV), ena = 50 mV,
 *      ek = -77 mV, q10 = 3^((celsius - 6.3)/10); vtrap(x, y) = x/(exp(x/y)-1), or y(1 - x/y/2) when |x/y| < 1e-6.
 *   R5 km and cahi are project-defined (pinned by held-voltage relaxation and steady-state tests):
 *      km:   ninf = 1/(1+exp(-(v+35)/10)), tau = 400/(3.3 exp((v+35)/20) + exp(-(v+35)/20)) ms, i = gbar n (v-ek);
 *      cahi: minf = 1/(1+exp(-(v+20)/9)), tau_m = 1 ms, i = gbar m^2 (v-eca), eca = 120 mV; calcium in a 0.1 um
 *            shell: dcai/dt = -1e4 ica/(2 F depth) - (cai - cai0)/tau_r, cai0 = 5e-5 mM, tau_r = 80 ms, integrated
 *            with the same exponential rule using ica at the new m and v.
 *   R6 point processes: a current I in nA at compartment i adds 100 I / A_i mA/cm^2 (Sec. 2, division by area).
 *   R7 delivery: D = floor(delay/dt + 0.5) steps; an event of a spike at step k is applied at the start of step
 *      k + D. Events of one step are applied kicks first (in kick order), then NetCon events by ascending NetCon
 *      index, then the background event.
 *   R8 threshold: a spike at step n+1 iff v_root(n) < theta <= v_root(n+1); reported time is the linear
 *      interpolation of the crossing within the step.
 *   R9 background: an event for synapse s at step n iff R(seed, k_s, n) < floor(p 2^32), p = rate dt 1e-3, where
 *      k_s is the synapse's stream id and R(seed, k, n) is word (n mod 4) of Philox4x32-10 with key (seed low,
 *      seed high) and counter (k low, k high, n/4 low, n/4 high). Its weight is that synapse's background weight.
 *   R10 IClamp: on for steps n with ceil(del/dt - 0.5) <= n < ceil((del+dur)/dt - 0.5).
 *   R11 ExpSyn: g decays as g exp(-dt/tau) after the solve; i = g (v - e) nA.
 *   R13 gap junctions: half-gap instances, each a current g (v_i - v_partner) nA at compartment i with the partner's
 *      potential from the start of the step and the own potential implicit (g on the diagonal).
 * Philox4x32-10 (R9) is parity unpinned: its statistics are tested, its identity with the published streams is not
 * (no known-answer vectors here).
 */
#include "orc.h"

#include <math.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define ENA 50.0
#define EK (-77.0)
#define ECA 120.0
#define CAI0 5e-5
#define TAU_R 80.0
#define DEPTH 0.1
#define FARADAY 96485.33212

static __thread char g_err[512];
static void set_err(const char *msg) { snprintf(g_err, sizeof g_err, "%s", msg); }
const char *orc_error(void) { return g_err; }

/* ------------------------------------------------------------------------------------------------------------- */
/* Philox4x32-10 (Salmon, Moraes, Dror, Shaw, SC'11): a 10-round bijection of a 128-bit counter under a 64-bit key.
 * Each round multiplies counter words 0 and 2 by fixed odd constants, keeping both halves of the 64-bit products,
 * and mixes the high halves with the other two words and the key; the key is bumped by Weyl constants between
 * rounds. */
static void mulhilo32(uint32_t a, uint32_t b, uint32_t *hi, uint32_t *lo) {
  uint64_t p = (uint64_t)a * (uint64_t)b;
  *hi = (uint32_t)(p >> 32);
  *lo = (uint32_t)p;
}

void orc_philox4x32_10(const uint32_t c_in[4], const uint32_t k_in[2], uint32_t out[4]) {
  uint32_t c[4] = {c_in[0], c_in[1], c_in[2], c_in[3]};
  uint32_t k0 = k_in[0], k1 = k_in[1];
  for (int r = 0; r < 10; ++r) {
    if (r > 0) {
      k0 += 0x9E3779B9u;
      k1 += 0xBB67AE85u;
    }
    uint32_t hi0, lo0, hi1, lo1;
    mulhilo32(0xD2511F53u, c[0], &hi0, &lo0);
    mulhilo32(0xCD9E8D57u, c[2], &hi1, &lo1);
    uint32_t n0 = hi1 ^ c[1] ^ k0;
    uint32_t n1 = lo1;
    uint32_t n2 = hi0 ^ c[3] ^ k1;
    uint32_t n3 = lo0;
    c[0] = n0; c[1] = n1; c[2] = n2; c[3] = n3;
  }
  out[0] = c[0]; out[1] = c[1]; out[2] = c[2]; out[3] = c[3];
}

uint32_t orc_poisson_draw(uint64_t seed, uint64_t syn, uint64_t step) {
  uint64_t blk = step / 4;
  uint32_t c[4] = {(uint32_t)syn, (uint32_t)(syn >> 32), (uint32_t)blk, (uint32_t)(blk >> 32)};
  uint32_t k[2] = {(uint32_t)seed, (uint32_t)(seed >> 32)};
  uint32_t out[4];
  orc_philox4x32_10(c, k, out);
  return out[step % 4];
}

/* ------------------------------------------------------------------------------------------------------------- */
/* Hines elimination for one cell (Sec. 2: direct Gaussian elimination of the tree system; Sec. 4.4: its number of
 * operations does not depend on the branching pattern). Row i holds d[i] on the diagonal, b[i] in column parent(i)
 * and, in row parent(i), a[i] in column i. Eliminate leaves-first (children have larger indices than their parent),
 * then substitute root-first. */
int64_t orc_hines(int32_t n, const int32_t *parent, const double *a, const double *b, double *d, double *rhs) {
  int64_t flops = 0;
  for (int32_t i = n - 1; i >= 1; --i) {
    int32_t p = parent[i];
    double f = a[i] / d[i];
    d[p] -= f * b[i];
    rhs[p] -= f * rhs[i];
    flops += 5;
  }
  rhs[0] /= d[0];
  flops += 1;
  for (int32_t i = 1; i < n; ++i) {
    int32_t p = parent[i];
    rhs[i] -= b[i] * rhs[p];
    rhs[i] /= d[i];
    flops += 3;
  }
  return flops;
}

/* ------------------------------------------------------------------------------------------------------------- */
/* rate functions (readings R4, R5) */
static double vtrap(double x, double y) {
  if (fabs(x / y) < 1e-6) return y * (1.0 - x / y / 2.0);
  return x / (exp(x / y) - 1.0);
}

typedef struct { double minf, mtau, hinf, htau, ninf, ntau; } hh_rates_t;

static hh_rates_t hh_rates(double v, double q10) {
  hh_rates_t r;
  double am = 0.1 * vtrap(-(v + 40.0), 10.0);
  double bm = 4.0 * exp(-(v + 65.0) / 18.0);
  double ah = 0.07 * exp(-(v + 65.0) / 20.0);
  double bh = 1.0 / (exp(-(v + 35.0) / 10.0) + 1.0);
  double an = 0.01 * vtrap(-(v + 55.0), 10.0);
  double bn = 0.125 * exp(-(v + 65.0) / 80.0);
  r.mtau = 1.0 / (q10 * (am + bm)); r.minf = am / (am + bm);
  r.htau = 1.0 / (q10 * (ah + bh)); r.hinf = ah / (ah + bh);
  r.ntau = 1.0 / (q10 * (an + bn)); r.ninf = an / (an + bn);
  return r;
}

static double km_ninf(double v) { return 1.0 / (1.0 + exp(-(v + 35.0) / 10.0)); }
static double km_tau(double v) { return 400.0 / (3.3 * exp((v + 35.0) / 20.0) + exp(-(v + 35.0) / 20.0)); }
static double cahi_minf(double v) { return 1.0 / (1.0 + exp(-(v + 20.0) / 9.0)); }

/* exponential update of one state toward xinf with time constant tau, v frozen over the step (reading R3) */
static double relax(double x, double xinf, double tau, double dt) { return x + (1.0 - exp(-dt / tau)) * (xinf - x); }

/* ------------------------------------------------------------------------------------------------------------- */
typedef struct { int64_t n, cap; int64_t *v; } ivec;
static int iv_push(ivec *a, int64_t x) {
  if (a->n == a->cap) {
    int64_t nc = a->cap ? 2 * a->cap : 16;
    int64_t *p = (int64_t *)realloc(a->v, (size_t)nc * sizeof *p);
    if (!p) return -1;
    a->v = p; a->cap = nc;
  }
  a->v[a->n++] = x;
  return 0;
}

typedef struct { int64_t *off; int64_t *idx; } csr_t; /* per-cell ascending instance lists */

struct orc_model {
  int32_t n_cells; int64_t n_comp;
  int64_t *cell_off; int32_t *parent; double *area, *a, *b, *c;
  double *v, *d, *rhs;
  double *last_d, *last_rhs, *last_dv; int keep_matrix;
  double dt, q10, v_init;
  /* mechanisms */
  int64_t n_hh; int64_t *hh_node; double *gna, *gk, *gl, *el, *hm, *hh, *hn; csr_t hh_c;
  int64_t n_pas; int64_t *pas_node; double *pas_g, *pas_e; csr_t pas_c;
  int64_t n_km; int64_t *km_node; double *km_g, *km_n; csr_t km_c;
  int64_t n_cahi; int64_t *cahi_node; double *ca_g, *ca_m, *ca_cai; csr_t cahi_c;
  int64_t n_syn; int64_t *syn_node; double *syn_e, *syn_f, *syn_g; csr_t syn_c;
  int64_t n_icl; int64_t *icl_node; double *icl_amp; int64_t *icl_on, *icl_off; csr_t icl_c;
  int64_t n_gap; int64_t *gap_node, *gap_partner; double *gap_g, *gap_vp; csr_t gap_c;
  /* network */
  int64_t n_nc; int64_t *nc_syn; double *nc_w; int64_t *nc_D; int64_t *out_off, *out_nc;
  double *theta;
  int64_t n_kick; int64_t *kick_step, *kick_syn; double *kick_w; int64_t kick_pos;
  double rate; double *pw; int64_t *pkey; uint64_t seed; uint64_t bg_thresh;
  int64_t Q; ivec *ring; int32_t M;
  ivec pend_gid, pend_step;
  /* run state */
  int64_t step;
  ivec sp_gid, sp_step; double *sp_t; int64_t sp_tcap;
  int64_t n_delivered;
  int n_threads;
  char *spiked; double *spike_t;
  uint64_t jitter; /* test hook: nonzero moves each potential by -1, 0 or +1 ulp after every step */
};

/* The rounding sensitivity probe behind orc_set_jitter: a counter-based choice of -1, 0 or +1 ulp for compartment i
 * after step n (SplitMix64 finaliser of the three numbers), the size of the difference two correctly rounded
 * implementations may have in any operation of a step. */
static double jitter_ulp(double v, uint64_t seed, int64_t i, int64_t n) {
  uint64_t z = seed ^ ((uint64_t)i * 0x9E3779B97F4A7C15ull) ^ ((uint64_t)n * 0xD1B54A32D192ED03ull);
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  z ^= z >> 31;
  switch ((z >> 32) % 3) {
    case 0: return nextafter(v, -INFINITY);
    case 1: return v;
    default: return nextafter(v, INFINITY);
  }
}

static void *xcalloc(size_t n, size_t s) { return calloc(n ? n : 1, s); }
#define DUP(dst, src, n, T) do { (dst) = (T *)xcalloc((size_t)(n), sizeof(T)); if (!(dst)) goto nomem; \
  if ((n) > 0) memcpy((dst), (src), (size_t)(n) * sizeof(T)); } while (0)

static int build_csr(csr_t *c, const int64_t *node, int64_t n, const int32_t *cell_of, int32_t n_cells) {
  c->off = (int64_t *)xcalloc((size_t)n_cells + 1, sizeof(int64_t));
  c->idx = (int64_t *)xcalloc((size_t)n, sizeof(int64_t));
  if (!c->off || !c->idx) return -1;
  for (int64_t k = 0; k < n; ++k) c->off[cell_of[node[k]] + 1]++;
  for (int32_t i = 0; i < n_cells; ++i) c->off[i + 1] += c->off[i];
  int64_t *fill = (int64_t *)xcalloc((size_t)n_cells, sizeof(int64_t));
  if (!fill) return -1;
  for (int64_t k = 0; k < n; ++k) {
    int32_t cl = cell_of[node[k]];
    c->idx[c->off[cl] + fill[cl]++] = k;
  }
  free(fill);
  return 0;
}

static int check_nodes(const int64_t *node, int64_t n, int64_t n_comp, int unique, const char *what) {
  char *seen = unique ? (char *)xcalloc((size_t)n_comp, 1) : NULL;
  for (int64_t k = 0; k < n; ++k) {
    if (node[k] < 0 || node[k] >= n_comp) {
      snprintf(g_err, sizeof g_err, "%s: instance %lld node out of range", what, (long long)k);
      free(seen);
      return -1;
    }
    if (unique) {
      if (seen[node[k]]) {
        snprintf(g_err, sizeof g_err, "%s: two instances at compartment %lld", what, (long long)node[k]);
        free(seen);
        return -1;
      }
      seen[node[k]] = 1;
    }
  }
  free(seen);
  return 0;
}

void orc_destroy(orc_model *m) {
  if (!m) return;
  void *ptrs[] = {m->cell_off, m->parent, m->area, m->a, m->b, m->c, m->v, m->d, m->rhs, m->last_d, m->last_rhs,
                  m->last_dv, m->hh_node, m->gna, m->gk, m->gl, m->el, m->hm, m->hh, m->hn, m->hh_c.off,
                  m->hh_c.idx, m->pas_node, m->pas_g, m->pas_e, m->pas_c.off, m->pas_c.idx, m->km_node, m->km_g,
                  m->km_n, m->km_c.off, m->km_c.idx, m->cahi_node, m->ca_g, m->ca_m, m->ca_cai, m->cahi_c.off,
                  m->cahi_c.idx, m->syn_node, m->syn_e, m->syn_f, m->syn_g, m->syn_c.off, m->syn_c.idx,
                  m->icl_node, m->icl_amp, m->icl_on, m->icl_off, m->icl_c.off, m->icl_c.idx, m->gap_node,
                  m->gap_partner, m->gap_g, m->gap_vp, m->gap_c.off, m->gap_c.idx, m->nc_syn, m->nc_w,
                  m->nc_D, m->out_off, m->out_nc, m->theta, m->kick_step, m->kick_syn, m->kick_w, m->pw, m->pkey,
                  m->pend_gid.v, m->pend_step.v, m->sp_gid.v, m->sp_step.v, m->sp_t, m->spiked, m->spike_t};
  for (size_t i = 0; i < sizeof ptrs / sizeof ptrs[0]; ++i) free(ptrs[i]);
  if (m->ring) {
    for (int64_t q = 0; q < m->Q; ++q) free(m->ring[q].v);
    free(m->ring);
  }
  free(m);
}

orc_model *orc_create(const orc_spec *s) {
  int32_t *cell_of = NULL;
  orc_model *m = (orc_model *)calloc(1, sizeof *m);
  if (!m) { set_err("out of memory"); return NULL; }
  if (s->n_cells <= 0 || s->n_comp <= 0 || !(s->dt > 0.0)) { set_err("empty model or dt <= 0"); goto fail; }
  if (s->cell_offset[0] != 0 || s->cell_offset[s->n_cells] != s->n_comp) { set_err("bad cell_offset"); goto fail; }
  for (int32_t c = 0; c < s->n_cells; ++c)
    if (s->cell_offset[c + 1] <= s->cell_offset[c]) { set_err("empty cell"); goto fail; }
  m->n_cells = s->n_cells; m->n_comp = s->n_comp; m->dt = s->dt; m->v_init = s->v_init;
  m->q10 = pow(3.0, (s->celsius - 6.3) / 10.0);
  m->keep_matrix = s->keep_matrix; m->n_threads = s->n_threads > 0 ? s->n_threads : 1;
  DUP(m->cell_off, s->cell_offset, s->n_cells + 1, int64_t);
  DUP(m->parent, s->parent, s->n_comp, int32_t);
  DUP(m->area, s->area, s->n_comp, double);
  cell_of = (int32_t *)xcalloc((size_t)s->n_comp, sizeof(int32_t));
  m->a = (double *)xcalloc((size_t)s->n_comp, sizeof(double));
  m->b = (double *)xcalloc((size_t)s->n_comp, sizeof(double));
  m->c = (double *)xcalloc((size_t)s->n_comp, sizeof(double));
  m->v = (double *)xcalloc((size_t)s->n_comp, sizeof(double));
  m->d = (double *)xcalloc((size_t)s->n_comp, sizeof(double));
  m->rhs = (double *)xcalloc((size_t)s->n_comp, sizeof(double));
  if (!cell_of || !m->a || !m->b || !m->c || !m->v || !m->d || !m->rhs) goto nomem;
  if (m->keep_matrix) {
    m->last_d = (double *)xcalloc((size_t)s->n_comp, sizeof(double));
    m->last_rhs = (double *)xcalloc((size_t)s->n_comp, sizeof(double));
    m->last_dv = (double *)xcalloc((size_t)s->n_comp, sizeof(double));
    if (!m->last_d || !m->last_rhs || !m->last_dv) goto nomem;
  }
  /* coefficients of the tree matrix (Sec. 2, Eq. 1 with its unit conventions): with the axial conductance
   * g = 1/ri (uS), a[i] = -100 g / A_parent and b[i] = -100 g / A_i are in S/cm^2; c = 1e-3 cm / dt likewise. */
  for (int32_t cl = 0; cl < s->n_cells; ++cl) {
    int64_t i0 = s->cell_offset[cl], n = s->cell_offset[cl + 1] - i0;
    for (int64_t k = 0; k < n; ++k) {
      int64_t i = i0 + k;
      int32_t p = s->parent[i];
      cell_of[i] = cl;
      if (!(s->area[i] > 0.0) || !(s->cm[i] > 0.0) || !isfinite(s->area[i]) || !isfinite(s->cm[i])) {
        set_err("area and cm must be positive and finite"); goto fail;
      }
      if (k == 0) {
        if (p != -1) { set_err("root parent must be -1"); goto fail; }
        continue;
      }
      if (p < 0 || p >= k) { set_err("parent[i] must lie in [0, i)"); goto fail; }
      if (!(s->ri[i] > 0.0) || !isfinite(s->ri[i])) { set_err("ri must be positive and finite"); goto fail; }
      double g = 1.0 / s->ri[i];
      m->a[i] = -100.0 * g / s->area[i0 + p];
      m->b[i] = -100.0 * g / s->area[i];
    }
  }
  for (int64_t i = 0; i < s->n_comp; ++i) {
    m->c[i] = 1e-3 * s->cm[i] / s->dt;
    m->v[i] = s->v_init;
  }
  /* mechanisms, with initial states at their steady-state values for v_init */
  if (check_nodes(s->hh_node, s->n_hh, s->n_comp, 1, "hh") || check_nodes(s->pas_node, s->n_pas, s->n_comp, 1, "pas")
      || check_nodes(s->km_node, s->n_km, s->n_comp, 1, "km") || check_nodes(s->cahi_node, s->n_cahi, s->n_comp, 1, "cahi")
      || check_nodes(s->syn_node, s->n_syn, s->n_comp, 0, "expsyn")
      || check_nodes(s->icl_node, s->n_icl, s->n_comp, 0, "iclamp")
      || check_nodes(s->gap_node, s->n_gap, s->n_comp, 0, "gap")
      || check_nodes(s->gap_partner, s->n_gap, s->n_comp, 0, "gap partner"))
    goto fail;
  m->n_hh = s->n_hh;
  DUP(m->hh_node, s->hh_node, s->n_hh, int64_t);
  DUP(m->gna, s->hh_gnabar, s->n_hh, double);
  DUP(m->gk, s->hh_gkbar, s->n_hh, double);
  DUP(m->gl, s->hh_gl, s->n_hh, double);
  DUP(m->el, s->hh_el, s->n_hh, double);
  m->hm = (double *)xcalloc((size_t)s->n_hh, sizeof(double));
  m->hh = (double *)xcalloc((size_t)s->n_hh, sizeof(double));
  m->hn = (double *)xcalloc((size_t)s->n_hh, sizeof(double));
  if (!m->hm || !m->hh || !m->hn) goto nomem;
  for (int64_t k = 0; k < s->n_hh; ++k) {
    hh_rates_t r = hh_rates(s->v_init, m->q10);
    m->hm[k] = r.minf; m->hh[k] = r.hinf; m->hn[k] = r.ninf;
  }
  m->n_pas = s->n_pas;
  DUP(m->pas_node, s->pas_node, s->n_pas, int64_t);
  DUP(m->pas_g, s->pas_g, s->n_pas, double);
  DUP(m->pas_e, s->pas_e, s->n_pas, double);
  m->n_km = s->n_km;
  DUP(m->km_node, s->km_node, s->n_km, int64_t);
  DUP(m->km_g, s->km_gbar, s->n_km, double);
  m->km_n = (double *)xcalloc((size_t)s->n_km, sizeof(double));
  if (!m->km_n) goto nomem;
  for (int64_t k = 0; k < s->n_km; ++k) m->km_n[k] = km_ninf(s->v_init);
  m->n_cahi = s->n_cahi;
  DUP(m->cahi_node, s->cahi_node, s->n_cahi, int64_t);
  DUP(m->ca_g, s->cahi_gbar, s->n_cahi, double);
  m->ca_m = (double *)xcalloc((size_t)s->n_cahi, sizeof(double));
  m->ca_cai = (double *)xcalloc((size_t)s->n_cahi, sizeof(double));
  if (!m->ca_m || !m->ca_cai) goto nomem;
  for (int64_t k = 0; k < s->n_cahi; ++k) { m->ca_m[k] = cahi_minf(s->v_init); m->ca_cai[k] = CAI0; }
  m->n_syn = s->n_syn;
  DUP(m->syn_node, s->syn_node, s->n_syn, int64_t);
  DUP(m->syn_e, s->syn_e, s->n_syn, double);
  m->syn_f = (double *)xcalloc((size_t)s->n_syn, sizeof(double));
  m->syn_g = (double *)xcalloc((size_t)s->n_syn, sizeof(double));
  if (!m->syn_f || !m->syn_g) goto nomem;
  for (int64_t k = 0; k < s->n_syn; ++k) {
    if (!(s->syn_tau[k] > 0.0)) { set_err("expsyn tau must be positive"); goto fail; }
    m->syn_f[k] = exp(-s->dt / s->syn_tau[k]);
  }
  m->n_icl = s->n_icl;
  DUP(m->icl_node, s->icl_node, s->n_icl, int64_t);
  DUP(m->icl_amp, s->icl_amp, s->n_icl, double);
  m->icl_on = (int64_t *)xcalloc((size_t)s->n_icl, sizeof(int64_t));
  m->icl_off = (int64_t *)xcalloc((size_t)s->n_icl, sizeof(int64_t));
  if (!m->icl_on || !m->icl_off) goto nomem;
  for (int64_t k = 0; k < s->n_icl; ++k) {
    m->icl_on[k] = (int64_t)ceil(s->icl_del[k] / s->dt - 0.5);
    m->icl_off[k] = (int64_t)ceil((s->icl_del[k] + s->icl_dur[k]) / s->dt - 0.5);
  }
  m->n_gap = s->n_gap;
  DUP(m->gap_node, s->gap_node, s->n_gap, int64_t);
  DUP(m->gap_partner, s->gap_partner, s->n_gap, int64_t);
  DUP(m->gap_g, s->gap_g, s->n_gap, double);
  m->gap_vp = (double *)xcalloc((size_t)s->n_gap, sizeof(double));
  if (s->n_gap && !m->gap_vp) goto nomem;
  for (int64_t k = 0; k < s->n_gap; ++k)
    if (!(s->gap_g[k] >= 0.0) || !isfinite(s->gap_g[k])) { set_err("gap conductance must be finite and >= 0"); goto fail; }
  if (build_csr(&m->gap_c, m->gap_node, m->n_gap, cell_of, m->n_cells) ||
      build_csr(&m->hh_c, m->hh_node, m->n_hh, cell_of, m->n_cells) ||
      build_csr(&m->pas_c, m->pas_node, m->n_pas, cell_of, m->n_cells) ||
      build_csr(&m->km_c, m->km_node, m->n_km, cell_of, m->n_cells) ||
      build_csr(&m->cahi_c, m->cahi_node, m->n_cahi, cell_of, m->n_cells) ||
      build_csr(&m->syn_c, m->syn_node, m->n_syn, cell_of, m->n_cells) ||
      build_csr(&m->icl_c, m->icl_node, m->n_icl, cell_of, m->n_cells))
    goto nomem;
  /* network */
  m->n_nc = s->n_nc;
  DUP(m->nc_syn, s->nc_syn, s->n_nc, int64_t);
  DUP(m->nc_w, s->nc_w, s->n_nc, double);
  DUP(m->theta, s->threshold, s->n_cells, double);
  m->nc_D = (int64_t *)xcalloc((size_t)s->n_nc, sizeof(int64_t));
  m->out_off = (int64_t *)xcalloc((size_t)s->n_cells + 1, sizeof(int64_t));
  m->out_nc = (int64_t *)xcalloc((size_t)s->n_nc, sizeof(int64_t));
  if (!m->nc_D || !m->out_off || !m->out_nc) goto nomem;
  int64_t maxD = 1, minD = INT64_MAX;
  for (int64_t k = 0; k < s->n_nc; ++k) {
    if (s->nc_src[k] < 0 || s->nc_src[k] >= s->n_cells) { set_err("netcon source out of range"); goto fail; }
    if (s->nc_syn[k] < 0 || s->nc_syn[k] >= s->n_syn) { set_err("netcon target out of range"); goto fail; }
    int64_t D = (int64_t)floor(s->nc_delay[k] / s->dt + 0.5);
    if (D < 1) { set_err("netcon delay shorter than one step"); goto fail; }
    m->nc_D[k] = D;
    if (D > maxD) maxD = D;
    if (D < minD) minD = D;
    m->out_off[s->nc_src[k] + 1]++;
  }
  for (int32_t c = 0; c < s->n_cells; ++c) m->out_off[c + 1] += m->out_off[c];
  {
    int64_t *fill = (int64_t *)xcalloc((size_t)s->n_cells, sizeof(int64_t));
    if (!fill) goto nomem;
    for (int64_t k = 0; k < s->n_nc; ++k) m->out_nc[m->out_off[s->nc_src[k]] + fill[s->nc_src[k]]++] = k;
    free(fill);
  }
  m->M = s->batch_steps;
  if (m->M < 0 || (m->M > 0 && s->n_nc > 0 && m->M > minD)) { set_err("batch_steps must not exceed the minimum delay"); goto fail; }
  m->Q = maxD + 2;
  m->ring = (ivec *)xcalloc((size_t)m->Q, sizeof(ivec));
  if (!m->ring) goto nomem;
  /* kicks, stably ordered by step so that kicks of one step keep their list order */
  m->n_kick = s->n_kick;
  m->kick_step = (int64_t *)xcalloc((size_t)s->n_kick, sizeof(int64_t));
  m->kick_syn = (int64_t *)xcalloc((size_t)s->n_kick, sizeof(int64_t));
  m->kick_w = (double *)xcalloc((size_t)s->n_kick, sizeof(double));
  if (!m->kick_step || !m->kick_syn || !m->kick_w) goto nomem;
  {
    int64_t w = 0;
    /* counting by a stable insertion sort on step: kick lists are short */
    for (int64_t k = 0; k < s->n_kick; ++k) {
      if (s->kick_step[k] < 0 || s->kick_syn[k] < 0 || s->kick_syn[k] >= s->n_syn) { set_err("bad kick"); goto fail; }
      int64_t j = w++;
      while (j > 0 && m->kick_step[j - 1] > s->kick_step[k]) {
        m->kick_step[j] = m->kick_step[j - 1]; m->kick_syn[j] = m->kick_syn[j - 1]; m->kick_w[j] = m->kick_w[j - 1];
        --j;
      }
      m->kick_step[j] = s->kick_step[k]; m->kick_syn[j] = s->kick_syn[k]; m->kick_w[j] = s->kick_w[k];
    }
  }
  m->rate = s->poisson_rate_hz;
  m->seed = s->seed;
  if (m->rate > 0.0) {
    DUP(m->pw, s->poisson_w, s->n_syn, double);
    DUP(m->pkey, s->poisson_key, s->n_syn, int64_t);
    for (int64_t k = 0; k < s->n_syn; ++k)
      if (m->pkey[k] < 0) { set_err("negative background stream id"); goto fail; }
    double p = m->rate * s->dt * 1e-3;
    double t = floor(p * 4294967296.0);
    m->bg_thresh = t >= 4294967296.0 ? (uint64_t)4294967296ULL : (uint64_t)t;
  }
  m->spiked = (char *)xcalloc((size_t)s->n_cells, 1);
  m->spike_t = (double *)xcalloc((size_t)s->n_cells, sizeof(double));
  if (!m->spiked || !m->spike_t) goto nomem;
  free(cell_of);
  return m;
nomem:
  set_err("out of memory");
fail:
  free(cell_of);
  orc_destroy(m);
  return NULL;
}

/* step 1 of Sec. 2's list: event-driven delivery at the start of step n (reading R7, R9) */
static int deliver(orc_model *m, int64_t n) {
  while (m->kick_pos < m->n_kick && m->kick_step[m->kick_pos] < n) m->kick_pos++; /* kicks before the start */
  while (m->kick_pos < m->n_kick && m->kick_step[m->kick_pos] == n) {
    m->syn_g[m->kick_syn[m->kick_pos]] += m->kick_w[m->kick_pos];
    m->kick_pos++;
    m->n_delivered++;
  }
  ivec *bk = &m->ring[n % m->Q];
  /* NetCon events of this step by ascending NetCon index (simple insertion sort: buckets are short) */
  for (int64_t i = 1; i < bk->n; ++i) {
    int64_t x = bk->v[i], j = i;
    while (j > 0 && bk->v[j - 1] > x) { bk->v[j] = bk->v[j - 1]; --j; }
    bk->v[j] = x;
  }
  for (int64_t i = 0; i < bk->n; ++i) m->syn_g[m->nc_syn[bk->v[i]]] += m->nc_w[bk->v[i]];
  m->n_delivered += bk->n;
  bk->n = 0;
  if (m->rate > 0.0) {
    int64_t cnt = 0;
#pragma omp parallel for num_threads(m->n_threads) reduction(+ : cnt) schedule(static)
    for (int64_t sy = 0; sy < m->n_syn; ++sy) {
      if ((uint64_t)orc_poisson_draw(m->seed, (uint64_t)m->pkey[sy], (uint64_t)n) < m->bg_thresh) {
        m->syn_g[sy] += m->pw[sy];
        cnt++;
      }
    }
    m->n_delivered += cnt;
  }
  return 0;
}

/* steps 2-5 of Sec. 2's list for one cell */
static void cell_step(orc_model *m, int32_t cl, int64_t n) {
  const double dt = m->dt;
  const int64_t i0 = m->cell_off[cl], nn = m->cell_off[cl + 1] - i0;
  double *v = m->v, *d = m->d, *rhs = m->rhs;
  for (int64_t i = i0; i < i0 + nn; ++i) { rhs[i] = 0.0; d[i] = 0.0; }
  /* currents and conductances at (v_n, states_n), mechanisms in the fixed order hh, pas, km, cahi, IClamp, ExpSyn
   * (Sec. 2, matrix assembly; reading R2 for the conductances) */
  for (int64_t q = m->hh_c.off[cl]; q < m->hh_c.off[cl + 1]; ++q) {
    int64_t k = m->hh_c.idx[q], i = m->hh_node[k];
    double mm = m->hm[k], hh = m->hh[k], nk = m->hn[k];
    double gna = m->gna[k] * mm * mm * mm * hh;
    double gk = m->gk[k] * nk * nk * nk * nk;
    double cur = gna * (v[i] - ENA) + gk * (v[i] - EK) + m->gl[k] * (v[i] - m->el[k]);
    rhs[i] -= cur;
    d[i] += gna + gk + m->gl[k];
  }
  for (int64_t q = m->pas_c.off[cl]; q < m->pas_c.off[cl + 1]; ++q) {
    int64_t k = m->pas_c.idx[q], i = m->pas_node[k];
    rhs[i] -= m->pas_g[k] * (v[i] - m->pas_e[k]);
    d[i] += m->pas_g[k];
  }
  for (int64_t q = m->km_c.off[cl]; q < m->km_c.off[cl + 1]; ++q) {
    int64_t k = m->km_c.idx[q], i = m->km_node[k];
    double g = m->km_g[k] * m->km_n[k];
    rhs[i] -= g * (v[i] - EK);
    d[i] += g;
  }
  for (int64_t q = m->cahi_c.off[cl]; q < m->cahi_c.off[cl + 1]; ++q) {
    int64_t k = m->cahi_c.idx[q], i = m->cahi_node[k];
    double g = m->ca_g[k] * m->ca_m[k] * m->ca_m[k];
    rhs[i] -= g * (v[i] - ECA);
    d[i] += g;
  }
  for (int64_t q = m->icl_c.off[cl]; q < m->icl_c.off[cl + 1]; ++q) {
    int64_t k = m->icl_c.idx[q], i = m->icl_node[k];
    if (m->icl_on[k] <= n && n < m->icl_off[k]) rhs[i] += 100.0 * m->icl_amp[k] / m->area[i];
  }
  for (int64_t q = m->syn_c.off[cl]; q < m->syn_c.off[cl + 1]; ++q) {
    int64_t k = m->syn_c.idx[q], i = m->syn_node[k];
    rhs[i] -= 100.0 * m->syn_g[k] * (v[i] - m->syn_e[k]) / m->area[i];
    d[i] += 100.0 * m->syn_g[k] / m->area[i];
  }
  /* half-gaps (reading R13): current g (v_i - v_partner) with the partner's potential from the start of the step,
   * conductance g on the diagonal, both divided by area like every point process */
  for (int64_t q = m->gap_c.off[cl]; q < m->gap_c.off[cl + 1]; ++q) {
    int64_t k = m->gap_c.idx[q], i = m->gap_node[k];
    rhs[i] -= 100.0 * m->gap_g[k] * (v[i] - m->gap_vp[k]) / m->area[i];
    d[i] += 100.0 * m->gap_g[k] / m->area[i];
  }
  /* capacitive term and axial coupling */
  for (int64_t i = i0; i < i0 + nn; ++i) d[i] += m->c[i];
  for (int64_t k = 1; k < nn; ++k) {
    int64_t i = i0 + k, p = i0 + m->parent[i];
    double dv = v[p] - v[i];
    rhs[i] -= m->b[i] * dv;
    rhs[p] += m->a[i] * dv;
    d[i] -= m->b[i];
    d[p] -= m->a[i];
  }
  if (m->keep_matrix)
    for (int64_t i = i0; i < i0 + nn; ++i) { m->last_d[i] = d[i]; m->last_rhs[i] = rhs[i]; }
  /* matrix resolution */
  orc_hines((int32_t)nn, m->parent + i0, m->a + i0, m->b + i0, d + i0, rhs + i0);
  if (m->keep_matrix)
    for (int64_t i = i0; i < i0 + nn; ++i) m->last_dv[i] = rhs[i];
  double v_root_old = v[i0];
  for (int64_t i = i0; i < i0 + nn; ++i) v[i] += rhs[i];
  if (m->jitter)
    for (int64_t i = i0; i < i0 + nn; ++i) v[i] = jitter_ulp(v[i], m->jitter, i, n);
  /* state update with v_{n+1} (reading R1, R3, R5, R11) */
  for (int64_t q = m->hh_c.off[cl]; q < m->hh_c.off[cl + 1]; ++q) {
    int64_t k = m->hh_c.idx[q];
    hh_rates_t r = hh_rates(v[m->hh_node[k]], m->q10);
    m->hm[k] = relax(m->hm[k], r.minf, r.mtau, dt);
    m->hh[k] = relax(m->hh[k], r.hinf, r.htau, dt);
    m->hn[k] = relax(m->hn[k], r.ninf, r.ntau, dt);
  }
  for (int64_t q = m->km_c.off[cl]; q < m->km_c.off[cl + 1]; ++q) {
    int64_t k = m->km_c.idx[q];
    double vv = v[m->km_node[k]];
    m->km_n[k] = relax(m->km_n[k], km_ninf(vv), km_tau(vv), dt);
  }
  for (int64_t q = m->cahi_c.off[cl]; q < m->cahi_c.off[cl + 1]; ++q) {
    int64_t k = m->cahi_c.idx[q];
    double vv = v[m->cahi_node[k]];
    m->ca_m[k] = relax(m->ca_m[k], cahi_minf(vv), 1.0, dt);
    double ica = m->ca_g[k] * m->ca_m[k] * m->ca_m[k] * (vv - ECA);
    double cainf = CAI0 - 1e4 * ica / (2.0 * FARADAY * DEPTH) * TAU_R;
    m->ca_cai[k] = relax(m->ca_cai[k], cainf, TAU_R, dt);
  }
  for (int64_t q = m->syn_c.off[cl]; q < m->syn_c.off[cl + 1]; ++q) {
    int64_t k = m->syn_c.idx[q];
    m->syn_g[k] *= m->syn_f[k];
  }
  /* threshold detection at the root (reading R8) */
  double th = m->theta[cl], v_new = v[i0];
  m->spiked[cl] = 0;
  if (v_root_old < th && th <= v_new) {
    m->spiked[cl] = 1;
    m->spike_t[cl] = ((double)n + (th - v_root_old) / (v_new - v_root_old)) * dt;
  }
}

static int fan_out(orc_model *m, int64_t gid, int64_t k) {
  for (int64_t q = m->out_off[gid]; q < m->out_off[gid + 1]; ++q) {
    int64_t nc = m->out_nc[q];
    if (iv_push(&m->ring[(k + m->nc_D[nc]) % m->Q], nc)) return -1;
  }
  return 0;
}

int orc_run(orc_model *m, int64_t n_target) {
  if (!m) { set_err("null model"); return -1; }
  if (n_target < m->step) { set_err("cannot run backwards"); return -1; }
  for (int64_t n = m->step; n < n_target; ++n) {
    deliver(m, n);
    /* the partners' potentials at the start of the step, before any cell advances */
    for (int64_t k = 0; k < m->n_gap; ++k) m->gap_vp[k] = m->v[m->gap_partner[k]];
#pragma omp parallel for num_threads(m->n_threads) schedule(dynamic, 16)
    for (int32_t cl = 0; cl < m->n_cells; ++cl) cell_step(m, cl, n);
    /* record spikes and queue their events in cell order */
    for (int32_t cl = 0; cl < m->n_cells; ++cl) {
      if (!m->spiked[cl]) continue;
      if (iv_push(&m->sp_gid, cl) || iv_push(&m->sp_step, n + 1)) { set_err("out of memory"); return -1; }
      if (m->sp_gid.n > m->sp_tcap) {
        int64_t nc = m->sp_tcap ? 2 * m->sp_tcap : 64;
        double *p = (double *)realloc(m->sp_t, (size_t)nc * sizeof(double));
        if (!p) { set_err("out of memory"); return -1; }
        m->sp_t = p; m->sp_tcap = nc;
      }
      m->sp_t[m->sp_gid.n - 1] = m->spike_t[cl];
      if (m->M > 0) {
        if (iv_push(&m->pend_gid, cl) || iv_push(&m->pend_step, n + 1)) { set_err("out of memory"); return -1; }
      } else if (fan_out(m, cl, n + 1)) {
        set_err("out of memory"); return -1;
      }
    }
    /* spike exchange at the end of each minimum-delay interval (Sec. 2) */
    if (m->M > 0 && (n + 1) % m->M == 0) {
      for (int64_t q = 0; q < m->pend_gid.n; ++q)
        if (fan_out(m, m->pend_gid.v[q], m->pend_step.v[q])) { set_err("out of memory"); return -1; }
      m->pend_gid.n = 0; m->pend_step.n = 0;
    }
    m->step = n + 1;
  }
  return 0;
}

/* Checkpoint-restart (Sec. 3.4): a run continues from a saved state - the step, the potentials, the mechanism
 * states and the synaptic conductances - with the events that were still travelling at the checkpoint recovered
 * from the spikes that sent them, instead of a saved event queue: every NetCon of a given spike (gid, k) whose
 * arrival step k + D lies at or after the restart step is queued again. The model must not have run yet. */
int orc_restore(orc_model *m, int64_t step, const double *v, const double *hh_m, const double *hh_h,
                const double *hh_n, const double *km_n, const double *cahi_m, const double *cahi_cai,
                const double *syn_g, int64_t n_spk, const int32_t *spk_gid, const int64_t *spk_step) {
  if (!m) { set_err("null model"); return -1; }
  if (m->step != 0 || m->sp_gid.n != 0) { set_err("restore needs a model that has not run"); return -1; }
  if (step < 0) { set_err("negative restart step"); return -1; }
  memcpy(m->v, v, (size_t)m->n_comp * sizeof(double));
  if (m->n_hh) {
    memcpy(m->hm, hh_m, (size_t)m->n_hh * sizeof(double));
    memcpy(m->hh, hh_h, (size_t)m->n_hh * sizeof(double));
    memcpy(m->hn, hh_n, (size_t)m->n_hh * sizeof(double));
  }
  if (m->n_km) memcpy(m->km_n, km_n, (size_t)m->n_km * sizeof(double));
  if (m->n_cahi) {
    memcpy(m->ca_m, cahi_m, (size_t)m->n_cahi * sizeof(double));
    memcpy(m->ca_cai, cahi_cai, (size_t)m->n_cahi * sizeof(double));
  }
  if (m->n_syn) memcpy(m->syn_g, syn_g, (size_t)m->n_syn * sizeof(double));
  for (int64_t q = 0; q < n_spk; ++q) {
    const int64_t gid = spk_gid[q], k = spk_step[q];
    if (gid < 0 || gid >= m->n_cells || k > step) { set_err("bad checkpoint spike"); return -1; }
    for (int64_t o = m->out_off[gid]; o < m->out_off[gid + 1]; ++o) {
      const int64_t nc = m->out_nc[o];
      const int64_t due = k + m->nc_D[nc];
      if (due < step) continue; /* delivered before the checkpoint */
      if (due - step >= m->Q) { set_err("checkpoint spike beyond the event horizon"); return -1; }
      if (iv_push(&m->ring[due % m->Q], nc)) { set_err("out of memory"); return -1; }
    }
  }
  m->step = step;
  return 0;
}

void orc_set_jitter(orc_model *m, uint64_t seed) { m->jitter = seed; }

/* new key for the background streams from the current step on (a restart with other random streams) */
void orc_set_seed(orc_model *m, uint64_t seed) { m->seed = seed; }

int64_t orc_step(const orc_model *m) { return m->step; }
int64_t orc_n_spikes(const orc_model *m) { return m->sp_gid.n; }
int64_t orc_n_delivered(const orc_model *m) { return m->n_delivered; }

void orc_get_spikes(const orc_model *m, int32_t *gid, int64_t *step, double *t) {
  for (int64_t q = 0; q < m->sp_gid.n; ++q) {
    if (gid) gid[q] = (int32_t)m->sp_gid.v[q];
    if (step) step[q] = m->sp_step.v[q];
    if (t) t[q] = m->sp_t[q];
  }
}

void orc_get_v(const orc_model *m, double *v) { memcpy(v, m->v, (size_t)m->n_comp * sizeof(double)); }

void orc_get_states(const orc_model *m, double *hh_m, double *hh_h, double *hh_n, double *km_n, double *cahi_m,
                    double *cahi_cai, double *syn_g) {
  if (hh_m) memcpy(hh_m, m->hm, (size_t)m->n_hh * sizeof(double));
  if (hh_h) memcpy(hh_h, m->hh, (size_t)m->n_hh * sizeof(double));
  if (hh_n) memcpy(hh_n, m->hn, (size_t)m->n_hh * sizeof(double));
  if (km_n) memcpy(km_n, m->km_n, (size_t)m->n_km * sizeof(double));
  if (cahi_m) memcpy(cahi_m, m->ca_m, (size_t)m->n_cahi * sizeof(double));
  if (cahi_cai) memcpy(cahi_cai, m->ca_cai, (size_t)m->n_cahi * sizeof(double));
  if (syn_g) memcpy(syn_g, m->syn_g, (size_t)m->n_syn * sizeof(double));
}

void orc_get_last_matrix(const orc_model *m, double *d, double *rhs, double *dv) {
  if (!m->keep_matrix) return;
  if (d) memcpy(d, m->last_d, (size_t)m->n_comp * sizeof(double));
  if (rhs) memcpy(rhs, m->last_rhs, (size_t)m->n_comp * sizeof(double));
  if (dv) memcpy(dv, m->last_dv, (size_t)m->n_comp * sizeof(double));
}
