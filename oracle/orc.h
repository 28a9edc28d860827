/*
 * Oracle: a plain, slow FP64 CPU simulator of the fixed-step cable-equation engine.
 *
 * TEST INFRASTRUCTURE ONLY. Only the test-suite, the smoke check and the benchmark's CPU-baseline leg may load
 * this library. The product path (the HIP library under paper_1901_10975_amd/) never calls, links or includes it,
 * and this file shares no code with that path.
 *
 * What it computes follows the paper (CoreNEURON, arXiv 1901.10975):
 *   - Sec. 2, Eq. 1: the cable equation per compartment, currents in mA/cm^2, point currents in nA divided by
 *     compartment area;
 *   - Sec. 2: implicit integration of the tree system by Gaussian elimination ordered from the leaves (Hines);
 *   - Sec. 2: the per-step operations in their stated order (event delivery, matrix assembly with ionic and
 *     synaptic contributions, matrix solve, state update, threshold detection) and spike exchange once per
 *     minimum-delay interval;
 *   - Sec. 3.5: fixed time step only; analytic conductances (the CONDUCTANCE hint); counter-based random streams
 *     (Random123; here Philox4x32-10).
 * Readings of points the paper leaves open are listed in the repository's design notes and in orc.c.
 *
 * Arrays are borrowed for the duration of orc_create and deep-copied. Every array must be given (no NULL
 * shortcuts): scalar parameters are expanded by the caller.
 */
#ifndef CN_ORACLE_ORC_H
#define CN_ORACLE_ORC_H
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct orc_spec {
  /* topology: cells are contiguous compartment ranges; parent is cell-local, -1 at the root, parent[i] < i */
  int32_t n_cells;
  int64_t n_comp;
  const int64_t *cell_offset; /* [n_cells+1] */
  const int32_t *parent;      /* [n_comp] */
  const double *area;         /* [n_comp] um^2 */
  const double *ri;           /* [n_comp] MOhm to parent, ignored at roots */
  const double *cm;           /* [n_comp] uF/cm^2 */
  double v_init, celsius;
  /* density mechanisms: at most one instance per compartment */
  int64_t n_hh;   const int64_t *hh_node;   const double *hh_gnabar, *hh_gkbar, *hh_gl, *hh_el;
  int64_t n_pas;  const int64_t *pas_node;  const double *pas_g, *pas_e;
  int64_t n_km;   const int64_t *km_node;   const double *km_gbar;
  int64_t n_cahi; const int64_t *cahi_node; const double *cahi_gbar;
  /* point processes */
  int64_t n_syn;  const int64_t *syn_node;  const double *syn_tau, *syn_e;
  int64_t n_icl;  const int64_t *icl_node;  const double *icl_del, *icl_dur, *icl_amp;
  /* gap junctions, as half-gap instances: the current g (v_node - v_partner) nA at node, with the partner's
   * potential taken at the start of the step (reading R13); a junction between two compartments is two instances */
  int64_t n_gap;  const int64_t *gap_node, *gap_partner; const double *gap_g;
  /* network */
  int64_t n_nc; const int32_t *nc_src; const int64_t *nc_syn; const double *nc_w, *nc_delay;
  const double *threshold; /* [n_cells] mV */
  int64_t n_kick; const int64_t *kick_step, *kick_syn; const double *kick_w;
  double poisson_rate_hz; const double *poisson_w; /* [n_syn] */
  const int64_t *poisson_key; /* [n_syn] stream id of each synapse */
  uint64_t seed;
  double dt;
  int32_t batch_steps; /* 0: spikes fan out at once; M > 0: spikes fan out at the end of each M-step interval */
  int32_t n_threads;   /* OpenMP threads for the per-cell loop (<= 0: 1) */
  int32_t keep_matrix; /* nonzero: keep d, rhs and Delta-v of the last step for orc_get_last_matrix */
} orc_spec;

typedef struct orc_model orc_model;

const char *orc_error(void);
orc_model *orc_create(const orc_spec *spec);
void orc_destroy(orc_model *m);
/* advance to absolute step n_target (t = n*dt); returns 0, or -1 with orc_error() set */
int orc_run(orc_model *m, int64_t n_target);
int64_t orc_step(const orc_model *m);
int64_t orc_n_spikes(const orc_model *m);
/* spikes in (step, gid) order: cell id, step index, linearly interpolated crossing time (ms) */
void orc_get_spikes(const orc_model *m, int32_t *gid, int64_t *step, double *t);
void orc_get_v(const orc_model *m, double *v);
/* mechanism states in instance order; NULL pointers are skipped */
void orc_get_states(const orc_model *m, double *hh_m, double *hh_h, double *hh_n, double *km_n, double *cahi_m,
                    double *cahi_cai, double *syn_g);
/* per-step matrix terms of the last completed step, for the charge-balance check: d and rhs after assembly
 * (before elimination) and the Delta-v solution */
void orc_get_last_matrix(const orc_model *m, double *d, double *rhs, double *dv);
/* number of network events delivered so far (kicks + NetCon events + background events) */
int64_t orc_n_delivered(const orc_model *m);

/* Checkpoint-restart (Sec. 3.4): continue from a saved step, potentials, mechanism states and conductances (arrays
 * laid out as orc_get_v / orc_get_states give them; NULL for absent mechanisms); the events still in flight at that
 * step are re-queued from the spikes (gid, step) that sent them. The model must not have run. 0 or -1. */
int orc_restore(orc_model *m, int64_t step, const double *v, const double *hh_m, const double *hh_h,
                const double *hh_n, const double *km_n, const double *cahi_m, const double *cahi_cai,
                const double *syn_g, int64_t n_spk, const int32_t *spk_gid, const int64_t *spk_step);
/* key of the background streams from the current step on */
void orc_set_seed(orc_model *m, uint64_t seed);

/* Test hook, a rounding-sensitivity probe (not part of the method): with seed != 0, after every step each
 * compartment's potential moves by -1, 0 or +1 ulp, chosen by a counter-based hash of (seed, compartment, step). Two
 * FP64 implementations that evaluate the same step with different but correctly rounded operations differ by about
 * this much per step; the spread this member shows is the deviation such an implementation may have from the oracle.
 * 0 turns it off (the default). */
void orc_set_jitter(orc_model *m, uint64_t seed);

/* Test hooks.
 * Hines elimination of one tree of n nodes in place (Sec. 2; Sec. 4.4 on its operation count): on return rhs
 * holds the solution. Returns the number of floating-point operations performed. */
int64_t orc_hines(int32_t n, const int32_t *parent, const double *a, const double *b, double *d, double *rhs);
/* the 32-bit uniform draw R(seed, syn, step) behind the background events */
uint32_t orc_poisson_draw(uint64_t seed, uint64_t syn, uint64_t step);
/* the four 32-bit words of Philox4x32-10 for counter c and key k */
void orc_philox4x32_10(const uint32_t c[4], const uint32_t k[2], uint32_t out[4]);

#ifdef __cplusplus
}
#endif
#endif
