/*
 * cn: an MI355X (gfx950) engine for the fixed-step cable equation over many multi-compartment neurons.
 *
 * The operation this library performs is the per-time-step computation of CoreNEURON (arXiv 1901.10975):
 * each cell is a tree of compartments obeying the cable equation (Sec. 2, Eq. 1); every step delivers the synaptic
 * events that are due, assembles the tree matrix from ionic and synaptic currents, solves it by Gaussian
 * elimination ordered from the leaves (Hines), updates channel and synapse states, and tests each cell's firing
 * threshold (Sec. 2, list of per-step operations); spikes reach their targets through NetCons whose delays are at
 * least one minimum-delay interval, so cells only exchange spikes once per interval (Sec. 2). Mechanism data is
 * held per type in structure-of-arrays form (Sec. 4.2) and pointers between objects are integer indices (Sec. 3.2).
 *
 * Units (Sec. 2, Eq. 1): mV, ms, um, um^2, MOhm, uF/cm^2, S/cm^2, nA, uS.
 *
 * Conventions for every entry point:
 *   - every function returns a status code (CN_OK or an error); no C++ exception crosses this boundary and nothing
 *     aborts; cn_last_error() gives a message for the calling thread's last failure;
 *   - all array arguments are HOST pointers; they are borrowed for the duration of the call only (the library
 *     deep-copies what it keeps); output buffers are owned by the caller;
 *   - a model is not thread-safe; different models may be used from different threads;
 *   - device memory belongs to the model (allocated through cn_options.dev_alloc when given, else hipMalloc) and is
 *     released by cn_model_destroy.
 */
#ifndef CN_H
#define CN_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* status codes */
#define CN_OK 0
#define CN_E_INVALID 1  /* bad argument or model description */
#define CN_E_NOMEM 2    /* host or device allocation failed */
#define CN_E_DEVICE 3   /* a HIP call failed (message kept in cn_last_error) */
#define CN_E_STATE 4    /* call not allowed in the model's current state (e.g. a second dt) */
#define CN_E_CAPACITY 5 /* an event or spike buffer overflowed; results of that run are not valid */
#define CN_E_NUMERIC 6  /* a non-finite membrane potential was found */

/* mechanism types. Density mechanisms (HH, PAS, KM, CAHI) have at most one instance per compartment; point
 * processes (EXPSYN, ICLAMP) may have many. Parameter columns, in order:
 *   CN_MECH_HH:     gnabar, gkbar, gl (S/cm^2), el (mV)      Hodgkin-Huxley Na/K/leak, ena 50 mV, ek -77 mV
 *   CN_MECH_PAS:    g (S/cm^2), e (mV)                        passive leak
 *   CN_MECH_KM:     gbar (S/cm^2)                             slow non-inactivating K (tau near 80-100 ms)
 *   CN_MECH_CAHI:   gbar (S/cm^2)                             high-threshold Ca, eca 120 mV, shell calcium decay
 *   CN_MECH_EXPSYN: tau (ms), e (mV)                          conductance synapse g(t) decaying with tau
 *   CN_MECH_ICLAMP: del (ms), dur (ms), amp (nA)              current clamp on for t in [del, del + dur)
 * The rate equations and integration rule of each type are stated in the repository's design notes. */
enum {
  CN_MECH_HH = 0,
  CN_MECH_PAS = 1,
  CN_MECH_KM = 2,
  CN_MECH_CAHI = 3,
  CN_MECH_EXPSYN = 4,
  CN_MECH_ICLAMP = 5,
  CN_MECH_COUNT = 6
};

enum { CN_PREC_FP64 = 0, CN_PREC_FP32_MECH = 1 };
/* Device node orderings (Sec. 4.4). LEVEL (the default): a workgroup keeps a group of cells on chip for an interval,
 * compartments ordered level by level (constant depth), the tree solve run level-parallel across the group.
 * INTERLEAVED: the paper's one-cell-per-thread ordering: up to 64 cells per wave, compartment k of every cell of the
 * wave side by side in global memory, each lane solving its own cell serially. */
enum { CN_LAYOUT_AUTO = 0, CN_LAYOUT_LEVEL = 1, CN_LAYOUT_INTERLEAVED = 2 };

/* Cell morphology (Sec. 2: each cell is a tree of compartments). Cells own contiguous compartment ranges
 * [cell_offset[c], cell_offset[c+1]); parent[] is cell-local with -1 at the root (local 0) and parent[i] < i. */
typedef struct cn_topology {
  int32_t n_cells;
  int64_t n_comp;
  const int64_t *cell_offset; /* [n_cells + 1], cell_offset[0] = 0, strictly increasing */
  const int32_t *parent;      /* [n_comp] */
  const double *area;         /* [n_comp] membrane area, um^2, > 0 */
  const double *ri;           /* [n_comp] axial resistance to the parent, MOhm, > 0 (ignored at roots) */
  const double *cm;           /* [n_comp] specific capacitance, uF/cm^2, > 0 */
  double v_init;              /* initial membrane potential, mV */
  double celsius;             /* temperature for the HH q10 factor, degC */
} cn_topology;

/* One instance table per mechanism type (Sec. 4.2: instances grouped by type, properties as separate arrays).
 * node[k] is the global compartment of instance k; node == NULL means dense: n == n_comp and instance k sits at
 * compartment k. param[j] is an [n] array or NULL, in which case every instance takes param_scalar[j]. */
typedef struct cn_mech_table {
  int32_t type;
  int64_t n;
  const int64_t *node;
  const double *param[4];
  double param_scalar[4];
} cn_mech_table;

/* Network: NetCons from a cell's threshold detector to an ExpSyn instance (Sec. 3.2 NetCon; Sec. 2 spike
 * delivery), external events ("kicks") and per-synapse background streams (Sec. 3.5, Random123). ExpSyn instances
 * are numbered in the order of the EXPSYN table. */
typedef struct cn_network {
  int64_t n_netcon;
  const int32_t *src_cell;   /* [n_netcon] */
  const int64_t *target_syn; /* [n_netcon] */
  const double *weight;      /* [n_netcon] uS, added to the target's g on delivery */
  const double *delay;       /* [n_netcon] ms; delivered floor(delay/dt + 0.5) >= 1 steps after the spike */
  const double *threshold;   /* [n_cells] mV, or NULL for threshold_scalar */
  double threshold_scalar;
  int64_t n_kick;            /* external events: g[kick_syn] += kick_weight at the start of step kick_step */
  const int64_t *kick_step;
  const int64_t *kick_syn;
  const double *kick_weight;
  double poisson_rate_hz;        /* background rate per synapse (0: none) */
  const double *poisson_weight;  /* [n_syn] uS, or NULL when poisson_rate_hz is 0 */
  uint64_t seed;                 /* key of the counter-based background streams */
  const int64_t *poisson_key;    /* [n_syn] stream id of each synapse (>= 0), or NULL: the instance index */
  /* Gap junctions (Sec. 1 and Table 1: the Traub and Dentate models' electrical coupling; Sec. 3.5: handled with the
   * fixed time step; Sec. 5: the voltages a junction reads, exchanged every step), as half-gap instances: instance k
   * puts the current gap_g[k] (v_node - v_partner) nA at compartment gap_node[k], the partner's potential taken at
   * the start of the step and the compartment's own implicit. A junction between two compartments is two instances.
   * Cells joined by junctions must fit together in one cell group (else CN_E_INVALID; at most 64 cells in the
   * interleaved layout). At most 15 instances per compartment. */
  int64_t n_gap;
  const int64_t *gap_node;    /* [n_gap] compartment */
  const int64_t *gap_partner; /* [n_gap] compartment whose potential drives the current (!= gap_node) */
  const double *gap_g;        /* [n_gap] uS, finite, >= 0 */
} cn_network;

/* Allocation callbacks let a host framework own device memory (e.g. PyTorch's caching allocator). dev_alloc
 * returns a device pointer of at least `bytes` bytes aligned to 256 bytes, or NULL; dev_free releases it. */
typedef void *(*cn_alloc_fn)(size_t bytes, void *ctx);
typedef void (*cn_free_fn)(void *ptr, void *ctx);

typedef struct cn_options {
  int32_t precision;      /* CN_PREC_FP64 or CN_PREC_FP32_MECH (FP32 mechanism states and rates; voltage,
                             matrix assembly and the tree solve stay FP64) */
  int32_t layout;         /* CN_LAYOUT_AUTO (= LEVEL), CN_LAYOUT_LEVEL or CN_LAYOUT_INTERLEAVED */
  void *stream;           /* hipStream_t for all device work, or NULL for the default stream */
  cn_alloc_fn dev_alloc;  /* optional */
  cn_free_fn dev_free;    /* required when dev_alloc is given */
  void *alloc_ctx;
  int32_t event_capacity; /* events per cell group per interval, rounded up to a power of two (0: default 512 per
                             1024 compartments of group capacity, at least 512);
                             each group holds one interval's events on chip, so larger values cost occupancy */
  int32_t max_interval;   /* upper bound on steps per interval (0: default 64) */
  int32_t group_threads;  /* threads per cell group (0: auto) */
  int32_t use_graph;      /* 1: replay one captured hipGraph per interval; 0: direct launches */
  int32_t timing;         /* 1: time the interval kernel with HIP events (see cn_stats) */
  int32_t validate_only;  /* 1: build and check the device layout on the host only, touching no device; the model
                             then answers cn_model_info and nothing else (cn_run returns CN_E_STATE) */
  int32_t fault_inject;   /* tests of the error paths only (0 in normal use): 1 makes the first spike-record drain of
                             cn_run report a device failure after real work was queued; 2 makes the graph capture
                             fail after it began */
  int32_t group_slots;    /* compartments per thread in a cell group (0: auto); with group_threads it sets the group
                             capacity group_threads * group_slots (shapes compiled: 128 x 2/4/8, 256 x 1/2/4,
                             512 x 2/4/8, 1024 x 2), as cn_autotune chooses it */
  int32_t group_fill_pct; /* cells are packed into a group up to this percentage of its capacity (0: 100) */
  int32_t reserved[3];
} cn_options;

typedef struct cn_model cn_model;

/* Build a model (Sec. 3.1 and 3.2: the model is set up once in memory, mechanism instances grouped by type, objects
 * referred to by integer indices; Sec. 4.4: the node order is the library's own): validate, order and pack cells for
 * the device, upload. On CN_OK *out receives a handle owned by
 * the library (free with cn_model_destroy). Errors: CN_E_INVALID (bad topology: parent order, non-positive or
 * non-finite area/ri/cm, index out of range, duplicate density instance, unknown type, NaN parameter, ...),
 * CN_E_NOMEM, CN_E_DEVICE. The time step is not fixed here: see cn_run. */
int cn_model_create(const cn_topology *topo, const cn_mech_table *mechs, int32_t n_mechs, const cn_network *net,
                    const cn_options *opt, cn_model **out);

/* Advance the simulation (Sec. 2: the per-step operations, fixed time step; spikes exchanged once per minimum-delay
 * interval) from its current step to step N = llround(tstop / dt) (tstop is absolute simulated time,
 * t = n * dt exactly; time is an integer step count, never accumulated). The first call fixes dt; a later call
 * with a different dt returns CN_E_STATE, and so does tstop below the current time. Work is queued on the model's
 * stream and the call returns after it completes. Errors: CN_E_CAPACITY (event queue overflow), CN_E_NUMERIC
 * (non-finite voltage, checked at interval ends), CN_E_DEVICE. */
int cn_run(cn_model *m, double tstop, double dt);

/* Spikes recorded so far (Sec. 2: threshold detection at each cell; the spike output the paper's benchmarks compare
 * between runs), sorted by (step, gid): cell index, step index (the spike happened during the step
 * ending at that index) and the linearly interpolated crossing time in ms. With gid == NULL only *n_out is set.
 * Otherwise cap must be >= the count (else CN_E_INVALID); any of step/t_interp may be NULL. */
int cn_spikes(const cn_model *m, int64_t *n_out, int32_t *gid, int64_t *step, double *t_interp, int64_t cap);

/* Membrane potential of every compartment at the current step (Sec. 2, Eq. 1's unknown v), in the caller's
 * compartment order (FP64 in both
 * precision modes). n_comp must equal the model's count (else CN_E_INVALID). */
int cn_voltages(const cn_model *m, double *v_out, int64_t n_comp);

/* A mechanism state at the current step (Sec. 2: channel and synapse states advanced every step; Sec. 4.2: one
 * table per mechanism type) in the caller's instance order, as double. type/which select:
 * HH 0:m 1:h 2:n; KM 0:n; CAHI 0:m 1:cai; EXPSYN 0:g. n must equal the instance count (else CN_E_INVALID). */
int cn_mech_state(const cn_model *m, int32_t type, int32_t which, double *out, int64_t n);

/* The same readout for callers that cannot allocate device memory: code under HIP graph capture, tight serving
 * loops, harnesses that forbid hipMalloc. cn_mech_state stages the gathered states in a device buffer it allocates for
 * the call; this variant stages them in a buffer of CN_NOALLOC_STATE_MAX doubles (32 MiB) that the library holds on
 * every device it runs on until the process ends, and calls no hipMalloc, hipFree or allocating library routine.
 * Arguments, layout and results are those of cn_mech_state. Errors: those of cn_mech_state, and CN_E_CAPACITY when n
 * exceeds CN_NOALLOC_STATE_MAX (read such a model with cn_mech_state). Every call on one device shares that buffer:
 * calls that overlap in time on the same device (from different threads) race and must be serialised by the
 * caller. */
#define CN_NOALLOC_STATE_MAX 4194304
int cn_mech_state_noalloc(const cn_model *m, int32_t type, int32_t which, double *out, int64_t n);

/* Checkpoint-restart (Sec. 3.4: a simulation saved at some step continues later, possibly with other stimuli or
 * random streams). A checkpoint is what the readouts give at a step n: the step, cn_voltages, cn_mech_state of every
 * state (the state update pending on the device is applied by that readout, so the states are those of step n) and
 * the spikes so far (cn_spikes). Events still in flight at n are not stored: each is folded into the spike that sent
 * it and rebuilt from the spike list on restore (every NetCon event of a listed spike due at or after step n is
 * queued again). Arrays are in the caller's order and layout (as the readouts give them); a mechanism the model
 * lacks takes NULL. */
typedef struct cn_checkpoint {
  int64_t step;                     /* the step n the state belongs to (t = n dt) */
  const double *v;                  /* [n_comp] mV */
  const double *hh_m, *hh_h, *hh_n; /* [instances of the HH table] */
  const double *km_n;               /* [instances of the KM table] */
  const double *cahi_m, *cahi_cai;  /* [instances of the CAHI table]; cai in mM */
  const double *syn_g;              /* [ExpSyn instances] uS */
  int64_t n_spikes;                 /* spikes with step <= n (older ones may be left out once their last event was
                                       delivered) */
  const int32_t *spike_gid;
  const int64_t *spike_step;
} cn_checkpoint;

/* Continue a model from a checkpoint (Sec. 3.4). The model must not have run (fresh from cn_model_create, same
 * description as the one checkpointed); the call fixes dt as a first cn_run would, writes potentials, states and
 * conductances, rebuilds the in-flight events, and sets the current step to ck->step. A later cn_run continues
 * exactly as the uninterrupted run would (bitwise, with the same seed). Spikes before the restart are not part of
 * the restored model's spike list. Errors: CN_E_INVALID (missing or non-finite arrays, a spike after ck->step, a
 * gid out of range), CN_E_STATE (the model has run, or dt differs from an earlier call), CN_E_CAPACITY (the rebuilt
 * events overflow the event ring), CN_E_DEVICE. After a failure that reached the device the model refuses further
 * runs (CN_E_STATE). */
int cn_restore(cn_model *m, double dt, const cn_checkpoint *ck);

/* Key of the per-synapse background streams (Sec. 3.5, counter-based Random123-type streams) from the current step
 * on: a restart with other random streams. The draws of a step depend only on (key, stream id, step). */
int cn_set_seed(cn_model *m, uint64_t seed);

/* Autotuner of the cell-group shape (Sec. 4.1: cells are grouped so that groups have equal cost; here the group is
 * what one workgroup advances through a minimum-delay interval). Candidate shapes (threads x compartments per thread,
 * and a packing fill) that hold the largest cell are each built as a model from the same description and options,
 * run for one warm-up interval and then timed over five intervals with HIP events on the model's stream; the
 * interleaved layout (one lane per cell) is timed as one more candidate unless the caller fixed a layout. The
 * candidate with the lowest median interval time wins. Results are cached in the process by a signature of the model
 * (cell-size histogram, synapse and mechanism counts, precision, dt, interval and capacity options): a second call
 * with the same signature returns the cached choice without timing. budget_ms bounds the wall time spent timing
 * (at least the default shape and one other are always timed). The caller then creates its model with
 * opt.layout, opt.group_threads, opt.group_slots and opt.group_fill_pct set from the result. A level-layout shape
 * changes only the grouping, never the arithmetic of a compartment, so such a tuned model's results equal the
 * default model's bitwise; the interleaved layout solves each tree in another order (results within rounding).
 * Arguments as for cn_model_create (borrowed); opt->group_threads/group_slots/group_fill_pct are ignored. Errors:
 * those of cn_model_create and cn_run for the default shape (a failing non-default candidate is skipped). */
#define CN_TUNE_MAX_CANDIDATES 16
typedef struct cn_tune_result {
  int32_t group_threads, group_slots, group_fill_pct; /* the chosen shape */
  int32_t default_threads, default_slots;              /* the shape of the default rule */
  int32_t n_candidates;                                /* shapes timed by this call (0 when taken from the cache) */
  int32_t from_cache;
  int32_t layout;                                      /* the chosen layout (CN_LAYOUT_LEVEL or _INTERLEAVED) */
  double interval_ms;                                  /* median interval time of the chosen shape */
  double default_ms;                                   /* median interval time of the default shape */
  uint64_t signature;
  int32_t cand_threads[CN_TUNE_MAX_CANDIDATES], cand_slots[CN_TUNE_MAX_CANDIDATES],
      cand_fill[CN_TUNE_MAX_CANDIDATES], cand_layout[CN_TUNE_MAX_CANDIDATES];
  double cand_ms[CN_TUNE_MAX_CANDIDATES];
} cn_tune_result;
int cn_autotune(const cn_topology *topo, const cn_mech_table *mechs, int32_t n_mechs, const cn_network *net,
                const cn_options *opt, double dt, double budget_ms, cn_tune_result *out);

/* Model facts for reporting (sizes of the device layout of Sec. 4.2 and 4.4 as built here). */
typedef struct cn_info {
  int64_t n_comp, n_syn, n_netcon, n_groups, step, device_bytes;
  int32_t n_cells, interval_steps, group_threads, group_slots, max_group_nodes, max_levels, ring_slots,
      event_capacity, precision, lds_bytes;
  double dt;
  int32_t layout; /* CN_LAYOUT_LEVEL or CN_LAYOUT_INTERLEAVED; for INTERLEAVED, group_threads is 64 (one lane per
                     cell) and group_slots the largest cell's compartment count */
  int32_t groups_per_cu; /* cell groups the interval kernel keeps co-resident on one compute unit (its registers,
                            LDS and waves allow); 0 before the first cn_run fixes dt */
} cn_info;
int cn_model_info(const cn_model *m, cn_info *out);

/* Measurement support (the per-step cost of Sec. 2's operations is what the paper's benchmarks time). With
 * cn_options.timing set: total milliseconds and launch count of the interval kernel over all cn_run calls,
 * from HIP events recorded on the model's stream around each launch. */
int cn_stats(const cn_model *m, double *kernel_ms, int64_t *kernel_launches);

/* Where a step's time goes (Sec. 2 lists the operations of a step; Sec. 4.4 finds the tree solve's ordering decisive
 * on GPUs). In a library built with CN_PHASE_CLOCKS (the profiling build, libcn_phase.so) the level layout's interval
 * kernel sums the shader clock of its first wave per phase over all groups and runs: out[0] a chunk's prologue and
 * epilogue (rows on chip, event sort, write-back), then per step out[1] events, threshold detection and synapse
 * staging, out[2] mechanisms and matrix assembly, out[3] the elimination, out[4] the root solves, out[5] the
 * substitution. out holds n >= CN_N_PHASES entries (host memory, caller-owned). CN_E_STATE from an ordinary build, a
 * validate-only model or the interleaved layout; CN_E_INVALID on NULL or a short buffer. */
#define CN_N_PHASES 6
int cn_phase_clocks(const cn_model *m, uint64_t *out, int32_t n);

/* Free everything the model owns (the counterpart of the memory setup of Sec. 3.1). NULL is a no-op. */
void cn_model_destroy(cn_model *m);

/* Message describing the calling thread's last non-OK status (error reporting of this boundary). */
const char *cn_last_error(void);

#ifdef __cplusplus
}
#endif
#endif
