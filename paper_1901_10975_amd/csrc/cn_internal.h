// Internal layout shared by the host driver (cn_host.cpp) and the kernels (cn_kernels.hip) of the cn library.
//
// Device order. Cells are packed into cell groups; one workgroup advances one group through a whole minimum-delay
// interval (cells do not interact inside an interval, Sec. 2). Inside a group the compartments are stored level by
// level (all roots, then all depth-1 nodes, ...), children of one parent contiguous and in ascending cell-local
// index: the constant-depth ordering of Sec. 4.4, which here lets each level of the tree elimination run in
// parallel, one thread per node of the level. Node q of a group sits in register slot q / T of thread q % T for the
// per-compartment work (mechanisms and assembly).
#pragma once
#include <stdint.h>

namespace cn {

constexpr int MF_HH = 1, MF_PAS = 2, MF_KM = 4, MF_CAHI = 8;

// event key: [63:54] step inside the interval, [53:32] group-local synapse, [31] kind (0 kick, 1 NetCon),
// [30:0] kick or NetCon id. Sorting the keys orders a step's events by synapse, then kicks before NetCon events,
// each by ascending id: the delivery order of the oracle.
constexpr int EV_STEP_SHIFT = 54;
constexpr int EV_SYN_SHIFT = 32;
constexpr uint32_t EV_SYN_MASK = 0x3FFFFFu;
constexpr uint32_t EV_KIND_NETCON = 0x80000000u;
constexpr int MAX_INTERVAL = 1023;
constexpr int64_t MAX_GROUP_SYN = (int64_t)EV_SYN_MASK + 1;
constexpr int MAX_NODE_SYN = 0xFFFF;  // synapses on one compartment
constexpr int MAX_NODE_ICL = 0xFF;    // IClamps on one compartment
constexpr int MAX_NODE_GAP = 0xF;     // half-gap junctions on one compartment

// per-node constants of the tree matrix (S/cm^2): a (row parent, column node), b (row node, column parent),
// k = 1e-3 cm/dt - b (capacitance and the node's own axial term on the diagonal), sa = 100/area (point processes)
struct NodeRec {
  double a, b, k, sa;
};
// per-node indices: parent (group-local, -1 at roots), children (first | count << 16, group-local), first synapse
// (group-local) and pk = synapse count | IClamp count << 16 | mechanism flags << 24 | half-gap count << 28
struct NodeIdx {
  int32_t par;
  uint32_t ch;
  int32_t syn0;
  uint32_t pk;
};

// synapse record (device order): background stream id, reversal potential, 100/area of its compartment, background
// weight, decay factor, and its compartment (group-local node)
template <typename S>
struct SynRec {
  uint64_t key;
  double e;
  double sa;
  S wbg;
  S f;
  int32_t q;
  int32_t pad;
};
// channel states of one compartment (hh m, h, n; km n; cahi m, cai), double or float
template <typename S>
struct StRec {
  S m, h, n, kn, cm, cai;
};
// half-gap record (device order): the partner compartment (group-local node) and 100 g / area (S/cm^2)
struct GapRec {
  int32_t q;
  int32_t pad;
  double gs;
};
// IClamp record (device order): on for steps on <= n < off, current density 100 amp / area (mA/cm^2)
struct IclRec {
  int64_t on, off;
  double cur;
  double pad;
};

// constants the interval kernel keeps in LDS (indices into a small double table)
enum { C_PRM = 0, C_Q10DT = 8, C_DT, C_CA_FM, C_CA_FR, C_CA_K, C_SEED, N_CST };

struct GroupDesc {
  int64_t node_base;  // first node of the group in the node arrays
  int64_t syn_base;   // first synapse of the group
  int32_t n_nodes, n_levels, lvl_base, n_cells;
  int32_t cell_base, n_syn, kick_base, n_kick;
  int32_t spk_base, icl_base, gap_base, pad1;
};

// non-uniform density-mechanism parameters, columns of the per-node parameter table
enum { P_HH_GNA = 0, P_HH_GK, P_HH_GL, P_HH_EL, P_PAS_G, P_PAS_E, P_KM_G, P_CA_G, N_PRM };

// phases of the interval kernel timed by the profiling build (CN_PHASE_CLOCKS): a chunk's prologue and epilogue,
// then per step the events, detection and synapse staging; the mechanisms and assembly; the elimination; the root
// solves; the substitution
enum { PH_CHUNK = 0, PH_EVENTS, PH_MECH, PH_ELIM, PH_ROOT, PH_SUBST, PH_COUNT };

struct KParams {
  const GroupDesc *groups;
  const int32_t *lvl_start;  // per group n_levels + 1 group-local starts
  int32_t n_groups;
  int32_t M;     // steps per interval
  int32_t ring;  // interval slots in the event ring
  int32_t ev_cap;
  int32_t nmax;  // nodes per group (LDS rows)
  int32_t has_bg;
  uint32_t mf_uni;   // the density-mechanism flags every compartment carries (kernels for uniform models)
  int32_t has_icl;   // any IClamp in the model
  int32_t uni;       // the uniform kernels run: one mechanism set everywhere, every parameter uniform, no gap junction
  int32_t lds_ev_off, lds_seg_off, lds_lvl_off, lds_bg_off, lds_cell_off, lds_misc_off, lds_cst_off, lds_exp_off;
  const double *exp_tab;   // 2^(j/64), j = 0..63
  // node tables (device order)
  const NodeRec *nrec;
  const NodeIdx *nidx;
  const int32_t *nd_icl0;  // group-local first IClamp of each node
  const int32_t *nd_gap0;  // group-local first half-gap of each node
  const GapRec *gap;       // half-gaps (device order)
  double *v;               // membrane potential between chunks
  void *st;                // StRec<double> or StRec<float> per node
  int64_t n_nodes_total;
  const double *prm;       // N_PRM columns of n_nodes_total values, or NULL when every column is uniform
  double prm_s[N_PRM];     // the uniform values
  // synapses (device order)
  void *syn_g;             // double or float
  const void *syn;         // SynRec<double> or SynRec<float>
  // IClamp (device order)
  const IclRec *icl;
  // cells (device order)
  const int32_t *cell_gid;
  const double *cell_theta;
  const int32_t *cell_soma;  // group-local position of each cell's soma (its threshold compartment)
  // network
  const void *nc_w;        // by NetCon id, double or float
  const int32_t *nc_tgt_group, *nc_tgt_lsyn, *nc_D;
  const int64_t *out_off;  // NetCons by source cell (caller's cell ids)
  const int32_t *out_nc;
  const int64_t *kick_step;  // kicks sorted by (group, step, id)
  const int32_t *kick_lsyn, *kick_id;
  const void *kick_w;        // by kick id, double or float
  // event ring
  int32_t *ev_cnt;         // [ring * n_groups]
  uint64_t *ev_key;        // [ring * n_groups * ev_cap]
  // spikes
  int32_t *gsp_cnt;        // per group: spikes of the last chunk
  int32_t *gsp_pack;       // per group scratch: cell | (step in interval << 16)
  double *gsp_frac;
  int32_t *rec_cnt;
  int32_t *rec_gid;
  int64_t *rec_step;
  double *rec_t;
  int32_t rec_cap;
  int32_t *flags;          // [0] event overflow, [1] spike record overflow, [2] non-finite voltage
  int64_t *ctl;            // [0] first step of the next chunk, [1] target step, [2] the step whose channel states
                           // carry no pending update (0, or the step of a restart), [3] key of the background streams
  // interleaved layout (one lane per cell): per-node work arrays of the tree solve: the elimination's accumulators of
  // the diagonal and right-hand side (zero between steps; w and u once a compartment is eliminated), the solution x
  double *lw_d, *lw_r, *lw_dv;
  // constants
  double dt, q10dt;
  double ca_fm, ca_fr, ca_k;  // cahi: 1-exp(-dt/tau_m), 1-exp(-dt/tau_r), 1e4 tau_r / (2 F depth)
  uint64_t bg_thresh;
  uint64_t *phase_clk;  // [PH_COUNT] shader-clock sums of the interval kernel (profiling builds only), else NULL
};

enum { FLAG_EV_OVERFLOW = 0, FLAG_REC_OVERFLOW = 1, FLAG_NONFINITE = 2 };

}  // namespace cn
