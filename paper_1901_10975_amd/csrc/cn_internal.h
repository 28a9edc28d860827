// Internal layout shared by the host driver (cn_host.cpp) and the kernels (cn_kernels.hip) of the cn library.
//
// Device order. Cells are packed into cell groups; one workgroup advances one group through a whole minimum-delay
// interval (cells do not interact inside an interval, Sec. 2). Inside a group the compartments are stored level by
// level (all roots, then all depth-1 nodes, ...), children of one parent contiguous and in ascending cell-local
// index: the constant-depth ordering of Sec. 4.4, which here lets each level of the tree elimination run in
// parallel. Node q of a group is handled by thread q % T in register slot q / T.
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

struct GroupDesc {
  int64_t node_base;  // first node of the group in the node arrays
  int64_t syn_base;   // first synapse of the group
  int32_t n_nodes, n_levels, lvl_base, n_cells;
  int32_t cell_base, n_syn, kick_base, n_kick;
  int32_t spk_base, icl_base, pad0, pad1;
};

struct KParams {
  const GroupDesc *groups;
  const int32_t *lvl_start;  // per group n_levels + 1 group-local starts
  int32_t n_groups;
  int32_t M;     // steps per interval
  int32_t ring;  // interval slots in the event ring
  int32_t ev_cap;
  int32_t smax;  // LDS synapse slots per group
  int32_t lds_ev_off, lds_seg_off, lds_misc_off, lds_syn_off;  // byte offsets into dynamic LDS
  int32_t has_bg;
  // node arrays (device order)
  const double *nd_a, *nd_b, *nd_k, *nd_sa;
  const int32_t *nd_par;
  const uint32_t *nd_ch;   // first child (low 16 bits) | child count (high 16 bits), group-local
  const uint8_t *nd_mf;    // MF_* flags
  const int2 *nd_syn;      // group-local synapse range (start, count)
  const int2 *nd_icl;      // group-local IClamp range (start, count)
  double *v;
  void *st[6];             // hh m, h, n; km n; cahi m, cai (double or float, one per node)
  // per-node parameters, NULL when the column is uniform (then the scalar is used)
  const double *hh_gna, *hh_gk, *hh_gl, *hh_el, *pas_g, *pas_e, *km_g, *ca_g;
  double hh_gna_s, hh_gk_s, hh_gl_s, hh_el_s, pas_g_s, pas_e_s, km_g_s, ca_g_s;
  // synapses (device order)
  void *syn_g;             // double or float
  const double *syn_e;     // NULL: syn_e_s
  double syn_e_s;
  const void *syn_f;       // decay factor exp(-dt/tau), double or float; NULL: syn_f_s
  double syn_f_s;
  const int64_t *syn_id;   // caller's instance index (background stream key)
  const void *syn_wbg;     // background weight, double or float
  // IClamp (device order)
  const double *icl_cur;   // 100 amp / area, mA/cm^2
  const int64_t *icl_on, *icl_off;
  // cells (device order)
  const int32_t *cell_gid;
  const double *cell_theta;
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
  int32_t *gsp_pack;       // per group scratch: cell | (step in interval << 16)
  double *gsp_frac;
  int32_t *rec_cnt;
  int32_t *rec_gid;
  int64_t *rec_step;
  double *rec_t;
  int32_t rec_cap;
  int32_t *flags;          // [0] event overflow, [1] spike record overflow, [2] non-finite voltage
  int64_t *ctl;            // [0] first step of the next chunk, [1] target step
  // constants
  double dt, q10dt;
  double ca_fm, ca_fr, ca_k;  // cahi: 1-exp(-dt/tau_m), 1-exp(-dt/tau_r), 1e4 tau_r / (2 F depth)
  uint64_t seed;
  uint64_t bg_thresh;
};

enum { FLAG_EV_OVERFLOW = 0, FLAG_REC_OVERFLOW = 1, FLAG_NONFINITE = 2 };

}  // namespace cn
