// Host side of the cn library: the C-ABI of include/cn.h, validation, the device layout (cell groups, level
// order, structure-of-arrays tables) and the interval driver.
//
// Model setup follows the paper's memory-setup phase (Sec. 3.1, Sec. 3.2, Sec. 4.2): mechanism instances grouped
// by type in structure-of-arrays columns, integer indices instead of pointers, and a node permutation for the
// device (Sec. 4.4). The driver runs the fixed-step loop in chunks of at most one minimum-delay interval
// (Sec. 2: spikes are exchanged once per minimum delay), one kernel launch per chunk, optionally replayed from a
// captured hipGraph.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <array>
#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <map>
#include <mutex>
#include <numeric>
#include <string>
#include <vector>

#include "cn.h"
#include "cn_internal.h"

namespace cn {
hipError_t launch_interval(const KParams &p, bool fp32, int threads, int slots, int lds_bytes, hipStream_t st);
hipError_t set_interval_lds(bool fp32, int threads, int slots, bool uni, int lds_bytes);
hipError_t launch_lpc(const KParams &p, bool fp32, int lds_bytes, hipStream_t st);
hipError_t set_lpc_lds(bool fp32, bool uni, int lds_bytes);
hipError_t interval_groups_per_cu(bool fp32, int threads, int slots, bool uni, int lds_bytes, int *n);
hipError_t lpc_groups_per_cu(bool fp32, bool uni, int lds_bytes, int *n);
int interval_row_bytes(int nmax);
hipError_t launch_advance(int64_t *ctl, int32_t M, hipStream_t st);
hipError_t launch_fanout(const KParams &p, hipStream_t st);
hipError_t launch_set_ctl(int64_t *ctl, int64_t n_begin, int64_t n_target, int64_t n_fresh, uint64_t seed,
                          hipStream_t st);
hipError_t launch_insert_events(int32_t *ev_cnt, uint64_t *ev_key, int32_t cap, int64_t n, const int64_t *bucket,
                                const uint64_t *key, int32_t *flags, hipStream_t st);
hipError_t launch_fill_i32(int32_t *ptr, int64_t n, int32_t v, hipStream_t st);
hipError_t launch_gather_state(const KParams &p, bool fp32, const int32_t *inst_dev, int64_t n, int64_t step,
                               int64_t n_fresh, int type, int which, double *out, hipStream_t st);
}  // namespace cn

using namespace cn;

namespace {

thread_local std::string g_err;

int fail(int code, const std::string &msg) {
  g_err = msg;
  return code;
}

struct Err {
  int code;
  std::string msg;
};

#define HIPCHK(expr)                                                                                   \
  do {                                                                                                 \
    hipError_t e_ = (expr);                                                                            \
    if (e_ != hipSuccess)                                                                              \
      throw Err{CN_E_DEVICE, std::string(#expr) + ": " + hipGetErrorString(e_)};                      \
  } while (0)

const int N_PARAMS[CN_MECH_COUNT] = {4, 2, 1, 1, 2, 3};
const char *MECH_NAME[CN_MECH_COUNT] = {"hh", "pas", "km", "cahi", "expsyn", "iclamp"};

// one parameter column of a mechanism table, expanded
struct Col {
  std::vector<double> v;
  bool uniform = true;
  double s = 0.0;
};

struct Table {
  bool present = false;
  int64_t n = 0;
  std::vector<int64_t> node;  // per instance
  Col p[4];
};

// Hodgkin-Huxley steady states at v (initial states), same kinetics as the device code, in double
void hh_inf(double v, double &m, double &h, double &n) {
  auto vtrap = [](double x, double y) { return std::fabs(x / y) < 1e-6 ? y * (1.0 - x / y / 2.0) : x / (std::exp(x / y) - 1.0); };
  const double am = 0.1 * vtrap(-(v + 40.0), 10.0), bm = 4.0 * std::exp(-(v + 65.0) / 18.0);
  const double ah = 0.07 * std::exp(-(v + 65.0) / 20.0), bh = 1.0 / (std::exp(-(v + 35.0) / 10.0) + 1.0);
  const double an = 0.01 * vtrap(-(v + 55.0), 10.0), bn = 0.125 * std::exp(-(v + 65.0) / 80.0);
  m = am / (am + bm);
  h = ah / (ah + bh);
  n = an / (an + bn);
}
double km_inf(double v) { return 1.0 / (1.0 + std::exp(-(v + 35.0) / 10.0)); }
double cahi_inf(double v) { return 1.0 / (1.0 + std::exp(-(v + 20.0) / 9.0)); }

}  // namespace

struct cn_model {
  // ---- caller's description (kept for dt-dependent setup and readouts)
  int32_t n_cells = 0;
  int64_t n_comp = 0;
  std::vector<int64_t> cell_off;
  std::vector<int32_t> parent;
  std::vector<double> area, ri, cm;
  double v_init = -65.0, celsius = 6.3;
  Table mech[CN_MECH_COUNT];
  int64_t n_syn = 0, n_nc = 0, n_kick = 0;
  std::vector<int32_t> nc_src;
  std::vector<int64_t> nc_syn;
  std::vector<double> nc_w, nc_delay, theta;
  std::vector<int64_t> kick_step, kick_syn;
  std::vector<double> kick_w;
  double rate = 0.0;
  std::vector<double> pw;
  std::vector<int64_t> pkey;
  uint64_t seed = 0;
  int64_t n_gap = 0;
  std::vector<int64_t> gap_node, gap_partner;
  std::vector<double> gap_g;
  std::vector<int32_t> cell_cluster;  // cells joined by gap junctions share a cluster id (its smallest cell)
  cn_options opt{};
  bool fp32 = false;

  // ---- layout
  int threads = 256, slots = 4, nmax = 1024;
  bool lpc = false;     // interleaved layout, one lane per cell (else the level layout)
  int64_t n_dev = 0;    // device node slots (the compartments, plus padding in the interleaved layout)
  int64_t n_groups = 0;
  std::vector<GroupDesc> groups;
  std::vector<int32_t> lvl_start;
  std::vector<int64_t> dev_of_node, node_of_dev;  // caller compartment <-> device node
  std::vector<int64_t> dev_of_syn, syn_of_dev;    // caller ExpSyn <-> device synapse
  std::vector<int64_t> icl_of_dev;                // device IClamp -> caller instance
  std::vector<int32_t> cell_of_devcell;           // device cell slot -> caller cell
  std::vector<int64_t> tree_par;                  // parent of each caller compartment in the rooted tree (-1: root)
  std::vector<int64_t> cell_root;                 // each caller cell's root compartment
  // per device node, kept for the dt-dependent node records
  std::vector<double> host_a, host_b, host_sa;
  std::vector<uint8_t> host_mf;
  std::vector<int32_t> host_par;
  std::vector<uint32_t> host_ch;
  std::vector<uint64_t> host_syn_key;
  std::vector<double> host_syn_e, host_syn_wbg;
  std::vector<int32_t> host_syn_q;
  // network on the host, for rebuilding in-flight events at a restart: NetCons by source cell, target group and
  // group-local synapse, delay in steps
  std::vector<int64_t> host_out_off;
  std::vector<int32_t> host_out_nc, host_tgt_g, host_tgt_l, host_D;
  int32_t max_levels = 0, max_group_syn = 0, max_group_nodes = 0, max_group_cells = 0;

  // ---- device
  hipStream_t stream = nullptr;
  bool own_stream = false;
  std::vector<void *> allocs;
  std::vector<size_t> alloc_bytes;
  int64_t device_bytes = 0;
  KParams kp{};
  int lds_bytes = 0;
  int groups_per_cu = 0;  // co-resident groups on one CU (registers, LDS, waves), from the occupancy query
  int32_t spk_total = 0;
  int32_t drain_every = 1;
  hipGraph_t graph = nullptr;
  hipGraphExec_t gexec = nullptr;

  // ---- run state
  bool dt_fixed = false, broken = false;
  double dt = 0.0;
  int64_t step = 0;
  int64_t fresh_step = 0;  // channel states on the device carry no pending update at this step (0, or a restart)
  int device = 0;          // the HIP device of the model's stream
  // per mechanism type, the device node (density mechanisms) or device synapse (ExpSyn) of each caller instance
  const int32_t *inst_dev[CN_MECH_COUNT] = {};
  std::vector<int32_t> sp_gid;
  std::vector<int64_t> sp_step;
  std::vector<double> sp_t;
  std::vector<hipEvent_t> ev_pool;
  double kernel_ms = 0.0;
  int64_t kernel_launches = 0;

  bool dry = false;  // validate_only: no device work

  void *dalloc(size_t bytes) {
    if (bytes == 0) bytes = 256;
    device_bytes += (int64_t)bytes;
    if (dry) return nullptr;
    void *p = nullptr;
    if (opt.dev_alloc) {
      p = opt.dev_alloc(bytes, opt.alloc_ctx);
      if (!p) throw Err{CN_E_NOMEM, "device allocation of " + std::to_string(bytes) + " bytes failed"};
    } else {
      hipError_t e = hipMalloc(&p, bytes);
      if (e != hipSuccess) throw Err{CN_E_NOMEM, std::string("hipMalloc: ") + hipGetErrorString(e)};
    }
    allocs.push_back(p);
    alloc_bytes.push_back(bytes);
    return p;
  }
  // release one allocation of dalloc before the model ends (temporary buffers)
  void dfree(void *p) {
    for (size_t k = 0; k < allocs.size(); ++k) {
      if (allocs[k] != p) continue;
      device_bytes -= (int64_t)alloc_bytes[k];
      allocs.erase(allocs.begin() + (long)k);
      alloc_bytes.erase(alloc_bytes.begin() + (long)k);
      if (opt.dev_alloc) opt.dev_free(p, opt.alloc_ctx);
      else (void)hipFree(p);
      return;
    }
  }
  template <typename T>
  T *upload(const std::vector<T> &h) {
    T *d = static_cast<T *>(dalloc(h.size() * sizeof(T)));
    if (!h.empty() && !dry) HIPCHK(hipMemcpyAsync(d, h.data(), h.size() * sizeof(T), hipMemcpyHostToDevice, stream));
    return d;
  }
  // upload as double or as float (FP32-mechanism path)
  void *upload_s(const std::vector<double> &h) {
    if (!fp32) return upload(h);
    std::vector<float> f(h.begin(), h.end());
    return upload(f);
  }
  ~cn_model() {
    if (gexec) (void)hipGraphExecDestroy(gexec);
    if (graph) (void)hipGraphDestroy(graph);
    for (hipEvent_t e : ev_pool) (void)hipEventDestroy(e);
    if (stream && !dry) (void)hipStreamSynchronize(stream);
    for (void *p : allocs) {
      if (opt.dev_alloc) opt.dev_free(p, opt.alloc_ctx);
      else (void)hipFree(p);
    }
    if (own_stream && stream) (void)hipStreamDestroy(stream);
  }
};

namespace {

bool finite_all(const double *p, int64_t n) {
  for (int64_t i = 0; i < n; ++i)
    if (!std::isfinite(p[i])) return false;
  return true;
}

void read_tables(cn_model *m, const cn_mech_table *mechs, int32_t n_mechs) {
  if (n_mechs < 0 || (n_mechs > 0 && !mechs)) throw Err{CN_E_INVALID, "bad mechanism table list"};
  for (int32_t k = 0; k < n_mechs; ++k) {
    const cn_mech_table &mt = mechs[k];
    if (mt.type < 0 || mt.type >= CN_MECH_COUNT) throw Err{CN_E_INVALID, "unknown mechanism type " + std::to_string(mt.type)};
    Table &t = m->mech[mt.type];
    const char *nm = MECH_NAME[mt.type];
    if (t.present) throw Err{CN_E_INVALID, std::string("two tables of type ") + nm};
    t.present = true;
    if (mt.n < 0) throw Err{CN_E_INVALID, std::string(nm) + ": negative count"};
    if (!mt.node && mt.n != m->n_comp)
      throw Err{CN_E_INVALID, std::string(nm) + ": dense table needs n == n_comp"};
    t.n = mt.n;
    t.node.resize(mt.n);
    for (int64_t i = 0; i < mt.n; ++i) {
      t.node[i] = mt.node ? mt.node[i] : i;
      if (t.node[i] < 0 || t.node[i] >= m->n_comp)
        throw Err{CN_E_INVALID, std::string(nm) + ": instance " + std::to_string(i) + " node out of range"};
    }
    if (mt.type <= CN_MECH_CAHI) {
      std::vector<char> seen(m->n_comp, 0);
      for (int64_t i = 0; i < mt.n; ++i) {
        if (seen[t.node[i]]) throw Err{CN_E_INVALID, std::string(nm) + ": two instances at one compartment"};
        seen[t.node[i]] = 1;
      }
    }
    for (int j = 0; j < N_PARAMS[mt.type]; ++j) {
      Col &c = t.p[j];
      if (mt.param[j]) {
        c.v.assign(mt.param[j], mt.param[j] + mt.n);
        if (!finite_all(c.v.data(), mt.n)) throw Err{CN_E_INVALID, std::string(nm) + ": non-finite parameter"};
        c.uniform = std::all_of(c.v.begin(), c.v.end(), [&](double x) { return x == c.v[0]; });
        c.s = mt.n ? c.v[0] : 0.0;
      } else {
        if (!std::isfinite(mt.param_scalar[j])) throw Err{CN_E_INVALID, std::string(nm) + ": non-finite parameter"};
        c.v.assign(mt.n, mt.param_scalar[j]);
        c.uniform = true;
        c.s = mt.param_scalar[j];
      }
    }
  }
  const Table &syn = m->mech[CN_MECH_EXPSYN];
  for (int64_t i = 0; i < syn.n; ++i)
    if (!(syn.p[0].v[i] > 0.0)) throw Err{CN_E_INVALID, "expsyn: tau must be positive"};
  m->n_syn = syn.n;
}

void read_network(cn_model *m, const cn_network *net) {
  m->theta.assign(m->n_cells, 0.0);
  if (!net) return;
  if (net->n_netcon < 0 || net->n_netcon >= (int64_t)0x7FFFFFFF) throw Err{CN_E_INVALID, "bad NetCon count"};
  if (net->n_kick < 0 || net->n_kick >= (int64_t)0x7FFFFFFF) throw Err{CN_E_INVALID, "bad kick count"};
  m->n_nc = net->n_netcon;
  if (m->n_nc > 0 && (!net->src_cell || !net->target_syn || !net->weight || !net->delay))
    throw Err{CN_E_INVALID, "NetCon arrays missing"};
  m->nc_src.assign(net->src_cell, net->src_cell + m->n_nc);
  m->nc_syn.assign(net->target_syn, net->target_syn + m->n_nc);
  m->nc_w.assign(net->weight, net->weight + m->n_nc);
  m->nc_delay.assign(net->delay, net->delay + m->n_nc);
  for (int64_t k = 0; k < m->n_nc; ++k) {
    if (m->nc_src[k] < 0 || m->nc_src[k] >= m->n_cells) throw Err{CN_E_INVALID, "NetCon source out of range"};
    if (m->nc_syn[k] < 0 || m->nc_syn[k] >= m->n_syn) throw Err{CN_E_INVALID, "NetCon target out of range"};
    if (!std::isfinite(m->nc_w[k]) || !std::isfinite(m->nc_delay[k]) || !(m->nc_delay[k] > 0.0))
      throw Err{CN_E_INVALID, "NetCon weight/delay must be finite, delay > 0"};
  }
  if (net->threshold) m->theta.assign(net->threshold, net->threshold + m->n_cells);
  else m->theta.assign(m->n_cells, net->threshold_scalar);
  if (!finite_all(m->theta.data(), m->n_cells)) throw Err{CN_E_INVALID, "non-finite threshold"};
  m->n_kick = net->n_kick;
  if (m->n_kick > 0 && (!net->kick_step || !net->kick_syn || !net->kick_weight))
    throw Err{CN_E_INVALID, "kick arrays missing"};
  m->kick_step.assign(net->kick_step, net->kick_step + m->n_kick);
  m->kick_syn.assign(net->kick_syn, net->kick_syn + m->n_kick);
  m->kick_w.assign(net->kick_weight, net->kick_weight + m->n_kick);
  for (int64_t k = 0; k < m->n_kick; ++k)
    if (m->kick_step[k] < 0 || m->kick_syn[k] < 0 || m->kick_syn[k] >= m->n_syn || !std::isfinite(m->kick_w[k]))
      throw Err{CN_E_INVALID, "bad kick"};
  m->rate = net->poisson_rate_hz;
  if (!std::isfinite(m->rate) || m->rate < 0.0) throw Err{CN_E_INVALID, "bad background rate"};
  if (m->rate > 0.0) {
    if (!net->poisson_weight) throw Err{CN_E_INVALID, "background weights missing"};
    m->pw.assign(net->poisson_weight, net->poisson_weight + m->n_syn);
    if (!finite_all(m->pw.data(), m->n_syn)) throw Err{CN_E_INVALID, "non-finite background weight"};
  }
  m->pkey.resize(m->n_syn);
  for (int64_t k = 0; k < m->n_syn; ++k) {
    m->pkey[k] = net->poisson_key ? net->poisson_key[k] : k;
    if (m->pkey[k] < 0) throw Err{CN_E_INVALID, "negative background stream id"};
  }
  m->seed = net->seed;
  if (net->n_gap < 0 || net->n_gap >= (int64_t)INT32_MAX) throw Err{CN_E_INVALID, "bad gap-junction count"};
  m->n_gap = net->n_gap;
  if (m->n_gap > 0 && (!net->gap_node || !net->gap_partner || !net->gap_g))
    throw Err{CN_E_INVALID, "gap-junction arrays missing"};
  m->gap_node.assign(net->gap_node, net->gap_node + m->n_gap);
  m->gap_partner.assign(net->gap_partner, net->gap_partner + m->n_gap);
  m->gap_g.assign(net->gap_g, net->gap_g + m->n_gap);
  for (int64_t k = 0; k < m->n_gap; ++k) {
    if (m->gap_node[k] < 0 || m->gap_node[k] >= m->n_comp || m->gap_partner[k] < 0 ||
        m->gap_partner[k] >= m->n_comp || m->gap_partner[k] == m->gap_node[k])
      throw Err{CN_E_INVALID, "gap junction " + std::to_string(k) + ": compartment out of range or its own partner"};
    if (!std::isfinite(m->gap_g[k]) || m->gap_g[k] < 0.0)
      throw Err{CN_E_INVALID, "gap junction " + std::to_string(k) + ": conductance must be finite and >= 0"};
  }
}

// Cells joined by gap junctions, found by union-find over cells: `cluster[c]` is the smallest cell of c's set.
// Returns the compartments of the largest set (one cell's when there are no junctions). Entries out of range are
// skipped here: they are refused where the network is read.
int64_t join_cells(const int64_t *cell_off, int32_t n_cells, int64_t n_comp, int64_t n_gap, const int64_t *gn,
                   const int64_t *gp, std::vector<int32_t> &cluster) {
  cluster.resize(n_cells);
  std::iota(cluster.begin(), cluster.end(), 0);
  if (n_gap > 0 && gn && gp) {
    std::vector<int32_t> cell_of(n_comp);
    for (int32_t c = 0; c < n_cells; ++c)
      for (int64_t i = cell_off[c]; i < cell_off[c + 1]; ++i) cell_of[i] = c;
    auto find = [&](int32_t x) {
      while (cluster[x] != x) x = cluster[x] = cluster[cluster[x]];
      return x;
    };
    for (int64_t k = 0; k < n_gap; ++k) {
      if (gn[k] < 0 || gn[k] >= n_comp || gp[k] < 0 || gp[k] >= n_comp) continue;
      const int32_t a = find(cell_of[gn[k]]), b = find(cell_of[gp[k]]);
      if (a != b) cluster[std::max(a, b)] = std::min(a, b);
    }
    for (int32_t c = 0; c < n_cells; ++c) cluster[c] = find(c);
  }
  std::vector<int64_t> size(n_cells, 0);
  int64_t big = 0;
  for (int32_t c = 0; c < n_cells; ++c) big = std::max(big, size[cluster[c]] += cell_off[c + 1] - cell_off[c]);
  return big;
}

void gap_clusters(cn_model *m) {
  join_cells(m->cell_off.data(), m->n_cells, m->n_comp, m->n_gap, m->gap_node.data(), m->gap_partner.data(),
             m->cell_cluster);
}

// ---- device layout: cell groups (bin packing), level order, tables

// Group shapes compiled: T threads x K register slots per thread, capacity T K compartments.
bool shape_compiled(int T, int K) {
  if (T == 128) return K == 2 || K == 4 || K == 8;
  if (T == 256) return K == 1 || K == 2 || K == 4;
  if (T == 512) return K == 2 || K == 4 || K == 8;
  if (T == 1024) return K == 2;
  return false;
}

// The default rule for the entries of (T, K) left at 0. Large models take groups of 1024 or more compartments on
// 512 threads: two slots per thread keep the register budget at four waves per SIMD, which hides the latency of the
// level sweeps; small models take smaller groups so that there are enough of them to fill the device. K is the
// smallest compiled slot count whose group holds the largest cell. In FP64, cells (or sets of cells joined by gap
// junctions) of 1,025 to 2,048 compartments take 1024 x 2 groups: one group per CU either way (its LDS), but with
// twice the waves of 512 x 4 (measured 8 % faster on the 200,000-cell cortex recipe; with FP32 mechanisms 2 % slower).
void default_shape(int64_t n_comp, int32_t max_cell, bool fp32, int &T, int &K) {
  const bool large = n_comp >= (int64_t)1024 * 1024;
  if (T == 0 && K == 0 && !fp32 && max_cell > 1024 && max_cell <= 2048) {
    T = 1024;
    K = 2;
    return;
  }
  if (T == 0) T = (large || max_cell > 1024) ? 512 : 256;
  if (K == 0) {
    const int kmin = T == 256 ? 1 : 2, kmax = T == 256 ? 4 : 8;
    K = kmin;
    while (K < kmax && T * K < max_cell) K *= 2;
    if (T == 256 && K < 4 && large) K = 4;  // large models on 256 threads: fuller groups
  }
}

void build_layout(cn_model *m) {
  const int64_t N = m->n_comp;
  std::vector<int32_t> depth(N, 0), cell_levels(m->n_cells, 0), cell_size(m->n_cells);
  std::vector<int64_t> syn_per_cell(m->n_cells, 0);
  std::vector<int32_t> cell_of(N);
  int32_t max_cell = 0;
  for (int32_t c = 0; c < m->n_cells; ++c) {
    const int64_t i0 = m->cell_off[c], n = m->cell_off[c + 1] - i0;
    cell_size[c] = (int32_t)n;
    max_cell = std::max<int32_t>(max_cell, (int32_t)n);
    for (int64_t k = 0; k < n; ++k) cell_of[i0 + k] = c;
  }
  // Each cell's tree is rooted at a centre, a compartment of least eccentricity (the first in caller order on
  // ties): the tree matrix is the same linear system whichever compartment the elimination ends at (an edge seen
  // from its other end swaps its a and b), and a centre gives the fewest levels to sweep. The soma (compartment 0)
  // stays the cell's threshold compartment.
  m->tree_par.assign(N, -1);
  m->cell_root.assign(m->n_cells, 0);
  {
    std::vector<int64_t> aoff(N + 1, 0), adj(2 * (size_t)std::max<int64_t>(N - m->n_cells, 0));
    for (int64_t i = 0; i < N; ++i) {
      const int64_t loc = i - m->cell_off[cell_of[i]];
      if (loc > 0) {
        aoff[i + 1]++;
        aoff[m->cell_off[cell_of[i]] + m->parent[i] + 1]++;
      }
    }
    for (int64_t i = 0; i < N; ++i) aoff[i + 1] += aoff[i];
    {
      std::vector<int64_t> fill(aoff.begin(), aoff.end() - 1);
      for (int64_t i = 0; i < N; ++i) {
        const int64_t loc = i - m->cell_off[cell_of[i]];
        if (loc > 0) {
          const int64_t pi = m->cell_off[cell_of[i]] + m->parent[i];
          adj[fill[i]++] = pi;
          adj[fill[pi]++] = i;
        }
      }
    }
    std::vector<int32_t> dist(N, -1);
    std::vector<int64_t> queue;
    queue.reserve(4096);
    // breadth-first distances from `src` over one cell; returns the farthest compartment (first on ties); when
    // `par` is given, records each compartment's predecessor
    auto bfs = [&](int32_t c, int64_t src, int64_t *par) {
      const int64_t i0 = m->cell_off[c], i1 = m->cell_off[c + 1];
      for (int64_t i = i0; i < i1; ++i) dist[i] = -1;
      queue.clear();
      queue.push_back(src);
      dist[src] = 0;
      if (par) par[src] = -1;
      int64_t far = src;
      for (size_t h = 0; h < queue.size(); ++h) {
        const int64_t u = queue[h];
        if (dist[u] > dist[far] || (dist[u] == dist[far] && u < far)) far = u;
        for (int64_t e = aoff[u]; e < aoff[u + 1]; ++e) {
          const int64_t w = adj[e];
          if (dist[w] < 0) {
            dist[w] = dist[u] + 1;
            if (par) par[w] = u;
            queue.push_back(w);
          }
        }
      }
      return far;
    };
    std::vector<int32_t> da;
    for (int32_t c = 0; c < m->n_cells; ++c) {
      const int64_t i0 = m->cell_off[c], i1 = m->cell_off[c + 1];
      int64_t root = i0;
      if (i1 - i0 > 2) {
        // the ends a, b of a longest path; eccentricity = max(dist to a, dist to b)
        const int64_t a = bfs(c, i0, nullptr);
        const int64_t b = bfs(c, a, nullptr);
        da.assign(dist.begin() + i0, dist.begin() + i1);
        bfs(c, b, nullptr);
        int32_t best = -1;
        for (int64_t i = i0; i < i1; ++i) {
          const int32_t e = std::max(da[i - i0], dist[i]);
          if (best < 0 || e < best) {
            best = e;
            root = i;
          }
        }
      }
      m->cell_root[c] = root;
      bfs(c, root, m->tree_par.data());
      int32_t lv = 0;
      for (int64_t i = i0; i < i1; ++i) {
        depth[i] = dist[i];
        lv = std::max(lv, dist[i] + 1);
      }
      cell_levels[c] = lv;
    }
  }
  const Table &syn = m->mech[CN_MECH_EXPSYN];
  for (int64_t k = 0; k < syn.n; ++k) syn_per_cell[cell_of[syn.node[k]]]++;

  // the default shape holds the largest set of cells joined by gap junctions (one cell when there are none)
  const int64_t max_unit = join_cells(m->cell_off.data(), m->n_cells, N, m->n_gap, m->gap_node.data(),
                                      m->gap_partner.data(), m->cell_cluster);
  int T = m->opt.group_threads, K = m->opt.group_slots;
  default_shape(N, (int32_t)std::min<int64_t>(max_unit, INT32_MAX), m->fp32, T, K);
  if (!shape_compiled(T, K))
    throw Err{CN_E_INVALID, "no compiled cell-group shape " + std::to_string(T) + " x " + std::to_string(K)};
  if (T * K < max_cell) throw Err{CN_E_INVALID, "a cell has more compartments (" + std::to_string(max_cell) +
                                                   ") than one cell group holds (" + std::to_string(T * K) + ")"};
  m->threads = T;
  m->slots = K;
  m->nmax = T * K;
  // packing capacity: the fill percentage of the group, never below the largest cell
  const int fill = m->opt.group_fill_pct > 0 ? std::min(100, m->opt.group_fill_pct) : 100;
  const int64_t cap = std::max<int64_t>(max_cell, (int64_t)m->nmax * fill / 100);
  // synapses per group: up to two LDS rows, so that their terms can be staged on chip
  const int64_t syn_cap = 2 * m->nmax;

  // best-fit decreasing on compartments, with a synapse cap per group. Cells joined by gap junctions are packed
  // as one unit (their junctions read each other's potentials from the group's LDS), listed in cell order.
  std::vector<std::vector<int32_t>> units;
  {
    std::vector<int32_t> unit_of(m->n_cells, -1);
    for (int32_t c = 0; c < m->n_cells; ++c) {
      const int32_t r = m->cell_cluster[c];
      if (unit_of[r] < 0) {
        unit_of[r] = (int32_t)units.size();
        units.emplace_back();
      }
      units[unit_of[r]].push_back(c);
    }
  }
  std::vector<int64_t> unit_size(units.size(), 0), unit_syn(units.size(), 0);
  for (size_t u = 0; u < units.size(); ++u)
    for (int32_t c : units[u]) {
      unit_size[u] += cell_size[c];
      unit_syn[u] += syn_per_cell[c];
    }
  std::vector<int32_t> order(units.size());
  std::iota(order.begin(), order.end(), 0);
  std::stable_sort(order.begin(), order.end(), [&](int32_t a, int32_t b) { return unit_size[a] > unit_size[b]; });
  std::vector<std::vector<int32_t>> gcells;
  std::vector<int64_t> gnodes, gsyn;
  std::multimap<int64_t, int32_t> room;  // remaining capacity -> group
  for (int32_t u : order) {
    const int64_t sz = unit_size[u], sy = unit_syn[u];
    if (sz > cap) throw Err{CN_E_INVALID, "cells joined by gap junctions hold " + std::to_string(sz) +
                                              " compartments, more than one cell group (" + std::to_string(cap) + ")"};
    if (sy >= MAX_GROUP_SYN) throw Err{CN_E_INVALID, "too many synapses on one cell group"};
    int32_t g = -1;
    int tries = 0;
    for (auto it = room.lower_bound(sz); it != room.end() && tries < 8; ++it, ++tries) {
      if (gsyn[it->second] + sy <= syn_cap) {
        g = it->second;
        room.erase(it);
        break;
      }
    }
    if (g < 0) {
      g = (int32_t)gcells.size();
      gcells.emplace_back();
      gnodes.push_back(0);
      gsyn.push_back(0);
    }
    for (int32_t c : units[u]) gcells[g].push_back(c);
    gnodes[g] += sz;
    gsyn[g] += sy;
    const int64_t rem = cap - gnodes[g];
    if (rem > 0) room.emplace(rem, g);
  }
  // heaviest groups first
  std::vector<int32_t> gorder(gcells.size());
  std::iota(gorder.begin(), gorder.end(), 0);
  std::stable_sort(gorder.begin(), gorder.end(), [&](int32_t a, int32_t b) { return gnodes[a] > gnodes[b]; });

  m->n_groups = (int64_t)gcells.size();
  m->n_dev = N;
  m->groups.assign(m->n_groups, GroupDesc{});
  m->dev_of_node.assign(N, -1);
  m->node_of_dev.assign(N, -1);
  m->cell_of_devcell.clear();
  m->lvl_start.clear();
  int64_t node_base = 0;
  int32_t cell_base = 0;
  // children lists per caller compartment, ascending local index
  std::vector<int64_t> ch_off(N + 1, 0), ch_list(N, 0);
  for (int64_t i = 0; i < N; ++i)
    if (m->tree_par[i] >= 0) ch_off[m->tree_par[i] + 1]++;
  for (int64_t i = 0; i < N; ++i) ch_off[i + 1] += ch_off[i];
  {
    std::vector<int64_t> fill(N, 0);
    for (int64_t i = 0; i < N; ++i) {
      const int64_t p = m->tree_par[i];
      if (p >= 0) ch_list[ch_off[p] + fill[p]++] = i;
    }
  }
  std::vector<int64_t> lvl_nodes, next;
  m->max_levels = 0;
  m->max_group_nodes = 0;
  for (int64_t gi = 0; gi < m->n_groups; ++gi) {
    const int32_t g = gorder[gi];
    GroupDesc &gd = m->groups[gi];
    gd.node_base = node_base;
    gd.n_cells = (int32_t)gcells[g].size();
    gd.cell_base = cell_base;
    gd.lvl_base = (int32_t)m->lvl_start.size();
    int64_t pos = 0;
    lvl_nodes.clear();
    for (int32_t c : gcells[g]) {
      lvl_nodes.push_back(m->cell_root[c]);
      m->cell_of_devcell.push_back(c);
    }
    int32_t levels = 0;
    while (!lvl_nodes.empty()) {
      m->lvl_start.push_back((int32_t)pos);
      next.clear();
      for (int64_t i : lvl_nodes) {
        m->dev_of_node[i] = node_base + pos;
        m->node_of_dev[node_base + pos] = i;
        ++pos;
        for (int64_t q = ch_off[i]; q < ch_off[i + 1]; ++q) next.push_back(ch_list[q]);
      }
      lvl_nodes.swap(next);
      ++levels;
    }
    m->lvl_start.push_back((int32_t)pos);
    gd.n_levels = levels;
    gd.n_nodes = (int32_t)pos;
    m->max_levels = std::max(m->max_levels, levels);
    m->max_group_nodes = std::max<int32_t>(m->max_group_nodes, (int32_t)pos);
    m->max_group_cells = std::max<int32_t>(m->max_group_cells, gd.n_cells);
    node_base += pos;
    cell_base += gd.n_cells;
  }
}

// ---- interleaved layout (one lane per cell): cells in groups of 64 consecutive cells, ordered by size (stable, so
// identical cells given next to each other stay together), compartment k of lane j at node_base + 64 k + j
void build_layout_lpc(cn_model *m) {
  const int64_t N = m->n_comp;
  auto size = [&](int32_t c) { return m->cell_off[c + 1] - m->cell_off[c]; };
  // units of cells that go to one group together: a cell, or the cells joined by gap junctions (in cell order);
  // units ordered by their largest cell, and a group closed early when the next unit does not fit its lanes
  gap_clusters(m);
  std::vector<std::vector<int32_t>> units;
  std::vector<int64_t> unit_max;
  {
    std::vector<int32_t> unit_of(m->n_cells, -1);
    for (int32_t c = 0; c < m->n_cells; ++c) {
      const int32_t r = m->cell_cluster[c];
      if (unit_of[r] < 0) {
        unit_of[r] = (int32_t)units.size();
        units.emplace_back();
        unit_max.push_back(0);
      }
      units[unit_of[r]].push_back(c);
      unit_max[unit_of[r]] = std::max(unit_max[unit_of[r]], size(c));
    }
  }
  std::vector<int32_t> uorder(units.size());
  std::iota(uorder.begin(), uorder.end(), 0);
  std::stable_sort(uorder.begin(), uorder.end(), [&](int32_t a, int32_t b) { return unit_max[a] > unit_max[b]; });
  std::vector<int32_t> order;
  std::vector<int32_t> gstart, gcount;  // each group's first entry in `order` and its cell count
  order.reserve(m->n_cells);
  for (int32_t u : uorder) {
    const int32_t n = (int32_t)units[u].size();
    if (n > 64) throw Err{CN_E_INVALID, "more than 64 cells joined by gap junctions (one interleaved group)"};
    if (gstart.empty() || gcount.back() + n > 64) {
      gstart.push_back((int32_t)order.size());
      gcount.push_back(0);
    }
    for (int32_t c : units[u]) order.push_back(c);
    gcount.back() += n;
  }
  m->tree_par.assign(N, -1);
  m->cell_root.assign(m->n_cells, 0);
  for (int32_t c = 0; c < m->n_cells; ++c) {
    m->cell_root[c] = m->cell_off[c];
    for (int64_t i = m->cell_off[c] + 1; i < m->cell_off[c + 1]; ++i) m->tree_par[i] = m->cell_off[c] + m->parent[i];
  }
  m->n_groups = (int64_t)gstart.size();
  m->groups.assign(m->n_groups, GroupDesc{});
  m->cell_of_devcell.assign(order.begin(), order.end());
  m->lvl_start.clear();
  int64_t base = 0;
  int32_t max_kn = 0;
  for (int64_t g = 0; g < m->n_groups; ++g) {
    GroupDesc &gd = m->groups[g];
    gd.cell_base = gstart[g];
    gd.n_cells = gcount[g];
    int32_t kn = 0;
    for (int32_t j = 0; j < gd.n_cells; ++j) kn = std::max<int32_t>(kn, (int32_t)size(order[gd.cell_base + j]));
    gd.node_base = base;
    gd.n_levels = kn;
    gd.n_nodes = 64 * kn;
    gd.lvl_base = 0;
    base += gd.n_nodes;
    max_kn = std::max(max_kn, kn);
  }
  m->n_dev = base;
  if (m->n_dev >= (int64_t)INT32_MAX) throw Err{CN_E_INVALID, "model too large for the interleaved layout"};
  m->dev_of_node.assign(N, -1);
  m->node_of_dev.assign(m->n_dev, -1);
  for (int64_t g = 0; g < m->n_groups; ++g) {
    const GroupDesc &gd = m->groups[g];
    for (int32_t j = 0; j < gd.n_cells; ++j) {
      const int32_t c = order[gd.cell_base + j];
      for (int64_t k = 0; k < size(c); ++k) {
        const int64_t dn = gd.node_base + 64 * k + j;
        m->dev_of_node[m->cell_off[c] + k] = dn;
        m->node_of_dev[dn] = m->cell_off[c] + k;
      }
    }
  }
  m->threads = 64;
  m->slots = max_kn;
  m->nmax = 64 * max_kn;
  m->max_levels = max_kn;
  m->max_group_nodes = m->nmax;
  m->max_group_cells = 64;
}

}  // namespace

// ---- invariants the interval kernel relies on for every index it forms (checked on the host before upload)
static void layout_fail(const char *what) { throw Err{CN_E_INVALID, std::string("internal layout check failed: ") + what}; }

static void check_tree_layout(const cn_model *m, const std::vector<int32_t> &par, const std::vector<uint32_t> &ch) {
  int64_t total = 0;
  for (int64_t g = 0; g < m->n_groups; ++g) {
    const GroupDesc &gd = m->groups[g];
    if (gd.node_base != total) layout_fail("node base");
    if (gd.n_nodes < 1 || gd.n_nodes > m->nmax || gd.n_cells < 1) layout_fail("group size");
    if (gd.n_levels < 1 || gd.lvl_base < 0 || gd.lvl_base + gd.n_levels >= (int64_t)m->lvl_start.size())
      layout_fail("level table");
    const int32_t *lv = m->lvl_start.data() + gd.lvl_base;
    if (lv[0] != 0 || lv[gd.n_levels] != gd.n_nodes || lv[1] != gd.n_cells) layout_fail("level bounds");
    for (int L = 0; L < gd.n_levels; ++L)
      if (lv[L + 1] <= lv[L]) layout_fail("empty level");
    int64_t n_children = 0;
    for (int L = 0; L < gd.n_levels; ++L) {
      for (int32_t q = lv[L]; q < lv[L + 1]; ++q) {
        const int64_t i = gd.node_base + q;
        const int32_t pq = par[i];
        if (L == 0 ? pq != -1 : (pq < lv[L - 1] || pq >= lv[L])) layout_fail("parent level");
        const int32_t c0 = (int32_t)(ch[i] & 0xFFFFu), cn = (int32_t)(ch[i] >> 16);
        if (cn > 0) {
          if (L + 1 >= gd.n_levels || c0 < lv[L + 1] || c0 + cn > lv[L + 2]) layout_fail("children range");
          for (int32_t c = c0; c < c0 + cn; ++c)
            if (par[gd.node_base + c] != q) layout_fail("child's parent");
        }
        n_children += cn;
      }
    }
    if (n_children != gd.n_nodes - gd.n_cells) layout_fail("child count");
    total += gd.n_nodes;
  }
  if (total != m->n_comp) layout_fail("node total");
}

// the interleaved layout: group g holds 64 lanes x n_levels slots from node_base on, slot 64 k + lane; lane j < n_cells
// holds its cell's compartments at k = 0 .. size-1 (caller order, parent index below the compartment's), padding after
static void check_lpc_layout(const cn_model *m, const std::vector<int32_t> &par) {
  int64_t total = 0, real = 0, cells = 0;
  for (int64_t g = 0; g < m->n_groups; ++g) {
    const GroupDesc &gd = m->groups[g];
    if (gd.node_base != total) layout_fail("node base");
    if (gd.cell_base != cells) layout_fail("cell base");
    cells += gd.n_cells;
    if (gd.n_cells < 1 || gd.n_cells > 64 || gd.n_levels < 1 || gd.n_nodes != 64 * gd.n_levels) layout_fail("group size");
    for (int32_t j = 0; j < 64; ++j) {
      int64_t size = 0;
      if (j < gd.n_cells) {
        const int32_t c = m->cell_of_devcell[gd.cell_base + j];
        size = m->cell_off[c + 1] - m->cell_off[c];
        if (size > gd.n_levels) layout_fail("cell larger than its group's slots");
      }
      for (int32_t k = 0; k < gd.n_levels; ++k) {
        const int64_t dn = gd.node_base + 64 * (int64_t)k + j;
        const int64_t i = m->node_of_dev[dn];
        if ((k < size) != (i >= 0)) layout_fail("padding slot");
        if (k < size && i != m->cell_off[m->cell_of_devcell[gd.cell_base + j]] + k) layout_fail("compartment slot");
        if (k > 0 && (par[dn] < 0 || par[dn] >= (k < size ? k : 1))) layout_fail("parent index");
        if (k == 0 && par[dn] != (i >= 0 ? -1 : 0)) layout_fail("root parent");
      }
      real += size;
    }
    total += gd.n_nodes;
  }
  if (total != m->n_dev || real != m->n_comp || cells != m->n_cells) layout_fail("node total");
}

static void check_ranges(const cn_model *m, const std::vector<int2> &r, bool syn) {
  int64_t covered_total = 0;
  for (int64_t g = 0; g < m->n_groups; ++g) {
    const GroupDesc &gd = m->groups[g];
    int64_t next = 0;
    for (int32_t q = 0; q < gd.n_nodes; ++q) {
      const int2 x = r[gd.node_base + q];
      if (x.y < 0) layout_fail("instance range");
      if (x.y == 0) continue;
      if (x.x != next) layout_fail("instance ranges do not tile");
      next += x.y;
    }
    if (syn && next != gd.n_syn) layout_fail("synapse count");
    covered_total += next;
  }
  const int64_t want = syn ? m->mech[CN_MECH_EXPSYN].n : m->mech[CN_MECH_ICLAMP].n;
  if (covered_total != want) layout_fail("instance total");
}

// ---- tables that do not depend on dt
static void build_tables(cn_model *m) {
  const int64_t N = m->n_dev;  // device node slots; a slot with no compartment (padding) is inert
  const bool f32 = m->fp32;
  std::vector<double> a(N, 0.0), b(N, 0.0), sa(N, 0.0);
  std::vector<int32_t> par(N, 0);
  std::vector<uint32_t> ch(N, 0);
  std::vector<uint8_t> mf(N, 0);
  // group of each device node, and group-local index
  std::vector<int32_t> grp_of_dev(N);
  for (int64_t g = 0; g < m->n_groups; ++g)
    for (int32_t q = 0; q < m->groups[g].n_nodes; ++q) grp_of_dev[m->groups[g].node_base + q] = (int32_t)g;
  std::vector<int32_t> first_child(N, -1), n_child(N, 0), cell_of(m->n_comp);
  for (int32_t c = 0; c < m->n_cells; ++c)
    for (int64_t i = m->cell_off[c]; i < m->cell_off[c + 1]; ++i) cell_of[i] = c;
  for (int64_t dn = 0; dn < N; ++dn) {
    const int64_t i = m->node_of_dev[dn];
    if (i < 0) continue;  // padding
    const GroupDesc &gd = m->groups[grp_of_dev[dn]];
    const int64_t c = cell_of[i];  // caller cell of i
    sa[dn] = 100.0 / m->area[i];
    const int64_t pi = m->tree_par[i];
    if (pi < 0) {
      a[dn] = b[dn] = 0.0;
      par[dn] = -1;
    } else {
      // the edge's axial resistance sits at the compartment that is the child in the caller's tree
      const bool same = i != m->cell_off[c] && m->cell_off[c] + m->parent[i] == pi;
      const double g = 1.0 / m->ri[same ? i : pi];
      a[dn] = -100.0 * g / m->area[pi];
      b[dn] = -100.0 * g / m->area[i];
      const int64_t pd = m->dev_of_node[pi];
      if (m->lpc) {  // the parent's compartment index within the cell (its slot is 64 index + lane)
        par[dn] = (int32_t)(pi - m->cell_off[c]);
        continue;
      }
      par[dn] = (int32_t)(pd - gd.node_base);
      const int32_t ql = (int32_t)(dn - gd.node_base);
      if (first_child[pd] < 0 || ql < first_child[pd]) first_child[pd] = ql;
      n_child[pd]++;
    }
  }
  if (m->lpc) {
    check_lpc_layout(m, par);
  } else {
    for (int64_t dn = 0; dn < N; ++dn)
      ch[dn] = (uint32_t)(first_child[dn] < 0 ? 0 : first_child[dn]) | ((uint32_t)n_child[dn] << 16);
    check_tree_layout(m, par, ch);
  }

  // density mechanisms: flags, per-node parameters when not uniform, initial states at v_init
  double hm, hh, hn;
  hh_inf(m->v_init, hm, hh, hn);
  const int flag_of[4] = {MF_HH, MF_PAS, MF_KM, MF_CAHI};
  std::vector<double> prm[4][4];
  for (int t = 0; t < 4; ++t) {
    const Table &tb = m->mech[t];
    if (!tb.present) continue;
    for (int j = 0; j < N_PARAMS[t]; ++j)
      if (!tb.p[j].uniform) prm[t][j].assign(N, 0.0);
    for (int64_t k = 0; k < tb.n; ++k) {
      const int64_t dn = m->dev_of_node[tb.node[k]];
      mf[dn] |= (uint8_t)flag_of[t];
      for (int j = 0; j < N_PARAMS[t]; ++j)
        if (!tb.p[j].uniform) prm[t][j][dn] = tb.p[j].v[k];
    }
  }
  // initial states: each mechanism's steady state at v_init where it is present, zero elsewhere
  auto init_states = [&](auto zero) {
    using S = decltype(zero);
    const double kn = km_inf(m->v_init), cm0 = cahi_inf(m->v_init);
    std::vector<StRec<S>> r(N);
    for (int64_t dn = 0; dn < N; ++dn) {
      const uint8_t f = mf[dn];
      StRec<S> x{};
      if (f & MF_HH) {
        x.m = (S)hm;
        x.h = (S)hh;
        x.n = (S)hn;
      }
      if (f & MF_KM) x.kn = (S)kn;
      if (f & MF_CAHI) {
        x.cm = (S)cm0;
        x.cai = (S)5e-5;
      }
      r[dn] = x;
    }
    return m->upload(r);
  };
  KParams &p = m->kp;
  m->host_a = a;
  m->host_b = b;
  m->host_sa = sa;
  m->host_mf = mf;
  m->host_par = par;
  m->host_ch = ch;
  p.v = m->upload(std::vector<double>(N, m->v_init));
  if (m->lpc) {
    // the elimination's accumulators start at zero (each step's substitution returns them there)
    p.lw_d = m->upload(std::vector<double>(N, 0.0));
    p.lw_r = m->upload(std::vector<double>(N, 0.0));
    p.lw_dv = static_cast<double *>(m->dalloc(N * sizeof(double)));
  }
  {
    std::vector<double> et(64);
    for (int j = 0; j < 64; ++j) et[j] = (double)exp2l((long double)j / 64.0L);
    p.exp_tab = m->upload(et);
  }
  p.n_nodes_total = N;
  if (m->fp32) p.st = init_states(0.0f);
  else p.st = init_states(0.0);
  // density-mechanism parameters: scalars when every column is uniform, else a per-node table of all columns
  {
    const int cols[N_PRM][2] = {{CN_MECH_HH, 0}, {CN_MECH_HH, 1}, {CN_MECH_HH, 2}, {CN_MECH_HH, 3},
                                {CN_MECH_PAS, 0}, {CN_MECH_PAS, 1}, {CN_MECH_KM, 0}, {CN_MECH_CAHI, 0}};
    bool any = false;
    for (int c = 0; c < N_PRM; ++c) {
      const Table &tb = m->mech[cols[c][0]];
      p.prm_s[c] = tb.present ? tb.p[cols[c][1]].s : 0.0;
      if (tb.present && !tb.p[cols[c][1]].uniform) any = true;
    }
    // the uniform kernels also need one mechanism set on every compartment and carry no gap-junction terms; the
    // general kernels read uniform parameters from the same constants and take the table only when a column varies
    const bool same_mechs = N == 0 || std::all_of(mf.begin(), mf.end(), [&](uint8_t x) { return x == mf[0]; });
    p.mf_uni = N ? mf[0] : 0;
    p.uni = !any && same_mechs && m->n_gap == 0;
    p.prm = nullptr;
    if (any) {
      std::vector<double> t(N_PRM * (size_t)N, 0.0);
      for (int c = 0; c < N_PRM; ++c) {
        const Table &tb = m->mech[cols[c][0]];
        if (!tb.present) continue;
        for (int64_t k = 0; k < tb.n; ++k) t[(size_t)c * N + m->dev_of_node[tb.node[k]]] = tb.p[cols[c][1]].v[k];
      }
      p.prm = m->upload(t);
    }
  }

  // point processes in device order: per node, instances in ascending caller index
  auto order_pp = [&](const Table &tb, std::vector<int64_t> &of_dev, std::vector<int64_t> *dev_of) {
    // a stable counting sort by device node
    std::vector<int64_t> start(N + 1, 0), idx(tb.n);
    for (int64_t k = 0; k < tb.n; ++k) start[m->dev_of_node[tb.node[k]] + 1]++;
    for (int64_t dn = 0; dn < N; ++dn) start[dn + 1] += start[dn];
    for (int64_t k = 0; k < tb.n; ++k) idx[start[m->dev_of_node[tb.node[k]]]++] = k;
    of_dev = idx;
    if (dev_of) {
      dev_of->assign(tb.n, 0);
      for (int64_t d = 0; d < tb.n; ++d) (*dev_of)[idx[d]] = d;
    }
  };
  const Table &syn = m->mech[CN_MECH_EXPSYN];
  order_pp(syn, m->syn_of_dev, &m->dev_of_syn);
  const Table &icl = m->mech[CN_MECH_ICLAMP];
  order_pp(icl, m->icl_of_dev, nullptr);
  std::vector<int2> nd_syn(N, int2{0, 0}), nd_icl(N, int2{0, 0});
  // group bases and per-node ranges
  {
    int64_t sd = 0, id = 0;
    m->host_syn_q.assign(syn.n, 0);
    for (int64_t g = 0; g < m->n_groups; ++g) {
      GroupDesc &gd = m->groups[g];
      gd.syn_base = sd;
      gd.icl_base = (int32_t)id;
      const int64_t end = gd.node_base + gd.n_nodes;
      const int64_t s0 = sd, i0 = id;
      while (sd < syn.n && m->dev_of_node[syn.node[m->syn_of_dev[sd]]] < end) {
        const int64_t dn = m->dev_of_node[syn.node[m->syn_of_dev[sd]]];
        if (nd_syn[dn].y == 0) nd_syn[dn].x = (int)(sd - s0);
        nd_syn[dn].y++;
        m->host_syn_q[sd] = (int32_t)(dn - gd.node_base);
        ++sd;
      }
      while (id < icl.n && m->dev_of_node[icl.node[m->icl_of_dev[id]]] < end) {
        const int64_t dn = m->dev_of_node[icl.node[m->icl_of_dev[id]]];
        if (nd_icl[dn].y == 0) nd_icl[dn].x = (int)(id - i0);
        nd_icl[dn].y++;
        ++id;
      }
      gd.n_syn = (int32_t)(sd - s0);
      m->max_group_syn = std::max(m->max_group_syn, gd.n_syn);
    }
  }
  check_ranges(m, nd_syn, true);
  check_ranges(m, nd_icl, false);
  // half-gap junctions in device order (per node, ascending caller index). The partner sits in the same group
  // (cells joined by a junction are packed together); its record holds the partner's group-local slot and the
  // conductance per unit area of the junction's own compartment.
  std::vector<int2> nd_gap(N, int2{0, 0});
  p.gap = nullptr;
  p.nd_gap0 = nullptr;
  if (m->n_gap > 0) {
    std::vector<int64_t> start(N + 1, 0), idx(m->n_gap);
    for (int64_t k = 0; k < m->n_gap; ++k) start[m->dev_of_node[m->gap_node[k]] + 1]++;
    for (int64_t dn = 0; dn < N; ++dn) start[dn + 1] += start[dn];
    for (int64_t k = 0; k < m->n_gap; ++k) idx[start[m->dev_of_node[m->gap_node[k]]]++] = k;
    std::vector<GapRec> gr(m->n_gap);
    int64_t d = 0;
    for (int64_t g = 0; g < m->n_groups; ++g) {
      GroupDesc &gd = m->groups[g];
      gd.gap_base = (int32_t)d;
      const int64_t end = gd.node_base + gd.n_nodes, d0 = d;
      while (d < m->n_gap && m->dev_of_node[m->gap_node[idx[d]]] < end) {
        const int64_t k = idx[d], dn = m->dev_of_node[m->gap_node[k]], pd = m->dev_of_node[m->gap_partner[k]];
        if (dn < gd.node_base || pd < gd.node_base || pd >= end) layout_fail("gap-junction partner outside its group");
        if (nd_gap[dn].y == 0) nd_gap[dn].x = (int)(d - d0);
        nd_gap[dn].y++;
        gr[d] = GapRec{(int32_t)(pd - gd.node_base), 0, 100.0 * m->gap_g[k] / m->area[m->gap_node[k]]};
        ++d;
      }
    }
    if (d != m->n_gap) layout_fail("gap-junction order");
    std::vector<int32_t> gap0(N, 0);
    for (int64_t dn = 0; dn < N; ++dn) {
      if (nd_gap[dn].y > MAX_NODE_GAP) throw Err{CN_E_INVALID, "more than 15 gap junctions on one compartment"};
      gap0[dn] = nd_gap[dn].x;
    }
    p.gap = m->upload(gr);
    p.nd_gap0 = m->upload(gap0);
  }
  {
    std::vector<NodeIdx> nx(N);
    std::vector<int32_t> icl0(N, 0);
    for (int64_t dn = 0; dn < N; ++dn) {
      if (nd_syn[dn].y > MAX_NODE_SYN) throw Err{CN_E_INVALID, "more than 65535 synapses on one compartment"};
      if (nd_icl[dn].y > MAX_NODE_ICL) throw Err{CN_E_INVALID, "more than 255 IClamps on one compartment"};
      nx[dn].par = m->host_par[dn];
      nx[dn].ch = m->host_ch[dn];
      nx[dn].syn0 = nd_syn[dn].x;
      nx[dn].pk = (uint32_t)nd_syn[dn].y | ((uint32_t)nd_icl[dn].y << 16) | ((uint32_t)m->host_mf[dn] << 24) |
                  ((uint32_t)nd_gap[dn].y << 28);
      icl0[dn] = nd_icl[dn].x;
    }
    p.nidx = m->upload(nx);
    p.nd_icl0 = m->upload(icl0);
  }
  {
    m->host_syn_key.assign(syn.n, 0);
    m->host_syn_e.assign(syn.n, 0.0);
    m->host_syn_wbg.assign(syn.n, 0.0);
    for (int64_t d = 0; d < syn.n; ++d) {
      const int64_t k = m->syn_of_dev[d];
      m->host_syn_e[d] = syn.p[1].v[k];
      m->host_syn_key[d] = (uint64_t)(m->pkey.empty() ? k : m->pkey[k]);
      if (m->rate > 0.0) m->host_syn_wbg[d] = m->pw[k];
    }
    p.syn_g = m->upload_s(std::vector<double>(syn.n, 0.0));
  }
  // cells in device order
  {
    std::vector<int32_t> gid(m->n_cells), soma(m->n_cells);
    std::vector<double> th(m->n_cells);
    for (int64_t g = 0; g < m->n_groups; ++g) {
      const GroupDesc &gd = m->groups[g];
      for (int32_t k = 0; k < gd.n_cells; ++k) {
        const int32_t c = gd.cell_base + k;
        gid[c] = m->cell_of_devcell[c];
        th[c] = m->theta[m->cell_of_devcell[c]];
        const int64_t sd = m->dev_of_node[m->cell_off[m->cell_of_devcell[c]]] - gd.node_base;
        if (sd < 0 || sd >= gd.n_nodes) layout_fail("soma position");
        soma[c] = (int32_t)sd;
      }
    }
    p.cell_gid = m->upload(gid);
    p.cell_theta = m->upload(th);
    p.cell_soma = m->upload(soma);
  }
  // network: targets, source CSR; kicks by (group, step, id)
  {
    std::vector<int32_t> tgt_g(m->n_nc), tgt_l(m->n_nc);
    std::vector<int32_t> grp_of_dsyn(syn.n);
    for (int64_t g = 0; g < m->n_groups; ++g)
      for (int32_t s = 0; s < m->groups[g].n_syn; ++s) grp_of_dsyn[m->groups[g].syn_base + s] = (int32_t)g;
    for (int64_t k = 0; k < m->n_nc; ++k) {
      const int64_t d = m->dev_of_syn[m->nc_syn[k]];
      tgt_g[k] = grp_of_dsyn[d];
      tgt_l[k] = (int32_t)(d - m->groups[tgt_g[k]].syn_base);
    }
    p.nc_tgt_group = m->upload(tgt_g);
    p.nc_tgt_lsyn = m->upload(tgt_l);
    p.nc_w = m->upload_s(m->nc_w);
    std::vector<int64_t> off(m->n_cells + 1, 0);
    for (int64_t k = 0; k < m->n_nc; ++k) off[m->nc_src[k] + 1]++;
    for (int32_t c = 0; c < m->n_cells; ++c) off[c + 1] += off[c];
    std::vector<int32_t> onc(m->n_nc);
    std::vector<int64_t> fill(m->n_cells, 0);
    for (int64_t k = 0; k < m->n_nc; ++k) onc[off[m->nc_src[k]] + fill[m->nc_src[k]]++] = (int32_t)k;
    p.out_off = m->upload(off);
    p.out_nc = m->upload(onc);
    m->host_out_off = off;
    m->host_out_nc = onc;
    m->host_tgt_g = tgt_g;
    m->host_tgt_l = tgt_l;
    std::vector<int64_t> kidx(m->n_kick);
    std::iota(kidx.begin(), kidx.end(), 0);
    std::vector<int32_t> kg(m->n_kick);
    for (int64_t k = 0; k < m->n_kick; ++k) kg[k] = grp_of_dsyn[m->dev_of_syn[m->kick_syn[k]]];
    std::stable_sort(kidx.begin(), kidx.end(), [&](int64_t x, int64_t y) {
      if (kg[x] != kg[y]) return kg[x] < kg[y];
      return m->kick_step[x] < m->kick_step[y];
    });
    std::vector<int64_t> ks(m->n_kick);
    std::vector<int32_t> kl(m->n_kick), kid(m->n_kick);
    for (auto &gd : m->groups) gd.kick_base = gd.n_kick = 0;
    for (int64_t q = 0; q < m->n_kick; ++q) {
      const int64_t k = kidx[q];
      ks[q] = m->kick_step[k];
      const int64_t d = m->dev_of_syn[m->kick_syn[k]];
      kl[q] = (int32_t)(d - m->groups[kg[k]].syn_base);
      kid[q] = (int32_t)k;
    }
    for (int64_t q = m->n_kick - 1; q >= 0; --q) {
      GroupDesc &gd = m->groups[kg[kidx[q]]];
      gd.kick_base = (int32_t)q;
      gd.n_kick++;
    }
    for (int64_t k = 0; k < m->n_nc; ++k)
      if (tgt_g[k] < 0 || tgt_g[k] >= m->n_groups || tgt_l[k] < 0 || tgt_l[k] >= m->groups[tgt_g[k]].n_syn)
        throw Err{CN_E_INVALID, "internal layout check failed: NetCon target"};
    for (int64_t g = 0; g < m->n_groups; ++g) {
      const GroupDesc &gd = m->groups[g];
      if (gd.kick_base < 0 || gd.n_kick < 0 || gd.kick_base + gd.n_kick > m->n_kick)
        throw Err{CN_E_INVALID, "internal layout check failed: kick range"};
      for (int32_t q = gd.kick_base; q < gd.kick_base + gd.n_kick; ++q)
        if (kl[q] < 0 || kl[q] >= gd.n_syn || (q > gd.kick_base && ks[q] < ks[q - 1]))
          throw Err{CN_E_INVALID, "internal layout check failed: kick order"};
    }
    p.kick_step = m->upload(ks);
    p.kick_lsyn = m->upload(kl);
    p.kick_id = m->upload(kid);
    p.kick_w = m->upload_s(m->kick_w);
  }
  p.lvl_start = m->upload(m->lvl_start);
#ifdef CN_PHASE_CLOCKS
  p.phase_clk = m->upload(std::vector<uint64_t>(PH_COUNT, 0));
#else
  p.phase_clk = nullptr;
#endif
  p.n_groups = (int32_t)m->n_groups;
  // readout tables: caller instance -> device node (density mechanisms with states; a dense table shares one) or
  // device synapse (ExpSyn)
  {
    const int32_t *dense = nullptr;
    for (int t : {CN_MECH_HH, CN_MECH_KM, CN_MECH_CAHI}) {
      const Table &tb = m->mech[t];
      if (!tb.present) continue;
      bool is_dense = tb.n == N;
      for (int64_t k = 0; is_dense && k < tb.n; ++k) is_dense = tb.node[k] == k;
      if (is_dense && dense) {
        m->inst_dev[t] = dense;
        continue;
      }
      std::vector<int32_t> id(tb.n);
      for (int64_t k = 0; k < tb.n; ++k) id[k] = (int32_t)m->dev_of_node[tb.node[k]];
      m->inst_dev[t] = m->upload(id);
      if (is_dense) dense = m->inst_dev[t];
    }
    if (syn.present) {
      std::vector<int32_t> id(syn.n);
      for (int64_t k = 0; k < syn.n; ++k) id[k] = (int32_t)m->dev_of_syn[k];
      m->inst_dev[CN_MECH_EXPSYN] = m->upload(id);
    }
  }
}

// the kernel that advances every group through one chunk
static hipError_t launch_chunk(cn_model *m) {
  if (m->lpc) return launch_lpc(m->kp, m->fp32, m->lds_bytes, m->stream);
  return launch_interval(m->kp, m->fp32, m->threads, m->slots, m->lds_bytes, m->stream);
}

// ---- tables that depend on dt; allocation of the event ring and spike buffers; graph capture
static void prepare_dt(cn_model *m, double dt) {
  KParams &p = m->kp;
  const int64_t N = m->n_dev;
  p.dt = dt;
  p.q10dt = std::pow(3.0, (m->celsius - 6.3) / 10.0) * dt;
  p.ca_fm = 1.0 - std::exp(-dt / 1.0);
  p.ca_fr = 1.0 - std::exp(-dt / 80.0);
  p.ca_k = 1e4 / (2.0 * 96485.33212 * 0.1) * 80.0;
  {
    std::vector<double> k(N);
    // capacitance term 1e-3 cm/dt (S/cm^2) and the node's own axial coupling -b
    std::vector<NodeRec> rec(N);
    for (int64_t dn = 0; dn < N; ++dn) {
      const int64_t i = m->node_of_dev[dn];
      k[dn] = i < 0 ? 1.0 : 1e-3 * m->cm[i] / dt - m->host_b[dn];  // a padding slot solves d = 1, rhs = 0
      rec[dn] = NodeRec{m->host_a[dn], m->host_b[dn], k[dn], m->host_sa[dn]};
    }
    p.nrec = m->upload(rec);
  }
  const Table &syn = m->mech[CN_MECH_EXPSYN];
  {
    // synapse records: stream id, reversal, 100/area of the compartment, background weight, decay factor
    // exp(-dt/tau), compartment
    std::vector<double> f(syn.n);
    auto syn_sa = [&](int64_t d) { return m->host_sa[m->dev_of_node[syn.node[m->syn_of_dev[d]]]]; };
    for (int64_t d = 0; d < syn.n; ++d) f[d] = std::exp(-dt / syn.p[0].v[m->syn_of_dev[d]]);
    if (m->fp32) {
      std::vector<SynRec<float>> r(syn.n);
      for (int64_t d = 0; d < syn.n; ++d)
        r[d] = SynRec<float>{m->host_syn_key[d], m->host_syn_e[d], syn_sa(d), (float)m->host_syn_wbg[d], (float)f[d],
                             m->host_syn_q[d], 0};
      p.syn = m->upload(r);
    } else {
      std::vector<SynRec<double>> r(syn.n);
      for (int64_t d = 0; d < syn.n; ++d)
        r[d] = SynRec<double>{m->host_syn_key[d], m->host_syn_e[d], syn_sa(d), m->host_syn_wbg[d], f[d],
                              m->host_syn_q[d], 0};
      p.syn = m->upload(r);
    }
  }
  const Table &icl = m->mech[CN_MECH_ICLAMP];
  {
    std::vector<IclRec> r(icl.n);
    for (int64_t d = 0; d < icl.n; ++d) {
      const int64_t k = m->icl_of_dev[d];
      r[d].cur = 100.0 * icl.p[2].v[k] / m->area[icl.node[k]];
      r[d].on = (int64_t)std::ceil(icl.p[0].v[k] / dt - 0.5);
      r[d].off = (int64_t)std::ceil((icl.p[0].v[k] + icl.p[1].v[k]) / dt - 0.5);
      r[d].pad = 0.0;
    }
    p.icl = m->upload(r);
  }
  // delays in steps, interval length M, ring of interval slots
  int64_t minD = INT64_MAX, maxD = 0;
  std::vector<int32_t> D(m->n_nc);
  for (int64_t k = 0; k < m->n_nc; ++k) {
    const double x = std::floor(m->nc_delay[k] / dt + 0.5);
    if (!(x >= 1.0) || x > 1e9) throw Err{CN_E_INVALID, "NetCon delay must be at least one step"};
    D[k] = (int32_t)x;
    minD = std::min<int64_t>(minD, D[k]);
    maxD = std::max<int64_t>(maxD, D[k]);
  }
  int64_t M = m->opt.max_interval > 0 ? m->opt.max_interval : 64;
  if (M > MAX_INTERVAL) M = MAX_INTERVAL;
  if (m->n_nc > 0) M = std::min(M, minD);
  p.M = (int32_t)M;
  p.ring = (int32_t)(2 + maxD / M);
  p.nc_D = m->upload(D);
  m->host_D = D;
  // background stream threshold: event iff word < floor(p 2^32), p = rate dt 1e-3
  p.has_bg = m->rate > 0.0 ? 1 : 0;
  p.has_icl = m->mech[CN_MECH_ICLAMP].present && m->mech[CN_MECH_ICLAMP].n > 0 ? 1 : 0;
  {
    const double pr = m->rate * dt * 1e-3;
    const double t = std::floor(pr * 4294967296.0);
    p.bg_thresh = t >= 4294967296.0 ? 4294967296ull : (uint64_t)t;
  }
  // event ring
  // default capacity: 512 events per 1024 compartments of group capacity (a group's events grow with its synapses)
  // (interleaved layout: a quarter of the largest group's synapse count, at least 512)
  int cap = m->opt.event_capacity > 0 ? m->opt.event_capacity
                                      : (m->lpc ? std::max(512, m->max_group_syn / 4) : std::max(512, m->nmax / 2));
  int pc = 1;
  while (pc < cap) pc <<= 1;
  p.ev_cap = pc;
  const int64_t nbk = (int64_t)p.ring * m->n_groups;
  p.ev_cnt = static_cast<int32_t *>(m->dalloc(nbk * sizeof(int32_t)));
  HIPCHK(launch_fill_i32(p.ev_cnt, nbk, 0, m->stream));
  p.ev_key = static_cast<uint64_t *>(m->dalloc(nbk * (int64_t)pc * sizeof(uint64_t)));
  // per-group spike scratch: at most ceil(M/2) spikes per cell per chunk
  const int32_t per_cell = (int32_t)((M + 1) / 2);
  int64_t sb = 0;
  for (auto &gd : m->groups) {
    gd.spk_base = (int32_t)sb;
    sb += (int64_t)gd.n_cells * per_cell;
  }
  if (sb >= INT32_MAX) throw Err{CN_E_INVALID, "model too large for the spike scratch"};
  p.gsp_pack = static_cast<int32_t *>(m->dalloc(sb * sizeof(int32_t)));
  p.gsp_cnt = static_cast<int32_t *>(m->dalloc(m->n_groups * sizeof(int32_t)));
  HIPCHK(launch_fill_i32(p.gsp_cnt, m->n_groups, 0, m->stream));
  p.gsp_frac = static_cast<double *>(m->dalloc(sb * sizeof(double)));
  // spike record drained to the host every drain_every chunks
  const int64_t per_chunk = (int64_t)m->n_cells * per_cell;
  int64_t de = std::max<int64_t>(1, std::min<int64_t>(64, (16ll << 20) / std::max<int64_t>(1, per_chunk)));
  m->drain_every = (int32_t)de;
  const int64_t rc = per_chunk * de;
  if (rc >= INT32_MAX) throw Err{CN_E_INVALID, "model too large for the spike record"};
  p.rec_cap = (int32_t)rc;
  p.rec_cnt = static_cast<int32_t *>(m->dalloc(sizeof(int32_t) * 4));
  p.flags = static_cast<int32_t *>(m->dalloc(sizeof(int32_t) * 4));
  HIPCHK(launch_fill_i32(p.rec_cnt, 4, 0, m->stream));
  HIPCHK(launch_fill_i32(p.flags, 4, 0, m->stream));
  p.rec_gid = static_cast<int32_t *>(m->dalloc(rc * sizeof(int32_t)));
  p.rec_step = static_cast<int64_t *>(m->dalloc(rc * sizeof(int64_t)));
  p.rec_t = static_cast<double *>(m->dalloc(rc * sizeof(double)));
  p.ctl = static_cast<int64_t *>(m->dalloc(4 * sizeof(int64_t)));
  p.groups = m->upload(m->groups);
  // LDS: four working rows of doubles per node (the kernel sizes rows by the group capacity T K), the per-node
  // constants (three doubles and three 32-bit indices) for groups of up to 2048 nodes, event keys, step segments,
  // level starts, background bits, counters
  p.nmax = m->nmax;
  int off = m->lpc ? 0 : interval_row_bytes(m->nmax);  // the interleaved layout keeps no node rows on chip
  p.lds_ev_off = off;
  off += p.ev_cap * 8;
  p.lds_seg_off = off;
  off += (p.M + 1) * 4;
  p.lds_lvl_off = off;
  off += (m->max_levels + 1) * 4;
  p.lds_bg_off = off;
  off += std::max<int32_t>(m->max_group_syn, 1);
  off = (off + 15) / 16 * 16;
  p.lds_cell_off = off;  // per cell: threshold and soma potential (doubles), soma position (32-bit)
  off += m->max_group_cells * 20;
  off = (off + 15) / 16 * 16;
  p.lds_misc_off = off;
  off += 16;
  p.lds_cst_off = off;
  off += N_CST * 8;
  p.lds_exp_off = off;
  off += 64 * 8;
  m->lds_bytes = off;
  if (m->lds_bytes > 160 * 1024)
    throw Err{CN_E_INVALID, "cell groups need " + std::to_string(m->lds_bytes) + " bytes of LDS (event_capacity "
                                "or synapses per group too large)"};
  if (m->lpc) {
    HIPCHK(set_lpc_lds(m->fp32, p.uni != 0, m->lds_bytes));
    HIPCHK(lpc_groups_per_cu(m->fp32, p.uni != 0, m->lds_bytes, &m->groups_per_cu));
  } else {
    HIPCHK(set_interval_lds(m->fp32, m->threads, m->slots, p.uni != 0, m->lds_bytes));
    HIPCHK(interval_groups_per_cu(m->fp32, m->threads, m->slots, p.uni != 0, m->lds_bytes, &m->groups_per_cu));
  }
  HIPCHK(hipStreamSynchronize(m->stream));
  if (m->opt.use_graph) {
    HIPCHK(hipStreamBeginCapture(m->stream, hipStreamCaptureModeThreadLocal));
    // whatever fails below, the capture is ended before the error is reported, so that the caller's stream never
    // stays in capture mode
    hipError_t e1 = launch_chunk(m);
    if (e1 == hipSuccess) e1 = launch_fanout(m->kp, m->stream);
    hipError_t e2 = launch_advance(p.ctl, p.M, m->stream);
    if (m->opt.fault_inject == 2 && e2 == hipSuccess) e2 = hipErrorLaunchFailure;
    hipError_t e3 = hipStreamEndCapture(m->stream, &m->graph);
    if (e1 != hipSuccess || e2 != hipSuccess || e3 != hipSuccess) {
      if (m->graph) (void)hipGraphDestroy(m->graph);
      m->graph = nullptr;
    }
    HIPCHK(e1);
    HIPCHK(e2);
    HIPCHK(e3);
    HIPCHK(hipGraphInstantiate(&m->gexec, m->graph, nullptr, nullptr, 0));
  }
}

static void drain(cn_model *m, int32_t n_timed) {
  KParams &p = m->kp;
  HIPCHK(hipStreamSynchronize(m->stream));
  if (m->opt.fault_inject == 1) HIPCHK(hipErrorLaunchFailure);
  int32_t cnt = 0, flags[4];
  HIPCHK(hipMemcpy(&cnt, p.rec_cnt, sizeof cnt, hipMemcpyDeviceToHost));
  HIPCHK(hipMemcpy(flags, p.flags, sizeof flags, hipMemcpyDeviceToHost));
  const int32_t got = std::min(cnt, p.rec_cap);
  if (got > 0) {
    const size_t b = m->sp_gid.size();
    m->sp_gid.resize(b + got);
    m->sp_step.resize(b + got);
    m->sp_t.resize(b + got);
    HIPCHK(hipMemcpy(m->sp_gid.data() + b, p.rec_gid, got * sizeof(int32_t), hipMemcpyDeviceToHost));
    HIPCHK(hipMemcpy(m->sp_step.data() + b, p.rec_step, got * sizeof(int64_t), hipMemcpyDeviceToHost));
    HIPCHK(hipMemcpy(m->sp_t.data() + b, p.rec_t, got * sizeof(double), hipMemcpyDeviceToHost));
  }
  HIPCHK(launch_fill_i32(p.rec_cnt, 1, 0, m->stream));
  for (int32_t k = 0; k < n_timed; ++k) {
    float ms = 0.f;
    HIPCHK(hipEventElapsedTime(&ms, m->ev_pool[2 * k], m->ev_pool[2 * k + 1]));
    m->kernel_ms += ms;
    m->kernel_launches++;
  }
  if (flags[FLAG_EV_OVERFLOW] || flags[FLAG_REC_OVERFLOW]) {
    m->broken = true;
    throw Err{CN_E_CAPACITY, flags[FLAG_EV_OVERFLOW] ? "event ring overflow: raise cn_options.event_capacity"
                                                     : "spike record overflow"};
  }
  if (flags[FLAG_NONFINITE]) {
    m->broken = true;
    throw Err{CN_E_NUMERIC, "non-finite membrane potential"};
  }
}

namespace cn {

int set_error(int code, const char *msg) { return fail(code, msg); }

int model_device(const cn_model *m) { return m->device; }

// argument checks of the state readouts
int mech_state_check(const cn_model *m, int32_t type, int32_t which, const double *out, int64_t n) {
  if (!m || !out) return fail(CN_E_INVALID, "NULL argument");
  if (m->dry) return fail(CN_E_STATE, "model was built with validate_only");
  if (type < 0 || type >= CN_MECH_COUNT || !m->mech[type].present) return fail(CN_E_INVALID, "no such mechanism");
  if (n != m->mech[type].n) return fail(CN_E_INVALID, "n does not match the instance count");
  const int nw[CN_MECH_COUNT] = {3, 0, 1, 2, 1, 0};
  if (which < 0 || which >= nw[type]) return fail(CN_E_INVALID, "no such state");
  return CN_OK;
}

// A state readout after mech_state_check: one gather kernel writes the state of every instance, in the caller's
// instance order, into the device buffer dbuf (n doubles; unused before the first run), which is then copied to out.
// Allocates nothing itself.
int mech_state_run(const cn_model *m, int32_t type, int32_t which, double *out, int64_t n, double *dbuf) {
  if (n == 0) return CN_OK;
  try {
    if (!m->dt_fixed && type != CN_MECH_EXPSYN) {  // before the first run, states sit at their initial values
      double hm, hh, hn;
      hh_inf(m->v_init, hm, hh, hn);
      double x = 0.0;
      if (type == CN_MECH_HH) x = which == 0 ? hm : (which == 1 ? hh : hn);
      else if (type == CN_MECH_KM) x = km_inf(m->v_init);
      else x = which == 0 ? cahi_inf(m->v_init) : 5e-5;
      for (int64_t k = 0; k < n; ++k) out[k] = m->fp32 ? (double)(float)x : x;
      return CN_OK;
    }
    if (!m->dt_fixed) {  // no conductance before the first run
      for (int64_t k = 0; k < n; ++k) out[k] = 0.0;
      return CN_OK;
    }
    HIPCHK(launch_gather_state(m->kp, m->fp32, m->inst_dev[type], n, m->step, m->fresh_step, type, which, dbuf,
                               m->stream));
    HIPCHK(hipMemcpyAsync(out, dbuf, n * sizeof(double), hipMemcpyDeviceToHost, m->stream));
    HIPCHK(hipStreamSynchronize(m->stream));
  } catch (const Err &e) {
    return fail(e.code, e.msg);
  }
  return CN_OK;
}

}  // namespace cn

extern "C" {

const char *cn_last_error(void) { return g_err.c_str(); }

int cn_model_create(const cn_topology *topo, const cn_mech_table *mechs, int32_t n_mechs, const cn_network *net,
                    const cn_options *opt, cn_model **out) {
  if (!out) return fail(CN_E_INVALID, "out is NULL");
  *out = nullptr;
  cn_model *m = nullptr;
  try {
    m = new cn_model();
  } catch (...) {
    return fail(CN_E_NOMEM, "out of host memory");
  }
  try {
    if (!topo) throw Err{CN_E_INVALID, "topology is NULL"};
    if (opt) m->opt = *opt;
    if (m->opt.precision != CN_PREC_FP64 && m->opt.precision != CN_PREC_FP32_MECH)
      throw Err{CN_E_INVALID, "unknown precision"};
    if (m->opt.layout != CN_LAYOUT_AUTO && m->opt.layout != CN_LAYOUT_LEVEL && m->opt.layout != CN_LAYOUT_INTERLEAVED)
      throw Err{CN_E_INVALID, "unknown layout"};
    m->lpc = m->opt.layout == CN_LAYOUT_INTERLEAVED;
    if (m->opt.dev_alloc && !m->opt.dev_free) throw Err{CN_E_INVALID, "dev_alloc without dev_free"};
    m->fp32 = m->opt.precision == CN_PREC_FP32_MECH;
    if (topo->n_cells <= 0 || topo->n_comp <= 0) throw Err{CN_E_INVALID, "empty model"};
    if (topo->n_comp >= (int64_t)INT32_MAX) throw Err{CN_E_INVALID, "more than 2^31 - 2 compartments"};
    if (!topo->cell_offset || !topo->parent || !topo->area || !topo->ri || !topo->cm)
      throw Err{CN_E_INVALID, "topology arrays missing"};
    if (!std::isfinite(topo->v_init) || !std::isfinite(topo->celsius)) throw Err{CN_E_INVALID, "non-finite v_init/celsius"};
    m->n_cells = topo->n_cells;
    m->n_comp = topo->n_comp;
    m->cell_off.assign(topo->cell_offset, topo->cell_offset + m->n_cells + 1);
    if (m->cell_off[0] != 0 || m->cell_off[m->n_cells] != m->n_comp) throw Err{CN_E_INVALID, "bad cell_offset"};
    for (int32_t c = 0; c < m->n_cells; ++c)
      if (m->cell_off[c + 1] <= m->cell_off[c]) throw Err{CN_E_INVALID, "cell_offset must be strictly increasing"};
    m->parent.assign(topo->parent, topo->parent + m->n_comp);
    m->area.assign(topo->area, topo->area + m->n_comp);
    m->ri.assign(topo->ri, topo->ri + m->n_comp);
    m->cm.assign(topo->cm, topo->cm + m->n_comp);
    for (int32_t c = 0; c < m->n_cells; ++c) {
      const int64_t i0 = m->cell_off[c], n = m->cell_off[c + 1] - i0;
      for (int64_t k = 0; k < n; ++k) {
        const int64_t i = i0 + k;
        const int32_t pp = m->parent[i];
        if (!(m->area[i] > 0.0) || !std::isfinite(m->area[i]) || !(m->cm[i] > 0.0) || !std::isfinite(m->cm[i]))
          throw Err{CN_E_INVALID, "area and cm must be positive and finite (compartment " + std::to_string(i) + ")"};
        if (k == 0) {
          if (pp != -1) throw Err{CN_E_INVALID, "root parent must be -1 (cell " + std::to_string(c) + ")"};
        } else {
          if (pp < 0 || pp >= k) throw Err{CN_E_INVALID, "parent[i] must lie in [0, i) (compartment " + std::to_string(i) + ")"};
          if (!(m->ri[i] > 0.0) || !std::isfinite(m->ri[i]))
            throw Err{CN_E_INVALID, "ri must be positive and finite (compartment " + std::to_string(i) + ")"};
        }
      }
    }
    m->v_init = topo->v_init;
    m->celsius = topo->celsius;
    read_tables(m, mechs, n_mechs);
    read_network(m, net);
    m->dry = m->opt.validate_only != 0;
    if (m->dry) {
      m->stream = nullptr;
    } else if (m->opt.stream) {
      m->stream = static_cast<hipStream_t>(m->opt.stream);
    } else {
      HIPCHK(hipStreamCreateWithFlags(&m->stream, hipStreamNonBlocking));
      m->own_stream = true;
    }
    if (!m->dry) HIPCHK(hipGetDevice(&m->device));
    if (m->lpc) build_layout_lpc(m);
    else build_layout(m);
    build_tables(m);
    if (!m->dry) HIPCHK(hipStreamSynchronize(m->stream));
  } catch (const Err &e) {
    delete m;
    return fail(e.code, e.msg);
  } catch (const std::bad_alloc &) {
    delete m;
    return fail(CN_E_NOMEM, "out of host memory");
  } catch (...) {
    delete m;
    return fail(CN_E_INVALID, "unexpected failure in cn_model_create");
  }
  *out = m;
  return CN_OK;
}

int cn_run(cn_model *m, double tstop, double dt) {
  if (!m) return fail(CN_E_INVALID, "model is NULL");
  if (m->broken) return fail(CN_E_STATE, "model is in an error state after a failed run");
  if (m->dry) return fail(CN_E_STATE, "model was built with validate_only");
  if (!(dt > 0.0) || !std::isfinite(dt) || !std::isfinite(tstop)) return fail(CN_E_INVALID, "bad tstop or dt");
  if (m->dt_fixed && dt != m->dt) return fail(CN_E_STATE, "dt differs from the first cn_run call");
  const double nd = tstop / dt;
  if (!(std::fabs(nd) < 9.0e18)) return fail(CN_E_INVALID, "tstop / dt out of range");
  const int64_t N = llround(nd);
  if (N < m->step) return fail(CN_E_STATE, "tstop lies before the current time");
  // From the first device call on, a failure leaves the device state (potentials, states, event ring, spike record)
  // out of step with the host's step counter: the model is then marked broken and refuses further runs.
  bool touched = false;
  try {
    if (!m->dt_fixed) {
      touched = true;
      prepare_dt(m, dt);
      m->dt = dt;
      m->dt_fixed = true;
    }
    if (N == m->step) return CN_OK;
    KParams &p = m->kp;
    touched = true;
    HIPCHK(launch_set_ctl(p.ctl, m->step, N, m->fresh_step, m->seed, m->stream));
    const bool timing = m->opt.timing != 0;
    if (timing && (int32_t)m->ev_pool.size() < 2 * m->drain_every) {
      while ((int32_t)m->ev_pool.size() < 2 * m->drain_every) {
        hipEvent_t e;
        HIPCHK(hipEventCreate(&e));
        m->ev_pool.push_back(e);
      }
    }
    int64_t cur = m->step;
    int32_t since = 0;
    while (cur < N) {
      if (timing) HIPCHK(hipEventRecord(m->ev_pool[2 * since], m->stream));
      if (m->gexec) {
        HIPCHK(hipGraphLaunch(m->gexec, m->stream));
      } else {
        HIPCHK(launch_chunk(m));
        HIPCHK(launch_fanout(p, m->stream));
        HIPCHK(launch_advance(p.ctl, p.M, m->stream));
      }
      if (timing) HIPCHK(hipEventRecord(m->ev_pool[2 * since + 1], m->stream));
      cur = std::min<int64_t>(N, (cur / p.M + 1) * p.M);
      ++since;
      if (since == m->drain_every || cur == N) {
        drain(m, timing ? since : 0);
        since = 0;
      }
    }
    m->step = N;
  } catch (const Err &e) {
    if (touched) m->broken = true;
    return fail(e.code, e.msg);
  } catch (const std::bad_alloc &) {
    if (touched) m->broken = true;
    return fail(CN_E_NOMEM, "out of host memory");
  } catch (...) {
    if (touched) m->broken = true;
    return fail(CN_E_DEVICE, "unexpected failure in cn_run");
  }
  return CN_OK;
}

int cn_spikes(const cn_model *m, int64_t *n_out, int32_t *gid, int64_t *step, double *t_interp, int64_t cap) {
  if (!m || !n_out) return fail(CN_E_INVALID, "NULL argument");
  const int64_t n = (int64_t)m->sp_gid.size();
  *n_out = n;
  if (!gid) return CN_OK;
  if (cap < n) return fail(CN_E_INVALID, "spike buffer too small");
  std::vector<int64_t> idx(n);
  std::iota(idx.begin(), idx.end(), 0);
  std::sort(idx.begin(), idx.end(), [&](int64_t a, int64_t b) {
    if (m->sp_step[a] != m->sp_step[b]) return m->sp_step[a] < m->sp_step[b];
    return m->sp_gid[a] < m->sp_gid[b];
  });
  for (int64_t k = 0; k < n; ++k) {
    gid[k] = m->sp_gid[idx[k]];
    if (step) step[k] = m->sp_step[idx[k]];
    if (t_interp) t_interp[k] = m->sp_t[idx[k]];
  }
  return CN_OK;
}

int cn_phase_clocks(const cn_model *m, uint64_t *out, int32_t n) {
  if (!m || !out) return fail(CN_E_INVALID, "NULL argument");
  if (n < CN_N_PHASES) return fail(CN_E_INVALID, "out needs CN_N_PHASES entries");
  static_assert(CN_N_PHASES == PH_COUNT, "phase count");
#ifndef CN_PHASE_CLOCKS
  return fail(CN_E_STATE, "this library was built without phase clocks (build with CN_PHASE_CLOCKS)");
#else
  if (m->dry) return fail(CN_E_STATE, "model was built with validate_only");
  if (m->lpc) return fail(CN_E_STATE, "phase clocks cover the level layout's interval kernel only");
  try {
    HIPCHK(hipStreamSynchronize(m->stream));
    HIPCHK(hipMemcpy(out, m->kp.phase_clk, PH_COUNT * sizeof(uint64_t), hipMemcpyDeviceToHost));
  } catch (const Err &e) {
    return fail(e.code, e.msg);
  }
  return CN_OK;
#endif
}

int cn_voltages(const cn_model *m, double *v_out, int64_t n_comp) {
  if (!m || !v_out) return fail(CN_E_INVALID, "NULL argument");
  if (m->dry) return fail(CN_E_STATE, "model was built with validate_only");
  if (n_comp != m->n_comp) return fail(CN_E_INVALID, "n_comp does not match the model");
  try {
    std::vector<double> dv(m->n_dev);
    HIPCHK(hipStreamSynchronize(m->stream));
    HIPCHK(hipMemcpy(dv.data(), m->kp.v, m->n_dev * sizeof(double), hipMemcpyDeviceToHost));
    for (int64_t i = 0; i < m->n_comp; ++i) v_out[i] = dv[m->dev_of_node[i]];
  } catch (const Err &e) {
    return fail(e.code, e.msg);
  }
  return CN_OK;
}

int cn_mech_state(const cn_model *m, int32_t type, int32_t which, double *out, int64_t n) {
  const int rc = mech_state_check(m, type, which, out, n);
  if (rc != CN_OK) return rc;
  double *buf = nullptr;
  if (m->dt_fixed && n > 0) {
    const hipError_t e = hipMalloc(&buf, n * sizeof(double));
    if (e != hipSuccess) return fail(CN_E_NOMEM, std::string("hipMalloc: ") + hipGetErrorString(e));
  }
  const int r = mech_state_run(m, type, which, out, n, buf);
  if (buf) (void)hipFree(buf);
  return r;
}

int cn_restore(cn_model *m, double dt, const cn_checkpoint *ck) {
  if (!m || !ck) return fail(CN_E_INVALID, "NULL argument");
  if (m->broken) return fail(CN_E_STATE, "model is in an error state after a failed run");
  if (m->dry) return fail(CN_E_STATE, "model was built with validate_only");
  if (m->step != 0 || !m->sp_gid.empty()) return fail(CN_E_STATE, "restore needs a model that has not run");
  if (!(dt > 0.0) || !std::isfinite(dt)) return fail(CN_E_INVALID, "bad dt");
  if (m->dt_fixed && dt != m->dt) return fail(CN_E_STATE, "dt differs from the first cn_run call");
  if (ck->step < 0) return fail(CN_E_INVALID, "negative restart step");
  if (!ck->v || !finite_all(ck->v, m->n_comp)) return fail(CN_E_INVALID, "checkpoint potentials missing or non-finite");
  const Table &hh = m->mech[CN_MECH_HH], &km = m->mech[CN_MECH_KM], &ca = m->mech[CN_MECH_CAHI],
              &syn = m->mech[CN_MECH_EXPSYN];
  auto need = [&](const Table &t, const double *x) { return !t.present || t.n == 0 || (x && finite_all(x, t.n)); };
  if (!need(hh, ck->hh_m) || !need(hh, ck->hh_h) || !need(hh, ck->hh_n) || !need(km, ck->km_n) ||
      !need(ca, ck->cahi_m) || !need(ca, ck->cahi_cai) || !need(syn, ck->syn_g))
    return fail(CN_E_INVALID, "checkpoint state of a present mechanism missing or non-finite");
  if (ck->n_spikes < 0 || (ck->n_spikes > 0 && (!ck->spike_gid || !ck->spike_step)))
    return fail(CN_E_INVALID, "checkpoint spike arrays missing");
  for (int64_t q = 0; q < ck->n_spikes; ++q)
    if (ck->spike_gid[q] < 0 || ck->spike_gid[q] >= m->n_cells || ck->spike_step[q] < 0 ||
        ck->spike_step[q] > ck->step)
      return fail(CN_E_INVALID, "checkpoint spike " + std::to_string(q) + " out of range");
  bool touched = false;
  void *tmp_b = nullptr, *tmp_k = nullptr;
  try {
    if (!m->dt_fixed) {
      touched = true;
      prepare_dt(m, dt);
      m->dt = dt;
      m->dt_fixed = true;
    }
    touched = true;
    KParams &p = m->kp;
    const int64_t N = m->n_dev;
    HIPCHK(hipStreamSynchronize(m->stream));
    {
      std::vector<double> dv(N, m->v_init);
      for (int64_t i = 0; i < m->n_comp; ++i) dv[m->dev_of_node[i]] = ck->v[i];
      HIPCHK(hipMemcpy(p.v, dv.data(), N * sizeof(double), hipMemcpyHostToDevice));
    }
    // channel states: the device copy (initial values where a mechanism is absent) with the checkpoint's values
    // written over it; the states are fresh at the restart step (no pending update)
    auto put_states = [&](auto zero) {
      using S = decltype(zero);
      std::vector<StRec<S>> r(N);
      HIPCHK(hipMemcpy(r.data(), p.st, N * sizeof(StRec<S>), hipMemcpyDeviceToHost));
      for (int64_t k = 0; k < hh.n && hh.present; ++k) {
        StRec<S> &x = r[m->dev_of_node[hh.node[k]]];
        x.m = (S)ck->hh_m[k];
        x.h = (S)ck->hh_h[k];
        x.n = (S)ck->hh_n[k];
      }
      for (int64_t k = 0; k < km.n && km.present; ++k) r[m->dev_of_node[km.node[k]]].kn = (S)ck->km_n[k];
      for (int64_t k = 0; k < ca.n && ca.present; ++k) {
        StRec<S> &x = r[m->dev_of_node[ca.node[k]]];
        x.cm = (S)ck->cahi_m[k];
        x.cai = (S)ck->cahi_cai[k];
      }
      HIPCHK(hipMemcpy(p.st, r.data(), N * sizeof(StRec<S>), hipMemcpyHostToDevice));
      std::vector<S> g(syn.n);
      for (int64_t k = 0; k < syn.n; ++k) g[m->dev_of_syn[k]] = (S)ck->syn_g[k];
      if (syn.n) HIPCHK(hipMemcpy(p.syn_g, g.data(), syn.n * sizeof(S), hipMemcpyHostToDevice));
    };
    if (m->fp32) put_states(0.0f);
    else put_states(0.0);
    // events still in flight at the restart step, rebuilt from the spikes that sent them: every NetCon event due at
    // or after the step goes to the ring bucket of its interval and target group
    const int64_t s = ck->step, M = p.M, ival = s / M;
    std::vector<int64_t> bucket;
    std::vector<uint64_t> key;
    for (int64_t q = 0; q < ck->n_spikes; ++q) {
      const int32_t gid = ck->spike_gid[q];
      for (int64_t o = m->host_out_off[gid]; o < m->host_out_off[gid + 1]; ++o) {
        const int32_t nc = m->host_out_nc[o];
        const int64_t due = ck->spike_step[q] + m->host_D[nc];
        if (due < s) continue;  // delivered before the checkpoint
        const int64_t it = due / M;
        if (it - ival >= p.ring) throw Err{CN_E_INVALID, "checkpoint spike beyond the event horizon"};
        const uint64_t k = ((uint64_t)(due - it * M) << EV_STEP_SHIFT) |
                           ((uint64_t)(uint32_t)m->host_tgt_l[nc] << EV_SYN_SHIFT) | EV_KIND_NETCON | (uint32_t)nc;
        bucket.push_back((it % p.ring) * m->n_groups + m->host_tgt_g[nc]);
        key.push_back(k);
      }
    }
    HIPCHK(launch_fill_i32(p.ev_cnt, (int64_t)p.ring * m->n_groups, 0, m->stream));
    HIPCHK(launch_fill_i32(p.flags, 4, 0, m->stream));
    if (!key.empty()) {
      tmp_b = m->dalloc(bucket.size() * sizeof(int64_t));
      tmp_k = m->dalloc(key.size() * sizeof(uint64_t));
      HIPCHK(hipMemcpyAsync(tmp_b, bucket.data(), bucket.size() * sizeof(int64_t), hipMemcpyHostToDevice, m->stream));
      HIPCHK(hipMemcpyAsync(tmp_k, key.data(), key.size() * sizeof(uint64_t), hipMemcpyHostToDevice, m->stream));
      HIPCHK(launch_insert_events(p.ev_cnt, p.ev_key, p.ev_cap, (int64_t)key.size(), static_cast<int64_t *>(tmp_b),
                                  static_cast<uint64_t *>(tmp_k), p.flags, m->stream));
    }
    HIPCHK(hipStreamSynchronize(m->stream));
    if (tmp_b) m->dfree(tmp_b);
    if (tmp_k) m->dfree(tmp_k);
    tmp_b = tmp_k = nullptr;
    int32_t flags[4];
    HIPCHK(hipMemcpy(flags, p.flags, sizeof flags, hipMemcpyDeviceToHost));
    if (flags[FLAG_EV_OVERFLOW]) throw Err{CN_E_CAPACITY, "event ring overflow: raise cn_options.event_capacity"};
    m->step = s;
    m->fresh_step = s;
  } catch (const Err &e) {
    if (touched) m->broken = true;
    return fail(e.code, e.msg);
  } catch (const std::bad_alloc &) {
    if (touched) m->broken = true;
    return fail(CN_E_NOMEM, "out of host memory");
  } catch (...) {
    if (touched) m->broken = true;
    return fail(CN_E_DEVICE, "unexpected failure in cn_restore");
  }
  return CN_OK;
}

int cn_set_seed(cn_model *m, uint64_t seed) {
  if (!m) return fail(CN_E_INVALID, "model is NULL");
  m->seed = seed;
  return CN_OK;
}

}  // extern "C"

namespace {

std::mutex g_tune_mu;
std::map<uint64_t, cn_tune_result> g_tune_cache;

// FNV-1a over the facts that decide the best group shape
struct Fnv {
  uint64_t h = 1469598103934665603ull;
  void add(const void *p, size_t n) {
    const unsigned char *c = static_cast<const unsigned char *>(p);
    for (size_t i = 0; i < n; ++i) h = (h ^ c[i]) * 1099511628211ull;
  }
  template <typename T>
  void put(T x) { add(&x, sizeof x); }
};

uint64_t tune_signature(const cn_topology *topo, const cn_mech_table *mechs, int32_t n_mechs, const cn_network *net,
                        const cn_options *opt, double dt, int64_t max_joined) {
  Fnv f;
  f.put(max_joined);  // compartments of the largest set of cells joined by gap junctions
  f.put(topo->n_cells);
  f.put(topo->n_comp);
  // cell sizes in quarter-octave bins
  int64_t hist[128] = {};
  for (int32_t c = 0; c < topo->n_cells; ++c) {
    const double n = (double)(topo->cell_offset[c + 1] - topo->cell_offset[c]);
    hist[std::min<int>(127, (int)std::floor(4.0 * std::log2(std::max(1.0, n))))]++;
  }
  f.add(hist, sizeof hist);
  for (int32_t k = 0; k < n_mechs; ++k) {
    f.put(mechs[k].type);
    f.put(mechs[k].n);
    f.put((int32_t)(mechs[k].node == nullptr));
  }
  f.put(net ? net->n_netcon : (int64_t)0);
  f.put(net ? net->poisson_rate_hz : 0.0);
  f.put(net ? net->n_gap : (int64_t)0);
  f.put(opt ? opt->precision : 0);
  f.put(opt ? opt->layout : 0);
  f.put(opt ? opt->event_capacity : 0);
  f.put(opt ? opt->max_interval : 0);
  f.put(dt);
  return f.h;
}

// median interval-kernel time of one shape (ms), or a negative value when the shape cannot run this model
double time_shape(const cn_topology *topo, const cn_mech_table *mechs, int32_t n_mechs, const cn_network *net,
                  cn_options o, double dt, int layout, int T, int K, int fill, int *err, std::string *msg) {
  o.layout = layout;
  o.group_threads = T;
  o.group_slots = K;
  o.group_fill_pct = fill;
  o.timing = 1;
  o.validate_only = 0;
  o.fault_inject = 0;
  cn_model *m = nullptr;
  int rc = cn_model_create(topo, mechs, n_mechs, net, &o, &m);
  if (rc == CN_OK) rc = cn_run(m, dt, dt);  // fixes dt and captures the interval graph
  std::vector<double> ms;
  if (rc == CN_OK) {
    const int64_t M = m->kp.M;
    rc = cn_run(m, (double)M * dt, dt);  // warm-up: the rest of the first interval
    for (int r = 0; rc == CN_OK && r < 5; ++r) {
      const double before = m->kernel_ms;
      rc = cn_run(m, (double)((2 + r) * M) * dt, dt);
      if (rc == CN_OK) ms.push_back(m->kernel_ms - before);
    }
  }
  if (rc != CN_OK) {
    *err = rc;
    *msg = g_err;
  }
  cn_model_destroy(m);
  if (rc != CN_OK || ms.empty()) return -1.0;
  std::sort(ms.begin(), ms.end());
  return ms[ms.size() / 2];
}

}  // namespace

extern "C" {

int cn_autotune(const cn_topology *topo, const cn_mech_table *mechs, int32_t n_mechs, const cn_network *net,
                const cn_options *opt, double dt, double budget_ms, cn_tune_result *out) {
  if (!topo || !out) return fail(CN_E_INVALID, "NULL argument");
  if (!(dt > 0.0) || !std::isfinite(dt)) return fail(CN_E_INVALID, "bad dt");
  if (topo->n_cells <= 0 || !topo->cell_offset) return fail(CN_E_INVALID, "empty model");
  if (opt && opt->validate_only) return fail(CN_E_STATE, "autotuning needs a device");
  for (int32_t c = 0; c < topo->n_cells; ++c)
    if (topo->cell_offset[c + 1] <= topo->cell_offset[c]) return fail(CN_E_INVALID, "cell_offset must be strictly increasing");
  if (topo->cell_offset[0] != 0 || topo->cell_offset[topo->n_cells] != topo->n_comp)
    return fail(CN_E_INVALID, "cell_offset must run from 0 to n_comp");
  cn_options base{};
  if (opt) base = *opt;
  int32_t max_cell = 0;
  for (int32_t c = 0; c < topo->n_cells; ++c)
    max_cell = std::max<int32_t>(max_cell, (int32_t)(topo->cell_offset[c + 1] - topo->cell_offset[c]));
  {
    std::vector<int32_t> cl;
    const int64_t u = join_cells(topo->cell_offset, topo->n_cells, topo->n_comp, net ? net->n_gap : 0,
                                 net ? net->gap_node : nullptr, net ? net->gap_partner : nullptr, cl);
    max_cell = (int32_t)std::min<int64_t>(std::max<int64_t>(max_cell, u), INT32_MAX);
  }
  const uint64_t sig = tune_signature(topo, mechs, n_mechs, net, &base, dt, max_cell);
  {
    std::lock_guard<std::mutex> lock(g_tune_mu);
    auto it = g_tune_cache.find(sig);
    if (it != g_tune_cache.end()) {
      *out = it->second;
      out->from_cache = 1;
      out->n_candidates = 0;
      return CN_OK;
    }
  }
  int dT = 0, dK = 0;
  default_shape(topo->n_comp, max_cell, base.precision == CN_PREC_FP32_MECH, dT, dK);
  // candidates: the default first; for each thread count, the smallest slot count that holds the largest cell and
  // twice that; then the best of these with a 90 % packing fill
  const int L = CN_LAYOUT_LEVEL;
  std::vector<std::array<int, 4>> cand{{L, dT, dK, 100}};
  for (int T : {128, 256, 512, 1024}) {
    int K = 0;
    for (int k : {1, 2, 4, 8})
      if (shape_compiled(T, k) && T * k >= max_cell) {
        K = k;
        break;
      }
    if (!K) continue;
    for (int k : {K, 2 * K}) {
      if (!shape_compiled(T, k)) continue;
      const std::array<int, 4> c{L, T, k, 100};
      if (std::find(cand.begin(), cand.end(), c) == cand.end()) cand.push_back(c);
    }
  }
  if (base.layout == CN_LAYOUT_AUTO) cand.push_back({CN_LAYOUT_INTERLEAVED, 0, 0, 100});
  if (base.layout == CN_LAYOUT_INTERLEAVED) cand = {{CN_LAYOUT_INTERLEAVED, 0, 0, 100}};
  cn_tune_result r{};
  r.signature = sig;
  r.default_threads = dT;
  r.default_slots = dK;
  const auto t0 = std::chrono::steady_clock::now();
  auto elapsed_ms = [&]() {
    return std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
  };
  int best = -1;
  double best_ms = 0.0;
  auto try_shape = [&](const std::array<int, 4> &c) -> int {
    int err = CN_OK;
    std::string msg;
    const double ms = time_shape(topo, mechs, n_mechs, net, base, dt, c[0], c[1], c[2], c[3], &err, &msg);
    if (ms < 0.0) return err;
    const int i = r.n_candidates++;
    r.cand_layout[i] = c[0];
    r.cand_threads[i] = c[1];
    r.cand_slots[i] = c[2];
    r.cand_fill[i] = c[3];
    r.cand_ms[i] = ms;
    if (best < 0 || ms < best_ms) {
      best = i;
      best_ms = ms;
    }
    return CN_OK;
  };
  const int rc0 = try_shape(cand[0]);
  if (rc0 != CN_OK || r.n_candidates == 0) {
    const std::string msg = g_err;
    return fail(rc0 != CN_OK ? rc0 : CN_E_DEVICE, "autotune: the default shape failed: " + msg);
  }
  r.default_ms = r.cand_ms[0];
  for (size_t k = 1; k < cand.size() && r.n_candidates < CN_TUNE_MAX_CANDIDATES - 1; ++k) {
    if (r.n_candidates >= 2 && elapsed_ms() > budget_ms) break;
    (void)try_shape(cand[k]);
  }
  if (r.cand_layout[best] == L && (elapsed_ms() <= budget_ms || r.n_candidates < 2)) {
    const std::array<int, 4> c{L, r.cand_threads[best], r.cand_slots[best], 90};
    (void)try_shape(c);
  }
  r.layout = r.cand_layout[best];
  r.group_threads = r.cand_threads[best];
  r.group_slots = r.cand_slots[best];
  r.group_fill_pct = r.cand_fill[best];
  r.interval_ms = best_ms;
  {
    std::lock_guard<std::mutex> lock(g_tune_mu);
    g_tune_cache[sig] = r;
  }
  *out = r;
  return CN_OK;
}

int cn_model_info(const cn_model *m, cn_info *o) {
  if (!m || !o) return fail(CN_E_INVALID, "NULL argument");
  std::memset(o, 0, sizeof *o);
  o->n_comp = m->n_comp;
  o->n_syn = m->n_syn;
  o->n_netcon = m->n_nc;
  o->n_groups = m->n_groups;
  o->step = m->step;
  o->device_bytes = m->device_bytes;
  o->n_cells = m->n_cells;
  o->interval_steps = m->dt_fixed ? m->kp.M : 0;
  o->group_threads = m->threads;
  o->group_slots = m->slots;
  o->max_group_nodes = m->max_group_nodes;
  o->max_levels = m->max_levels;
  o->ring_slots = m->dt_fixed ? m->kp.ring : 0;
  o->event_capacity = m->dt_fixed ? m->kp.ev_cap : 0;
  o->precision = m->fp32 ? CN_PREC_FP32_MECH : CN_PREC_FP64;
  o->lds_bytes = m->lds_bytes;
  o->dt = m->dt;
  o->layout = m->lpc ? CN_LAYOUT_INTERLEAVED : CN_LAYOUT_LEVEL;
  o->groups_per_cu = m->dt_fixed ? m->groups_per_cu : 0;
  return CN_OK;
}

int cn_stats(const cn_model *m, double *kernel_ms, int64_t *kernel_launches) {
  if (!m) return fail(CN_E_INVALID, "model is NULL");
  if (kernel_ms) *kernel_ms = m->kernel_ms;
  if (kernel_launches) *kernel_launches = m->kernel_launches;
  return CN_OK;
}

void cn_model_destroy(cn_model *m) { delete m; }

}  // extern "C"
