// The library handle (pgo_graph) and the host helpers that the host
// translation units share: error reporting, device allocation owned by the
// handle, and the typed device views the kernels take.  Nothing here is
// part of the C ABI.
#pragma once
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <numeric>
#include <string>
#include <vector>

#include "internal.hpp"
#include "pgo.h"

struct pgo_graph {
  int device = 0;
  hipStream_t own_stream = nullptr;
  hipStream_t stream = nullptr;
  pgo_options opt{};
  bool chordal = false;             // PGO_MODEL_CHORDAL
  bool aniso = false;               // PGO_MODEL_QUAT_INFO
  double* S9 = nullptr;             // information model: S_e per edge, caller order (m x 9)
  // The prepared FP64 edges again in out-order (by tail, caller order among
  // equal tails) for the reductions, whose gathers of the tail's state then
  // run through it in order; X9 is R9 (chordal) or S9 (information model).
  int32_t *r_ei = nullptr, *r_ej = nullptr;
  pgo::Q4<double>* r_qe = nullptr;
  double *r_tm = nullptr, *r_kappa = nullptr, *r_tau = nullptr, *r_X9 = nullptr;
  void *o_Sa = nullptr, *o_Sb = nullptr, *i_Sa = nullptr, *i_Sb = nullptr;
  int64_t n = 0, m = 0;
  int32_t G = 0;
  int32_t max_n = 0;
  std::vector<void*> allocs;
  std::vector<int64_t> voff_h, eoff_h;
  int32_t* voff32 = nullptr;
  int32_t* order = nullptr;
  int32_t* gid = nullptr;           // graph of each vertex
  double* beta_dev = nullptr;       // per-graph penalties of the last pgo_iterate_graphs
  std::vector<double> beta_h;       // penalty of each graph in the last iterate call
  std::vector<double> wbar_h;       // mean vertex weight of each graph (merit noise scale)
  double last_gamma = 1.0;
  int32_t* active_dev = nullptr;    // per-graph run flags (pgo_solve)
  int32_t* done_dev = nullptr;      // per-graph sweeps run (pgo_iterate_until)
  int32_t* flag_dev = nullptr;      // per-graph restore flags (pgo_solve)
  void* snap[6] = {nullptr, nullptr, nullptr, nullptr, nullptr, nullptr};
  // differentiation
  pgo::Q4<double>* qe0 = nullptr;        // prepared, sign-aligned edge quaternions of create
  double* omega = nullptr;          // current right perturbation of each measured rotation
  double* t0dev = nullptr;          // initial translations (for pgo_reset_state)
  int32_t *pos_out = nullptr, *pos_in = nullptr, *in2out = nullptr, *out2in = nullptr;
  std::vector<void*> sets;          // state sets: checkpoints, then segment snapshots
  int32_t rec_K = -1, rec_C = 0;
  int64_t rec_id = 0;               // count of pgo_forward_record calls on the handle
  double rec_beta = 0, rec_gamma = 0;
  void* adj[14] = {};               // vertex adjoints (6) and edge messages (8)
  void* gacc[4] = {};               // FP64 edge-gradient accumulators
  double* cgrad = nullptr;          // 3 x n FP64 vertex-constant adjoints
  int32_t *o_ptr = nullptr, *o_nbr = nullptr, *o_perm = nullptr;
  int32_t *i_ptr = nullptr, *i_nbr = nullptr, *i_perm = nullptr;
  void *o_tt = nullptr, *o_w = nullptr, *i_tt = nullptr, *i_w = nullptr;
  void *cQ = nullptr, *cT = nullptr, *cS = nullptr;
  void *p = nullptr, *q = nullptr, *lam = nullptr, *t = nullptr, *s = nullptr, *z = nullptr;
  void *xy = nullptr, *xm = nullptr;  // sweep scratch slot (quaternion models)
  unsigned* coop_bar = nullptr;       // barrier counter of the cooperative schedule
  void *q_prev = nullptr, *lam_prev = nullptr, *t_prev = nullptr, *s_prev = nullptr,
       *z_prev = nullptr;
  int32_t *ei = nullptr, *ej = nullptr;
  pgo::Q4<double>* qe = nullptr;
  double *tm = nullptr, *kappa = nullptr, *tau = nullptr;
  pgo::Q4<double>* p0 = nullptr;
  double* R9 = nullptr;             // chordal: projected measured rotations, caller order (m x 9)
  double* P0 = nullptr;             // chordal: projected initial rotations (n x 9)
  int n_ech = 0, n_vch = 0;
  int64_t *ec_beg = nullptr, *ec_end = nullptr, *vc_beg = nullptr, *vc_end = nullptr;
  int32_t *g_ec_off = nullptr, *g_vc_off = nullptr;
  int32_t *ec_gid = nullptr, *vc_gid = nullptr;  // graph of each reduction chunk
  double *part_e = nullptr, *part_v = nullptr, *red_out = nullptr;
  double* iobuf = nullptr;  // n x state width doubles, allocated on first use
  int sched = PGO_SCHED_PHASE;
  int block_phase = 256;  // per-phase and cooperative schedules
  int block_graph = 256;
  int graph_lds = 1;  // per-graph kernels keep each graph's state in LDS as far as it fits
  bool have_prev = false;
  // captured launch sequence of the per-phase schedule
  hipGraphExec_t gexec = nullptr;
  int g_k = -1, g_block = -1;
  double g_beta = 0, g_gamma = 0;
  bool g_per_graph = false;
  bool g_masked = false;
};


namespace pgo {
namespace host {

pgo_status fail(pgo_status s, const std::string& msg);
pgo_status hip_fail(hipError_t e, const char* what);
const char* last_error();

#define HIPCHK(expr)                                                    \
  do {                                                                  \
    hipError_t e_ = (expr);                                             \
    if (e_ != hipSuccess) return ::pgo::host::hip_fail(e_, #expr);      \
  } while (0)

constexpr int64_t kChunk = 8192;  // items per reduction chunk

template <typename X>
pgo_status dalloc(pgo_graph* g, X** ptr, size_t count) {
  *ptr = nullptr;
  if (count == 0) count = 1;
  void* raw = nullptr;
  hipError_t e = hipMalloc(&raw, count * sizeof(X));
  if (e != hipSuccess) return hip_fail(e, "hipMalloc");
  g->allocs.push_back(raw);
  *ptr = static_cast<X*>(raw);
  return PGO_OK;
}

pgo_status dalloc_bytes(pgo_graph* g, void** ptr, size_t bytes);
void dfree(pgo_graph* g, void* ptr);

template <typename X>
pgo_status upload(pgo_graph* g, X** dst, const X* src, size_t count) {
  pgo_status s = dalloc(g, dst, count);
  if (s != PGO_OK) return s;
  if (count) HIPCHK(hipMemcpyAsync(*dst, src, count * sizeof(X), hipMemcpyHostToDevice, g->stream));
  return PGO_OK;
}

template <typename T>
DevGraph<T> view(const pgo_graph* g) {
  DevGraph<T> d;
  d.n = int32_t(g->n);
  d.gid = g->gid;
  d.o_ptr = g->o_ptr;
  d.o_nbr = g->o_nbr;
  d.o_tt = static_cast<const P4<T>*>(g->o_tt);
  d.o_w = static_cast<const Q4<T>*>(g->o_w);
  d.i_ptr = g->i_ptr;
  d.i_nbr = g->i_nbr;
  d.i_tt = static_cast<const P4<T>*>(g->i_tt);
  d.i_w = static_cast<const Q4<T>*>(g->i_w);
  d.cQ = static_cast<const T*>(g->cQ);
  d.cT = static_cast<const T*>(g->cT);
  d.cS = static_cast<const T*>(g->cS);
  d.p = static_cast<Q4<T>*>(g->p);
  d.q = static_cast<Q4<T>*>(g->q);
  d.lam = static_cast<Q4<T>*>(g->lam);
  d.t = static_cast<V3<T>*>(g->t);
  d.s = static_cast<V3<T>*>(g->s);
  d.z = static_cast<V3<T>*>(g->z);
  d.xy = static_cast<Q4<T>*>(g->xy);
  d.xm = static_cast<T*>(g->xm);
  d.q_prev = static_cast<Q4<T>*>(g->q_prev);
  d.lam_prev = static_cast<Q4<T>*>(g->lam_prev);
  d.t_prev = static_cast<V3<T>*>(g->t_prev);
  d.s_prev = static_cast<V3<T>*>(g->s_prev);
  d.z_prev = static_cast<V3<T>*>(g->z_prev);
  return d;
}

template <typename T>
DevChordal<T> viewc(const pgo_graph* g) {
  DevChordal<T> d;
  d.n = int32_t(g->n);
  d.gid = g->gid;
  d.o_ptr = g->o_ptr;
  d.o_nbr = g->o_nbr;
  d.o_tt = static_cast<const P4<T>*>(g->o_tt);
  d.o_R = static_cast<const R3<T>*>(g->o_w);
  d.i_ptr = g->i_ptr;
  d.i_nbr = g->i_nbr;
  d.i_tt = static_cast<const P4<T>*>(g->i_tt);
  d.i_R = static_cast<const R3<T>*>(g->i_w);
  d.cQ = static_cast<const T*>(g->cQ);
  d.P = static_cast<R3<T>*>(g->p);
  d.Q = static_cast<R3<T>*>(g->q);
  d.L = static_cast<R3<T>*>(g->lam);
  d.t = static_cast<V3<T>*>(g->t);
  d.s = static_cast<V3<T>*>(g->s);
  d.z = static_cast<V3<T>*>(g->z);
  d.Q_prev = static_cast<R3<T>*>(g->q_prev);
  d.L_prev = static_cast<R3<T>*>(g->lam_prev);
  d.t_prev = static_cast<V3<T>*>(g->t_prev);
  d.s_prev = static_cast<V3<T>*>(g->s_prev);
  d.z_prev = static_cast<V3<T>*>(g->z_prev);
  return d;
}

template <typename T>
DevAniso<T> viewa(const pgo_graph* g) {
  return DevAniso<T>{view<T>(g),
                     static_cast<const V3<T>*>(g->o_Sa), static_cast<const V3<T>*>(g->o_Sb),
                     static_cast<const V3<T>*>(g->i_Sa), static_cast<const V3<T>*>(g->i_Sb)};
}

// words of T per vertex of a rotation-like block (p, q, lambda and edge w)
inline int rot_words(const pgo_graph* g) { return g->chordal ? 9 : 4; }
inline int state_width(const pgo_graph* g) { return g->chordal ? 36 : 21; }

bool finite_all(const double* a, size_t k);
// index of the first nonzero of count device flags, -1 if none (synchronises)
pgo_status first_bad(pgo_graph* g, const uint8_t* flags_dev, int64_t count, int64_t* idx);

// run.cpp: k sweeps in the given schedule and block size, one penalty per
// handle or per graph (beta_g, host array), graphs masked by active (host);
// snap_in_launch: the per-graph kernel copies each running graph's state to
// the snapshot arrays before its first sweep (quaternion model only)
pgo_status iterate_with(pgo_graph* g, int32_t k, double beta, double gamma, int sched, int block,
                        const double* beta_g = nullptr, const int32_t* active = nullptr,
                        bool snap_in_launch = false);
// the workgroup size of the handle's current schedule
inline int current_block(const pgo_graph* g) {
  return g->sched == PGO_SCHED_GRAPH ? g->block_graph : g->block_phase;
}
// bytes per vertex of the six state arrays (p, q, lambda, t, s, z)
void state_array_bytes(const pgo_graph* g, size_t out[6]);

// evaluate.cpp
pgo_status reduce(pgo_graph* g, std::vector<double>& out, bool allow_nonfinite = false,
                  const int32_t* active = nullptr);
bool finite_graph(const std::vector<double>& r, int32_t j);
void merit_of(const double* v, double beta, double gamma, double* L, double* psi);

// The out-ordered FP64 edges of the reductions from the caller-ordered ones
// (allocated on the first call).
pgo_status reduction_edges(pgo_graph* g);

// The sweep kernels' edge records and per-vertex constants, again from the
// prepared FP64 edges (after the edge parameters or signs changed), and the
// reductions' copy of those edges.
template <typename T>
pgo_status refill_edges(pgo_graph* g) {
  hipStream_t st = g->stream;
  HIPCHK(launch_fill_edges<T>(g->o_perm, g->ej, g->qe, g->tm, g->kappa, g->tau, g->m, g->o_nbr,
                              static_cast<P4<T>*>(g->o_tt), static_cast<Q4<T>*>(g->o_w), st));
  HIPCHK(launch_fill_edges<T>(g->i_perm, g->ei, g->qe, g->tm, g->kappa, g->tau, g->m, g->i_nbr,
                              static_cast<P4<T>*>(g->i_tt), static_cast<Q4<T>*>(g->i_w), st));
  HIPCHK(launch_vertex_consts<T>(int32_t(g->n), g->o_ptr, g->o_perm, g->i_ptr, g->i_perm, g->tm,
                                 g->kappa, g->tau, static_cast<T*>(g->cQ),
                                 static_cast<T*>(g->cT), static_cast<T*>(g->cS), st));
  if (g->aniso) {  // edge records (t~, c) and the information matrices
    HIPCHK(launch_fill_edges_a<T>(g->o_perm, g->tm, g->S9, g->m, static_cast<P4<T>*>(g->o_tt),
                                  static_cast<V3<T>*>(g->o_Sa), static_cast<V3<T>*>(g->o_Sb), st));
    HIPCHK(launch_fill_edges_a<T>(g->i_perm, g->tm, g->S9, g->m, static_cast<P4<T>*>(g->i_tt),
                                  static_cast<V3<T>*>(g->i_Sa), static_cast<V3<T>*>(g->i_Sb), st));
  }
  return reduction_edges(g);
}

// state.cpp
pgo_status ensure_iobuf(pgo_graph* g);
hipError_t state_io(pgo_graph* g, double* buf, int to_device);
pgo_status quaternion_only(pgo_graph* g, const char* what);

}  // namespace host
}  // namespace pgo
