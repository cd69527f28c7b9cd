// Host side of the C ABI declared in include/pgo.h: argument checking,
// device memory ownership, the boundary preparation sequence, schedule
// selection, the autotuner and the host<->device transfers.  All arithmetic
// of the method runs in the kernels of sweep.hip (quaternion model),
// chordal.hip (rotation-matrix model), prep.hip, reduce.hip and adjoint.hip.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <numeric>
#include <string>
#include <vector>

#include "internal.hpp"
#include "pgo.h"

using namespace pgo;

namespace {

thread_local std::string g_err;

pgo_status fail(pgo_status s, const std::string& msg) {
  g_err = msg;
  return s;
}

pgo_status hip_fail(hipError_t e, const char* what) {
  return fail(e == hipErrorOutOfMemory ? PGO_ENOMEM : PGO_EDEVICE,
              std::string(what) + ": " + hipGetErrorString(e));
}

#define HIPCHK(expr)                                   \
  do {                                                 \
    hipError_t e_ = (expr);                            \
    if (e_ != hipSuccess) return hip_fail(e_, #expr);  \
  } while (0)

constexpr int64_t kChunk = 8192;  // items per reduction chunk

}  // namespace

struct pgo_graph {
  int device = 0;
  hipStream_t own_stream = nullptr;
  hipStream_t stream = nullptr;
  pgo_options opt{};
  bool chordal = false;             // PGO_MODEL_CHORDAL
  bool aniso = false;               // PGO_MODEL_QUAT_INFO
  double* S9 = nullptr;             // information model: S_e per edge, caller order (m x 9)
  void *o_Sa = nullptr, *o_Sb = nullptr, *i_Sa = nullptr, *i_Sb = nullptr;
  void *cTa = nullptr, *cTb = nullptr, *cSa = nullptr, *cSb = nullptr;
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
  Q4<double>* qe0 = nullptr;        // prepared, sign-aligned edge quaternions of create
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
  Q4<double>* qe = nullptr;
  double *tm = nullptr, *kappa = nullptr, *tau = nullptr;
  Q4<double>* p0 = nullptr;
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

namespace {

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

pgo_status dalloc_bytes(pgo_graph* g, void** ptr, size_t bytes) {
  return dalloc<uint8_t>(g, reinterpret_cast<uint8_t**>(ptr), bytes);
}

void dfree(pgo_graph* g, void* ptr) {
  if (!ptr) return;
  auto it = std::find(g->allocs.begin(), g->allocs.end(), ptr);
  if (it != g->allocs.end()) {
    (void)hipFree(ptr);
    g->allocs.erase(it);
  }
}

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
  d.cT = static_cast<const T*>(g->cT);
  d.cS = static_cast<const T*>(g->cS);
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
                     static_cast<const V3<T>*>(g->i_Sa), static_cast<const V3<T>*>(g->i_Sb),
                     static_cast<const V3<T>*>(g->cTa), static_cast<const V3<T>*>(g->cTb),
                     static_cast<const V3<T>*>(g->cSa), static_cast<const V3<T>*>(g->cSb)};
}

// words of T per vertex of a rotation-like block (p, q, lambda and edge w)
int rot_words(const pgo_graph* g) { return g->chordal ? 9 : 4; }
int state_width(const pgo_graph* g) { return g->chordal ? 36 : 21; }

bool finite_all(const double* a, size_t k) {
  for (size_t i = 0; i < k; ++i)
    if (!std::isfinite(a[i])) return false;
  return true;
}

pgo_status check_options(const pgo_options& o) {
  const double h[4] = {o.h1, o.h2, o.h3, o.h4};
  for (int k = 0; k < 4; ++k)
    if (!(std::isfinite(h[k]) && h[k] > 0.0))
      return fail(PGO_EINVAL, "proximal weights h1..h4 must be finite and > 0");
  if (o.precision != PGO_FP64 && o.precision != PGO_FP32)
    return fail(PGO_EINVAL, "precision must be PGO_FP64 or PGO_FP32");
  if (o.schedule < PGO_SCHED_AUTO || o.schedule > PGO_SCHED_COOP)
    return fail(PGO_EINVAL, "unknown schedule");
  if (o.schedule == PGO_SCHED_COOP && o.model != PGO_MODEL_QUAT)
    return fail(PGO_EINVAL, "the cooperative schedule runs the quaternion model only");
  if (o.block != 0 && (o.block < 64 || o.block > 1024 || o.block % 64 != 0))
    return fail(PGO_EINVAL, "block must be 0 or a multiple of 64 in [64, 1024]");
  if (o.model != PGO_MODEL_QUAT && o.model != PGO_MODEL_CHORDAL && o.model != PGO_MODEL_QUAT_INFO)
    return fail(PGO_EINVAL, "model must be PGO_MODEL_QUAT, PGO_MODEL_CHORDAL or PGO_MODEL_QUAT_INFO");
  if (o.model == PGO_MODEL_QUAT_INFO && o.block > (o.schedule == PGO_SCHED_GRAPH ? 512 : 256))
    return fail(PGO_EINVAL,
                "the information model runs at most 256 threads per workgroup (512 in the "
                "per-graph schedule)");
  return PGO_OK;
}

// Validates everything that can be checked on the host.  Rotations are
// checked on the device during preparation.
pgo_status check_inputs(int32_t G, const int64_t* voff, const int64_t* eoff, const double* R0,
                        const double* t0, const int32_t* ei, const int32_t* ej, const double* Rm,
                        const double* tm, const double* kappa, const double* tau) {
  if (G < 1) return fail(PGO_EINVAL, "need at least one graph");
  if (voff[0] != 0 || eoff[0] != 0) return fail(PGO_EINVAL, "voff[0] and eoff[0] must be 0");
  for (int32_t g = 0; g < G; ++g) {
    if (voff[g + 1] - voff[g] < 1)
      return fail(PGO_EINVAL, "graph " + std::to_string(g) + " has no pose (n >= 1 required)");
    if (eoff[g + 1] < eoff[g])
      return fail(PGO_EINVAL, "eoff must be nondecreasing (graph " + std::to_string(g) + ")");
  }
  const int64_t n = voff[G], m = eoff[G];
  if (n >= INT32_MAX) return fail(PGO_EINVAL, "too many poses (n must be < 2^31 - 1)");
  if (m >= INT32_MAX) return fail(PGO_EINVAL, "too many edges (m must be < 2^31 - 1)");
  if (m > 0 && (!ei || !ej || !Rm || !tm || !kappa || !tau))
    return fail(PGO_EINVAL, "edge arrays must not be NULL");
  if (!R0 || !t0) return fail(PGO_EINVAL, "R0 and t0 must not be NULL");
  if (!finite_all(R0, size_t(9 * n)) || !finite_all(t0, size_t(3 * n)))
    return fail(PGO_EINVAL, "initial poses contain a non-finite value");
  if (m > 0 && (!finite_all(Rm, size_t(9 * m)) || !finite_all(tm, size_t(3 * m))))
    return fail(PGO_EINVAL, "measurements contain a non-finite value");
  for (int32_t g = 0; g < G; ++g) {
    const int64_t ng = voff[g + 1] - voff[g];
    for (int64_t e = eoff[g]; e < eoff[g + 1]; ++e) {
      if (ei[e] < 0 || ei[e] >= ng || ej[e] < 0 || ej[e] >= ng)
        return fail(PGO_EINVAL, "edge " + std::to_string(e) + " has an index out of range");
      if (ei[e] == ej[e]) return fail(PGO_EINVAL, "edge " + std::to_string(e) + " is a self-loop");
      if (!(std::isfinite(kappa[e]) && kappa[e] > 0.0) || !(std::isfinite(tau[e]) && tau[e] > 0.0))
        return fail(PGO_EINVAL, "edge " + std::to_string(e) + " has kappa or tau not finite and > 0");
    }
  }
  return PGO_OK;
}

pgo_status build_chunks(pgo_graph* g) {
  std::vector<int64_t> eb, ee, vb, ve;
  std::vector<int32_t> goe(g->G + 1, 0), gov(g->G + 1, 0), egid, vgid;
  for (int32_t k = 0; k < g->G; ++k) {
    for (int64_t a = g->eoff_h[k]; a < g->eoff_h[k + 1]; a += kChunk) {
      eb.push_back(a);
      ee.push_back(std::min(a + kChunk, g->eoff_h[k + 1]));
      egid.push_back(k);
    }
    goe[k + 1] = int32_t(eb.size());
    for (int64_t a = g->voff_h[k]; a < g->voff_h[k + 1]; a += kChunk) {
      vb.push_back(a);
      ve.push_back(std::min(a + kChunk, g->voff_h[k + 1]));
      vgid.push_back(k);
    }
    gov[k + 1] = int32_t(vb.size());
  }
  g->n_ech = int(eb.size());
  g->n_vch = int(vb.size());
  pgo_status s;
  if ((s = upload(g, &g->ec_beg, eb.data(), eb.size())) != PGO_OK) return s;
  if ((s = upload(g, &g->ec_end, ee.data(), ee.size())) != PGO_OK) return s;
  if ((s = upload(g, &g->vc_beg, vb.data(), vb.size())) != PGO_OK) return s;
  if ((s = upload(g, &g->vc_end, ve.data(), ve.size())) != PGO_OK) return s;
  if ((s = upload(g, &g->g_ec_off, goe.data(), goe.size())) != PGO_OK) return s;
  if ((s = upload(g, &g->g_vc_off, gov.data(), gov.size())) != PGO_OK) return s;
  if ((s = upload(g, &g->ec_gid, egid.data(), egid.size())) != PGO_OK) return s;
  if ((s = upload(g, &g->vc_gid, vgid.data(), vgid.size())) != PGO_OK) return s;
  if ((s = dalloc(g, &g->part_e, size_t(kEdgeVals) * std::max(1, g->n_ech))) != PGO_OK) return s;
  if ((s = dalloc(g, &g->part_v, size_t(kVertVals) * std::max(1, g->n_vch))) != PGO_OK) return s;
  if ((s = dalloc(g, &g->red_out, size_t(kRedVals) * g->G)) != PGO_OK) return s;
  return PGO_OK;
}

template <typename T>
pgo_status alloc_precision(pgo_graph* g) {
  const size_t n = size_t(g->n), m = size_t(g->m), rw = size_t(rot_words(g));
  pgo_status s;
  void** rot[] = {&g->p, &g->q, &g->lam, &g->q_prev, &g->lam_prev};
  for (void** v : rot)
    if ((s = dalloc_bytes(g, v, rw * sizeof(T) * n)) != PGO_OK) return s;
  void** vec3[] = {&g->t, &g->s, &g->z, &g->t_prev, &g->s_prev, &g->z_prev};
  for (void** v : vec3)
    if ((s = dalloc_bytes(g, v, 3 * sizeof(T) * n)) != PGO_OK) return s;
  void** e4[] = {&g->o_tt, &g->i_tt};
  for (void** v : e4)
    if ((s = dalloc_bytes(g, v, 4 * sizeof(T) * m)) != PGO_OK) return s;
  void** ew[] = {&g->o_w, &g->i_w};
  for (void** v : ew)
    if ((s = dalloc_bytes(g, v, rw * sizeof(T) * m)) != PGO_OK) return s;
  if (!g->chordal) {
    if ((s = dalloc_bytes(g, &g->xy, 4 * sizeof(T) * n)) != PGO_OK) return s;
    if ((s = dalloc_bytes(g, &g->xm, sizeof(T) * n)) != PGO_OK) return s;
  }
  if (!g->chordal && !g->aniso) {
    if ((s = dalloc(g, &g->coop_bar, 64)) != PGO_OK) return s;
    HIPCHK(hipMemsetAsync(g->coop_bar, 0, 64 * sizeof(unsigned), g->stream));
  }
  void** c1[] = {&g->cQ, &g->cT, &g->cS};
  for (void** v : c1)
    if ((s = dalloc_bytes(g, v, sizeof(T) * n)) != PGO_OK) return s;
  if (g->aniso) {
    void** es[] = {&g->o_Sa, &g->o_Sb, &g->i_Sa, &g->i_Sb};
    for (void** v : es)
      if ((s = dalloc_bytes(g, v, 3 * sizeof(T) * m)) != PGO_OK) return s;
    void** vs[] = {&g->cTa, &g->cTb, &g->cSa, &g->cSb};
    for (void** v : vs)
      if ((s = dalloc_bytes(g, v, 3 * sizeof(T) * n)) != PGO_OK) return s;
  }
  return PGO_OK;
}

template <typename T>
pgo_status prepare_precision(pgo_graph* g, const double* t0_dev) {
  hipStream_t st = g->stream;
  if (g->chordal) {
    HIPCHK(launch_fill_edges_c<T>(g->o_perm, g->ej, g->R9, g->tm, g->kappa, g->tau, g->m, g->o_nbr,
                                  static_cast<P4<T>*>(g->o_tt), static_cast<R3<T>*>(g->o_w), st));
    HIPCHK(launch_fill_edges_c<T>(g->i_perm, g->ei, g->R9, g->tm, g->kappa, g->tau, g->m, g->i_nbr,
                                  static_cast<P4<T>*>(g->i_tt), static_cast<R3<T>*>(g->i_w), st));
    HIPCHK(launch_vertex_consts_c<T>(int32_t(g->n), g->o_ptr, g->o_perm, g->i_ptr, g->i_perm,
                                     g->kappa, g->tau, static_cast<T*>(g->cQ),
                                     static_cast<T*>(g->cT), static_cast<T*>(g->cS), st));
    HIPCHK(launch_init_state_c<T>(viewc<T>(g), g->P0, t0_dev, st));
    return PGO_OK;
  }
  HIPCHK(launch_fill_edges<T>(g->o_perm, g->ej, g->qe, g->tm, g->kappa, g->tau, g->m, g->o_nbr,
                              static_cast<P4<T>*>(g->o_tt), static_cast<Q4<T>*>(g->o_w), st));
  HIPCHK(launch_fill_edges<T>(g->i_perm, g->ei, g->qe, g->tm, g->kappa, g->tau, g->m, g->i_nbr,
                              static_cast<P4<T>*>(g->i_tt), static_cast<Q4<T>*>(g->i_w), st));
  HIPCHK(launch_vertex_consts<T>(int32_t(g->n), g->o_ptr, g->o_perm, g->i_ptr, g->i_perm, g->tm,
                                 g->kappa, g->tau, static_cast<T*>(g->cQ),
                                 static_cast<T*>(g->cT), static_cast<T*>(g->cS), st));
  if (g->aniso) {
    HIPCHK(launch_fill_edges_a<T>(g->o_perm, g->tm, g->S9, g->m, static_cast<P4<T>*>(g->o_tt),
                                  static_cast<V3<T>*>(g->o_Sa), static_cast<V3<T>*>(g->o_Sb), st));
    HIPCHK(launch_fill_edges_a<T>(g->i_perm, g->tm, g->S9, g->m, static_cast<P4<T>*>(g->i_tt),
                                  static_cast<V3<T>*>(g->i_Sa), static_cast<V3<T>*>(g->i_Sb), st));
    HIPCHK(launch_vertex_consts_a<T>(int32_t(g->n), g->o_ptr, g->o_perm, g->i_ptr, g->i_perm, g->S9,
                                     static_cast<V3<T>*>(g->cTa), static_cast<V3<T>*>(g->cTb),
                                     static_cast<V3<T>*>(g->cSa), static_cast<V3<T>*>(g->cSb), st));
  }
  HIPCHK(launch_init_state<T>(view<T>(g), g->p0, t0_dev, st));
  return PGO_OK;
}

pgo_status sort_edges(pgo_graph* g, const int32_t* keys, int32_t* perm, int32_t* ptr,
                      int32_t* iota, int32_t* keys_sorted, void** tmp, size_t* tmp_bytes) {
  if (g->m > 0) {
    size_t need = 0;
    HIPCHK(sort_by_key(keys, perm, g->m, int32_t(g->n), iota, nullptr, &need, keys_sorted,
                       g->stream));
    if (need > *tmp_bytes) {
      dfree(g, *tmp);
      *tmp = nullptr;
      pgo_status s = dalloc_bytes(g, tmp, need);
      if (s != PGO_OK) return s;
      *tmp_bytes = need;
    }
    size_t have = *tmp_bytes;
    HIPCHK(sort_by_key(keys, perm, g->m, int32_t(g->n), iota, *tmp, &have, keys_sorted, g->stream));
  }
  HIPCHK(launch_ptr_from_sorted(keys_sorted, g->m, int32_t(g->n), ptr, g->stream));
  return PGO_OK;
}

pgo_status first_bad(pgo_graph* g, const uint8_t* flags_dev, int64_t count, int64_t* idx) {
  *idx = -1;
  if (count <= 0) return PGO_OK;
  std::vector<uint8_t> h(static_cast<size_t>(count));
  HIPCHK(hipMemcpyAsync(h.data(), flags_dev, size_t(count), hipMemcpyDeviceToHost, g->stream));
  HIPCHK(hipStreamSynchronize(g->stream));
  for (int64_t i = 0; i < count; ++i)
    if (h[size_t(i)]) {
      *idx = i;
      break;
    }
  return PGO_OK;
}

void choose_default_schedule(pgo_graph* g) {
  const int req = g->opt.schedule;
  const bool graph_ok = g->max_n <= PGO_GRAPH_SCHED_MAX_N;
  if (req == PGO_SCHED_COOP)
    g->sched = PGO_SCHED_COOP;
  else if (req == PGO_SCHED_GRAPH && graph_ok)
    g->sched = PGO_SCHED_GRAPH;
  else if (req == PGO_SCHED_PHASE || !graph_ok)
    g->sched = PGO_SCHED_PHASE;
  else  // auto: one persistent workgroup per graph fills the GPU only with at
        // least as many graphs as compute units; fewer or larger graphs
        // spread every phase over all of them
    g->sched = (g->max_n <= 8192 && g->G >= 256) ? PGO_SCHED_GRAPH : PGO_SCHED_PHASE;
  if (g->opt.block) {
    g->block_phase = g->opt.block;
    g->block_graph = g->opt.block;
  } else {
    g->block_phase = 256;
    // per graph: enough threads for one vertex each up to 1024 vertices
    int b = 64;
    while (b < g->max_n && b < 1024) b *= 2;
    g->block_graph = g->aniso ? std::min(b, 512) : b;
  }
}

pgo_status create_impl(pgo_graph** out, int32_t G, const int64_t* voff, const int64_t* eoff,
                       const double* R0, const double* t0, const int32_t* ei, const int32_t* ej,
                       const double* Rm, const double* tm, const double* kappa, const double* tau,
                       const pgo_options* opt_in, const double* info = nullptr) {
  if (!out) return fail(PGO_EINVAL, "out must not be NULL");
  *out = nullptr;
  pgo_options opt;
  pgo_default_options(&opt);
  if (opt_in) opt = *opt_in;
  if (info) opt.model = PGO_MODEL_QUAT_INFO;
  else if (opt.model == PGO_MODEL_QUAT_INFO)
    return fail(PGO_EINVAL, "PGO_MODEL_QUAT_INFO handles are made by pgo_create_info");
  pgo_status s = check_options(opt);
  if (s != PGO_OK) return s;
  if (!voff || !eoff) return fail(PGO_EINVAL, "voff and eoff must not be NULL");
  s = check_inputs(G, voff, eoff, R0, t0, ei, ej, Rm, tm, kappa, tau);
  if (s != PGO_OK) return s;

  int ndev = 0;
  HIPCHK(hipGetDeviceCount(&ndev));
  if (opt.device < 0 || opt.device >= ndev)
    return fail(PGO_EINVAL, "device " + std::to_string(opt.device) + " does not exist");
  HIPCHK(hipSetDevice(opt.device));

  pgo_graph* g = new pgo_graph();
  g->device = opt.device;
  g->opt = opt;
  g->chordal = opt.model == PGO_MODEL_CHORDAL;
  g->aniso = opt.model == PGO_MODEL_QUAT_INFO;
  g->G = G;
  g->n = voff[G];
  g->m = eoff[G];
  g->voff_h.assign(voff, voff + G + 1);
  g->eoff_h.assign(eoff, eoff + G + 1);
  // mean over a graph's vertices of the diagonal weight 2 sum_out (tau |t~|^2
  // + kappa) + 2 sum_in kappa: the size of one vertex's update direction
  g->wbar_h.assign(size_t(G), 0.0);
  for (int32_t k = 0; k < G; ++k) {
    double w = 0.0;
    for (int64_t e = eoff[k]; e < eoff[k + 1]; ++e)
      w += 2.0 * tau[e] * (tm[3 * e] * tm[3 * e] + tm[3 * e + 1] * tm[3 * e + 1] +
                           tm[3 * e + 2] * tm[3 * e + 2]) + 4.0 * kappa[e];
    g->wbar_h[size_t(k)] = w / double(voff[k + 1] - voff[k]);
  }
  for (int32_t k = 0; k < G; ++k) g->max_n = std::max<int32_t>(g->max_n, int32_t(voff[k + 1] - voff[k]));
  auto bail = [&](pgo_status st) {
    pgo_destroy(g);
    return st;
  };
  hipError_t he = hipStreamCreateWithFlags(&g->own_stream, hipStreamNonBlocking);
  if (he != hipSuccess) return bail(hip_fail(he, "hipStreamCreate"));
  g->stream = g->own_stream;

  const int64_t n = g->n, m = g->m;
  // global edge indices
  std::vector<int32_t> gei(static_cast<size_t>(m)), gej(static_cast<size_t>(m));
  for (int32_t k = 0; k < G; ++k)
    for (int64_t e = eoff[k]; e < eoff[k + 1]; ++e) {
      gei[size_t(e)] = int32_t(ei[e] + voff[k]);
      gej[size_t(e)] = int32_t(ej[e] + voff[k]);
    }
  std::vector<int32_t> voff32(static_cast<size_t>(G) + 1);
  for (int32_t k = 0; k <= G; ++k) voff32[size_t(k)] = int32_t(voff[k]);
  std::vector<int32_t> gidh(static_cast<size_t>(n));
  for (int32_t k = 0; k < G; ++k)
    for (int64_t v = voff[k]; v < voff[k + 1]; ++v) gidh[size_t(v)] = k;
  std::vector<int32_t> order(static_cast<size_t>(G));
  std::iota(order.begin(), order.end(), 0);
  std::stable_sort(order.begin(), order.end(), [&](int32_t a, int32_t b) {
    return (voff[a + 1] - voff[a]) + (eoff[a + 1] - eoff[a]) >
           (voff[b + 1] - voff[b]) + (eoff[b + 1] - eoff[b]);
  });

  double *R0d = nullptr, *t0d = nullptr, *Rmd = nullptr;
  uint8_t* bad = nullptr;
  if ((s = upload(g, &g->ei, gei.data(), size_t(m))) != PGO_OK) return bail(s);
  if ((s = upload(g, &g->ej, gej.data(), size_t(m))) != PGO_OK) return bail(s);
  if ((s = upload(g, &g->tm, tm, size_t(3 * m))) != PGO_OK) return bail(s);
  if ((s = upload(g, &g->kappa, kappa, size_t(m))) != PGO_OK) return bail(s);
  if ((s = upload(g, &g->tau, tau, size_t(m))) != PGO_OK) return bail(s);
  if (info && (s = upload(g, &g->S9, info, size_t(9 * m))) != PGO_OK) return bail(s);
  if ((s = upload(g, &R0d, R0, size_t(9 * n))) != PGO_OK) return bail(s);
  if ((s = upload(g, &t0d, t0, size_t(3 * n))) != PGO_OK) return bail(s);
  if ((s = upload(g, &Rmd, Rm, size_t(9 * m))) != PGO_OK) return bail(s);
  if ((s = upload(g, &g->voff32, voff32.data(), voff32.size())) != PGO_OK) return bail(s);
  if ((s = upload(g, &g->order, order.data(), order.size())) != PGO_OK) return bail(s);
  if ((s = upload(g, &g->gid, gidh.data(), gidh.size())) != PGO_OK) return bail(s);
  if ((s = dalloc(g, &g->beta_dev, size_t(G))) != PGO_OK) return bail(s);
  if ((s = dalloc(g, &g->active_dev, size_t(G))) != PGO_OK) return bail(s);
  if ((s = dalloc(g, &g->flag_dev, size_t(G))) != PGO_OK) return bail(s);
  g->beta_h.assign(size_t(G), 1.0);
  if ((s = dalloc(g, &bad, size_t(std::max(n, m)))) != PGO_OK) return bail(s);
  int64_t badi = -1;
  if (g->chordal) {
    // rotations projected onto SO(3) (with validity flags)
    if ((s = dalloc(g, &g->P0, size_t(9 * n))) != PGO_OK) return bail(s);
    if ((s = dalloc(g, &g->R9, size_t(9 * m))) != PGO_OK) return bail(s);
    he = launch_project_rot(R0d, n, g->P0, bad, g->stream);
    if (he != hipSuccess) return bail(hip_fail(he, "project_rot"));
    if ((s = first_bad(g, bad, n, &badi)) != PGO_OK) return bail(s);
    if (badi >= 0)
      return bail(fail(PGO_EINVAL, "initial rotation " + std::to_string(badi) +
                                       " is not a rotation (det <= 0 or ||R^T R - I||_F > 1e-2)"));
    he = launch_project_rot(Rmd, m, g->R9, bad, g->stream);
    if (he != hipSuccess) return bail(hip_fail(he, "project_rot"));
    if ((s = first_bad(g, bad, m, &badi)) != PGO_OK) return bail(s);
    if (badi >= 0)
      return bail(fail(PGO_EINVAL, "measured rotation of edge " + std::to_string(badi) +
                                       " is not a rotation (det <= 0 or ||R^T R - I||_F > 1e-2)"));
  } else {
    if ((s = dalloc(g, &g->p0, size_t(n))) != PGO_OK) return bail(s);
    if ((s = dalloc(g, &g->qe, size_t(m))) != PGO_OK) return bail(s);

    // rotations -> quaternions (with validity flags)
    he = launch_rot_to_quat(R0d, n, g->p0, 1, bad, g->stream);
    if (he != hipSuccess) return bail(hip_fail(he, "rot_to_quat"));
    if ((s = first_bad(g, bad, n, &badi)) != PGO_OK) return bail(s);
    if (badi >= 0)
      return bail(fail(PGO_EINVAL, "initial rotation " + std::to_string(badi) +
                                       " is not a rotation (det <= 0 or ||R^T R - I||_F > 1e-2)"));
    he = launch_rot_to_quat(Rmd, m, g->qe, 0, bad, g->stream);
    if (he != hipSuccess) return bail(hip_fail(he, "rot_to_quat"));
    if ((s = first_bad(g, bad, m, &badi)) != PGO_OK) return bail(s);
    if (badi >= 0)
      return bail(fail(PGO_EINVAL, "measured rotation of edge " + std::to_string(badi) +
                                       " is not a rotation (det <= 0 or ||R^T R - I||_F > 1e-2)"));
    he = launch_align(g->p0, g->qe, g->ei, g->ej, m, g->stream);
    if (he != hipSuccess) return bail(hip_fail(he, "align"));
    if ((s = dalloc(g, &g->qe0, size_t(m))) != PGO_OK) return bail(s);
    if (m) {
      he = launch_copy(g->qe0, g->qe, sizeof(Q4<double>) * size_t(m), g->stream);
      if (he != hipSuccess) return bail(hip_fail(he, "copy"));
    }
    {
      std::vector<double> zeros(size_t(3 * m), 0.0);
      if ((s = upload(g, &g->omega, zeros.data(), zeros.size())) != PGO_OK) return bail(s);
    }
  }
  dfree(g, R0d);
  dfree(g, Rmd);
  dfree(g, bad);

  // CSR by tail, CSC by head
  int32_t *iota = nullptr, *keys_sorted = nullptr;
  void* tmp = nullptr;
  size_t tmp_bytes = 0;
  if ((s = dalloc(g, &g->o_ptr, size_t(n + 1))) != PGO_OK) return bail(s);
  if ((s = dalloc(g, &g->i_ptr, size_t(n + 1))) != PGO_OK) return bail(s);
  if ((s = dalloc(g, &g->o_perm, size_t(m))) != PGO_OK) return bail(s);
  if ((s = dalloc(g, &g->i_perm, size_t(m))) != PGO_OK) return bail(s);
  if ((s = dalloc(g, &g->o_nbr, size_t(m))) != PGO_OK) return bail(s);
  if ((s = dalloc(g, &g->i_nbr, size_t(m))) != PGO_OK) return bail(s);
  if ((s = dalloc(g, &iota, size_t(m))) != PGO_OK) return bail(s);
  if ((s = dalloc(g, &keys_sorted, size_t(m))) != PGO_OK) return bail(s);
  if ((s = sort_edges(g, g->ei, g->o_perm, g->o_ptr, iota, keys_sorted, &tmp, &tmp_bytes)) != PGO_OK)
    return bail(s);
  if ((s = sort_edges(g, g->ej, g->i_perm, g->i_ptr, iota, keys_sorted, &tmp, &tmp_bytes)) != PGO_OK)
    return bail(s);

  if (opt.precision == PGO_FP64) {
    if ((s = alloc_precision<double>(g)) != PGO_OK) return bail(s);
    if ((s = prepare_precision<double>(g, t0d)) != PGO_OK) return bail(s);
  } else {
    if ((s = alloc_precision<float>(g)) != PGO_OK) return bail(s);
    if ((s = prepare_precision<float>(g, t0d)) != PGO_OK) return bail(s);
  }
  if ((s = build_chunks(g)) != PGO_OK) return bail(s);
  he = hipStreamSynchronize(g->stream);
  if (he != hipSuccess) return bail(hip_fail(he, "prepare"));
  dfree(g, iota);
  dfree(g, keys_sorted);
  dfree(g, tmp);
  g->t0dev = t0d;
  choose_default_schedule(g);
  *out = g;
  return PGO_OK;
}

template <typename T>
pgo_status run_sweeps(pgo_graph* g, int32_t k, double beta, double gamma, int sched, int block,
                      bool per_graph, bool masked) {
  SweepParams sp{beta, gamma, g->opt.h1, g->opt.h2, g->opt.h3, g->opt.h4,
                 per_graph ? g->beta_dev : nullptr, masked ? g->active_dev : nullptr};
  const DevGraph<T> d = view<T>(g);
  const DevChordal<T> dc = viewc<T>(g);
  const DevAniso<T> da = viewa<T>(g);
  if (sched == PGO_SCHED_COOP) {
    if (g->chordal || g->aniso) return fail(PGO_EINVAL, "cooperative schedule: quaternion model only");
    HIPCHK(launch_coop_sweeps<T>(d, k, sp, block, g->coop_bar, g->stream));
    return PGO_OK;
  }
  if (sched == PGO_SCHED_GRAPH) {
    if (g->chordal)
      HIPCHK(launch_graph_sweeps_c<T>(dc, g->voff32, g->order, g->G, k, sp, block, g->max_n,
                                      g->graph_lds, g->stream));
    else if (g->aniso)
      HIPCHK(launch_graph_sweeps_a<T>(da, g->voff32, g->order, g->G, k, sp, block, g->max_n,
                                      g->graph_lds, g->stream));
    else
      HIPCHK(launch_graph_sweeps<T>(d, g->voff32, g->order, g->G, k, sp, block, g->max_n,
                                    g->graph_lds, g->stream));
    return PGO_OK;
  }
  auto phases = [&](hipStream_t st) {
    return g->chordal ? launch_phase_sweeps_c<T>(dc, k, sp, block, st)
           : g->aniso ? launch_phase_sweeps_a<T>(da, k, sp, block, st)
                      : launch_phase_sweeps<T>(d, k, sp, block, st);
  };
  // per-phase launches, captured once into a HIP graph per (k, beta, gamma, block)
  if (k == 1) {
    HIPCHK(phases(g->stream));
    return PGO_OK;
  }
  if (!(g->gexec && g->g_k == k && g->g_beta == beta && g->g_gamma == gamma &&
        g->g_block == block && g->g_per_graph == per_graph && g->g_masked == masked)) {
    if (g->gexec) {
      (void)hipGraphExecDestroy(g->gexec);
      g->gexec = nullptr;
    }
    hipGraph_t graph = nullptr;
    HIPCHK(hipStreamBeginCapture(g->stream, hipStreamCaptureModeThreadLocal));
    const hipError_t le = phases(g->stream);
    const hipError_t ce = hipStreamEndCapture(g->stream, &graph);
    if (le != hipSuccess) {
      if (graph) (void)hipGraphDestroy(graph);
      return hip_fail(le, "launch_phase_sweeps (capture)");
    }
    if (ce != hipSuccess) return hip_fail(ce, "hipStreamEndCapture");
    const hipError_t ie = hipGraphInstantiate(&g->gexec, graph, nullptr, nullptr, 0);
    (void)hipGraphDestroy(graph);
    if (ie != hipSuccess) {
      g->gexec = nullptr;
      return hip_fail(ie, "hipGraphInstantiate");
    }
    g->g_k = k;
    g->g_beta = beta;
    g->g_gamma = gamma;
    g->g_block = block;
    g->g_per_graph = per_graph;
    g->g_masked = masked;
  }
  HIPCHK(hipGraphLaunch(g->gexec, g->stream));
  return PGO_OK;
}

pgo_status iterate_with(pgo_graph* g, int32_t k, double beta, double gamma, int sched, int block,
                        const double* beta_g = nullptr, const int32_t* active = nullptr) {
  const bool per_graph = beta_g != nullptr;
  const bool masked = active != nullptr;
  if (per_graph)
    HIPCHK(hipMemcpyAsync(g->beta_dev, beta_g, sizeof(double) * g->G, hipMemcpyHostToDevice,
                          g->stream));
  if (masked)
    HIPCHK(hipMemcpyAsync(g->active_dev, active, sizeof(int32_t) * g->G, hipMemcpyHostToDevice,
                          g->stream));
  pgo_status s =
      g->opt.precision == PGO_FP64
          ? run_sweeps<double>(g, k, beta, gamma, sched, block, per_graph, masked)
          : run_sweeps<float>(g, k, beta, gamma, sched, block, per_graph, masked);
  if (s == PGO_OK) {
    g->have_prev = true;
    g->last_gamma = gamma;
    if (per_graph)
      g->beta_h.assign(beta_g, beta_g + g->G);
    else
      g->beta_h.assign(size_t(g->G), beta);
  }
  return s;
}

// Per-graph reduction values (RedIdx order).  Unless allow_nonfinite, a
// non-finite value anywhere is reported as PGO_ENUMERIC.
// active (device, G flags) restricts the work to the graphs flagged 1; the
// others report zeros.
pgo_status reduce(pgo_graph* g, std::vector<double>& out, bool allow_nonfinite = false,
                  const int32_t* active = nullptr) {
  HIPCHK(hipSetDevice(g->device));
  EdgeF64 e{g->ei, g->ej, g->qe, g->tm, g->kappa, g->tau, g->R9, g->S9};
  hipError_t he;
  if (g->chordal && g->opt.precision == PGO_FP64)
    he = launch_reduce_c<double>(viewc<double>(g), e, g->have_prev, g->ec_gid, g->ec_beg,
                                 g->ec_end, g->n_ech, g->vc_gid, g->vc_beg, g->vc_end, g->n_vch,
                                 g->part_e, g->part_v, g->g_ec_off, g->g_vc_off, g->G, g->red_out,
                                 active, g->stream);
  else if (g->chordal)
    he = launch_reduce_c<float>(viewc<float>(g), e, g->have_prev, g->ec_gid, g->ec_beg, g->ec_end,
                                g->n_ech, g->vc_gid, g->vc_beg, g->vc_end, g->n_vch, g->part_e,
                                g->part_v, g->g_ec_off, g->g_vc_off, g->G, g->red_out, active,
                                g->stream);
  else if (g->opt.precision == PGO_FP64)
    he = launch_reduce<double>(view<double>(g), e, g->have_prev, g->ec_gid, g->ec_beg, g->ec_end,
                               g->n_ech, g->vc_gid, g->vc_beg, g->vc_end, g->n_vch, g->part_e,
                               g->part_v, g->g_ec_off, g->g_vc_off, g->G, g->red_out, active,
                               g->stream);
  else
    he = launch_reduce<float>(view<float>(g), e, g->have_prev, g->ec_gid, g->ec_beg, g->ec_end,
                              g->n_ech, g->vc_gid, g->vc_beg, g->vc_end, g->n_vch, g->part_e,
                              g->part_v, g->g_ec_off, g->g_vc_off, g->G, g->red_out, active,
                              g->stream);
  if (he != hipSuccess) return hip_fail(he, "reduce");
  out.resize(size_t(kRedVals) * g->G);
  HIPCHK(hipMemcpyAsync(out.data(), g->red_out, out.size() * sizeof(double),
                        hipMemcpyDeviceToHost, g->stream));
  HIPCHK(hipStreamSynchronize(g->stream));
  if (!allow_nonfinite)
    for (double v : out)
      if (!std::isfinite(v)) return fail(PGO_ENUMERIC, "the state contains a non-finite value");
  return PGO_OK;
}

bool finite_graph(const std::vector<double>& r, int32_t j) {
  for (int k = 0; k < kRedVals; ++k)
    if (!std::isfinite(r[size_t(kRedVals) * j + k])) return false;
  return true;
}

pgo_status ensure_iobuf(pgo_graph* g) {
  if (g->iobuf) return PGO_OK;
  return dalloc(g, &g->iobuf, size_t(state_width(g)) * g->n);
}

}  // namespace

namespace {

// L_beta (PRADMM section) and the merit of Theorem 1 without its unknown
// proximal-difference terms, from one graph's reduction values.
void merit_of(const double* v, double beta, double gamma, double* L, double* psi) {
  const double a1 = std::fabs(1.0 - gamma) / (1.0 - std::fabs(1.0 - gamma));
  *L = v[kSplit] - v[kLamPQ] + 0.5 * beta * v[kPQ2] - v[kZTS] + 0.5 * beta * v[kTS2];
  *psi = *L + a1 / (gamma * beta) * v[kDL2];
}

// bytes per vertex of the six state arrays (p, q, lambda, t, s, z)
void state_array_bytes(const pgo_graph* g, size_t out[6]) {
  const size_t w = g->opt.precision == PGO_FP64 ? 8 : 4;
  for (int k = 0; k < 3; ++k) out[k] = size_t(rot_words(g)) * w;
  for (int k = 3; k < 6; ++k) out[k] = 3 * w;
}

// Copies the state into the snapshot arrays: every vertex, or (active, G
// device flags) the vertices of the flagged graphs only.
pgo_status snapshot(pgo_graph* g, const int32_t* active = nullptr) {
  size_t vb[6];
  state_array_bytes(g, vb);
  void* cur[6] = {g->p, g->q, g->lam, g->t, g->s, g->z};
  for (int k = 0; k < 6; ++k)
    if (!g->snap[k]) {
      pgo_status s = dalloc_bytes(g, &g->snap[k], vb[k] * size_t(g->n));
      if (s != PGO_OK) return s;
    }
  if (active) {
    int words[6];
    for (int k = 0; k < 6; ++k) words[k] = int(vb[k] / 4);
    HIPCHK(launch_restore_words(int32_t(g->n), g->gid, active, g->snap, cur, words, g->stream));
    return PGO_OK;
  }
  for (int k = 0; k < 6; ++k)
    HIPCHK(launch_copy(g->snap[k], cur[k], vb[k] * size_t(g->n), g->stream));
  return PGO_OK;
}

pgo_status restore_flagged(pgo_graph* g, const std::vector<int32_t>& flags) {
  HIPCHK(hipMemcpyAsync(g->flag_dev, flags.data(), sizeof(int32_t) * g->G, hipMemcpyHostToDevice,
                        g->stream));
  size_t vb[6];
  state_array_bytes(g, vb);
  void* dst[6] = {g->p, g->q, g->lam, g->t, g->s, g->z};
  const void* src[6];
  int words[6];
  for (int k = 0; k < 6; ++k) {
    src[k] = g->snap[k];
    words[k] = int(vb[k] / 4);
  }
  HIPCHK(launch_restore_words(int32_t(g->n), g->gid, g->flag_dev, dst, src, words, g->stream));
  HIPCHK(hipStreamSynchronize(g->stream));  // flags live on the host stack
  return PGO_OK;
}

}  // namespace


namespace {

size_t state_bytes(const pgo_graph* g) {
  return size_t(4) * (g->opt.precision == PGO_FP64 ? 8 : 4) * size_t(g->n);
}

pgo_status ensure_sets(pgo_graph* g, size_t count) {
  while (g->sets.size() < 6 * count) {
    void* p = nullptr;
    pgo_status s = dalloc_bytes(g, &p, state_bytes(g));
    if (s != PGO_OK) return s;
    g->sets.push_back(p);
  }
  return PGO_OK;
}

void** state_ptrs(pgo_graph* g, void** out6) {
  out6[0] = g->p; out6[1] = g->q; out6[2] = g->lam; out6[3] = g->t; out6[4] = g->s; out6[5] = g->z;
  return out6;
}

pgo_status copy_state(pgo_graph* g, void* const* dst, void* const* src) {
  size_t vb[6];
  state_array_bytes(g, vb);
  for (int k = 0; k < 6; ++k)
    HIPCHK(launch_copy(dst[k], src[k], vb[k] * size_t(g->n), g->stream));
  return PGO_OK;
}

template <typename T>
StateRef<T> stateref(void* const* s6) {
  return StateRef<T>{static_cast<const Q4<T>*>(s6[0]), static_cast<const Q4<T>*>(s6[1]),
                     static_cast<const Q4<T>*>(s6[2]), static_cast<const V3<T>*>(s6[3]),
                     static_cast<const V3<T>*>(s6[4]), static_cast<const V3<T>*>(s6[5])};
}

template <typename T>
AdjRef<T> adjref(pgo_graph* g) {
  AdjRef<T> A;
  A.pb = static_cast<Q4<T>*>(g->adj[0]);
  A.qb = static_cast<Q4<T>*>(g->adj[1]);
  A.lb = static_cast<Q4<T>*>(g->adj[2]);
  A.tb = static_cast<P4<T>*>(g->adj[3]);
  A.sb = static_cast<P4<T>*>(g->adj[4]);
  A.zb = static_cast<P4<T>*>(g->adj[5]);
  A.moS = static_cast<P4<T>*>(g->adj[6]);
  A.miT3 = static_cast<P4<T>*>(g->adj[7]);
  A.miT4q = static_cast<Q4<T>*>(g->adj[8]);
  A.miT4p = static_cast<Q4<T>*>(g->adj[9]);
  A.moQ4 = static_cast<Q4<T>*>(g->adj[10]);
  A.moQ3 = static_cast<P4<T>*>(g->adj[11]);
  A.moP = static_cast<P4<T>*>(g->adj[12]);
  A.miP = static_cast<Q4<T>*>(g->adj[13]);
  A.ga_o = static_cast<P4<double>*>(g->gacc[0]);
  A.gw_o = static_cast<Q4<double>*>(g->gacc[1]);
  A.ga_i = static_cast<P4<double>*>(g->gacc[2]);
  A.gw_i = static_cast<Q4<double>*>(g->gacc[3]);
  A.cqb = g->cgrad;
  A.ctb = g->cgrad + g->n;
  A.csb = g->cgrad + 2 * g->n;
  A.in2out = g->in2out;
  A.out2in = g->out2in;
  return A;
}

pgo_status ensure_adjoint_buffers(pgo_graph* g) {
  if (g->cgrad) return PGO_OK;
  const size_t vb = state_bytes(g), eb = size_t(4) * (g->opt.precision == PGO_FP64 ? 8 : 4) * size_t(g->m);
  pgo_status s;
  for (int k = 0; k < 6; ++k)
    if ((s = dalloc_bytes(g, &g->adj[k], vb)) != PGO_OK) return s;
  for (int k = 6; k < 14; ++k)
    if ((s = dalloc_bytes(g, &g->adj[k], eb)) != PGO_OK) return s;
  for (int k = 0; k < 4; ++k)
    if ((s = dalloc_bytes(g, &g->gacc[k], 32 * size_t(g->m))) != PGO_OK) return s;
  if ((s = dalloc(g, &g->pos_out, size_t(g->m))) != PGO_OK) return s;
  if ((s = dalloc(g, &g->pos_in, size_t(g->m))) != PGO_OK) return s;
  if ((s = dalloc(g, &g->in2out, size_t(g->m))) != PGO_OK) return s;
  if ((s = dalloc(g, &g->out2in, size_t(g->m))) != PGO_OK) return s;
  HIPCHK(launch_edge_maps(g->m, g->o_perm, g->i_perm, g->pos_out, g->pos_in, g->in2out,
                          g->out2in, g->stream));
  return dalloc(g, &g->cgrad, size_t(3) * size_t(g->n));
}

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
  if (g->aniso) {  // edge records (t~, c) and the information sums
    HIPCHK(launch_fill_edges_a<T>(g->o_perm, g->tm, g->S9, g->m, static_cast<P4<T>*>(g->o_tt),
                                  static_cast<V3<T>*>(g->o_Sa), static_cast<V3<T>*>(g->o_Sb), st));
    HIPCHK(launch_fill_edges_a<T>(g->i_perm, g->tm, g->S9, g->m, static_cast<P4<T>*>(g->i_tt),
                                  static_cast<V3<T>*>(g->i_Sa), static_cast<V3<T>*>(g->i_Sb), st));
    HIPCHK(launch_vertex_consts_a<T>(int32_t(g->n), g->o_ptr, g->o_perm, g->i_ptr, g->i_perm, g->S9,
                                     static_cast<V3<T>*>(g->cTa), static_cast<V3<T>*>(g->cTb),
                                     static_cast<V3<T>*>(g->cSa), static_cast<V3<T>*>(g->cSb), st));
  }
  return PGO_OK;
}

template <typename T>
pgo_status adjoint_impl(pgo_graph* g, const double* dL, double* gk, double* gt, double* gtm,
                        double* gom, double* dL0) {
  hipStream_t st = g->stream;
  const int K = g->rec_K, C = g->rec_C;
  const int nseg = (K + C - 1) / C;
  const DevGraph<T> d = view<T>(g);
  const AdjRef<T> A = adjref<T>(g);
  SweepParams sp{g->rec_beta, g->rec_gamma, g->opt.h1, g->opt.h2, g->opt.h3, g->opt.h4, nullptr,
                 nullptr};
  HIPCHK(launch_adj_io<T>(int(g->n), A, const_cast<double*>(dL), 1, st));
  HIPCHK(launch_adj_zero_edges<T>(g->m, A, st));
  void* cur[6];
  state_ptrs(g, cur);
  const size_t snap0 = size_t(nseg + 1);  // first set after the checkpoints
  const int block = g->sched == PGO_SCHED_GRAPH ? g->block_graph : g->block_phase;
  pgo_status s;
  for (int seg = nseg - 1; seg >= 0; --seg) {
    const int k0 = seg * C, L = std::min(K, k0 + C) - k0;
    void* const* cp = &g->sets[6 * size_t(seg)];
    if ((s = copy_state(g, cur, cp)) != PGO_OK) return s;
    if ((s = copy_state(g, &g->sets[6 * snap0], cp)) != PGO_OK) return s;
    for (int j = 0; j < L; ++j) {
      if ((s = iterate_with(g, 1, g->rec_beta, g->rec_gamma, g->sched, block)) != PGO_OK) return s;
      if ((s = copy_state(g, &g->sets[6 * (snap0 + j + 1)], cur)) != PGO_OK) return s;
    }
    for (int j = L - 1; j >= 0; --j) {
      const StateRef<T> X = stateref<T>(&g->sets[6 * (snap0 + j)]);
      const StateRef<T> Y = stateref<T>(&g->sets[6 * (snap0 + j + 1)]);
      const int first = (seg == nseg - 1 && j == L - 1) ? 1 : 0;
      HIPCHK(launch_reverse_sweep<T>(d, X, Y, A, sp, first, st));
    }
  }
  HIPCHK(launch_reverse_finish<T>(d, A, st));
  HIPCHK(launch_adj_params<T>(g->m, A, g->pos_out, g->pos_in, g->ei, g->ej, g->tm, g->kappa, g->tau,
                              g->qe0, g->omega, gk, gt, gtm, gom, st));
  if (dL0) HIPCHK(launch_adj_io<T>(int(g->n), A, dL0, 0, st));
  if ((s = copy_state(g, cur, &g->sets[6 * size_t(nseg)])) != PGO_OK) return s;  // back to x^K
  HIPCHK(hipStreamSynchronize(st));
  return PGO_OK;
}

pgo_status check_device_values(pgo_graph* g, const double* dev, size_t count, bool positive,
                               const char* what) {
  std::vector<double> h(count);
  if (count)
    HIPCHK(hipMemcpyAsync(h.data(), dev, sizeof(double) * count, hipMemcpyDeviceToHost, g->stream));
  HIPCHK(hipStreamSynchronize(g->stream));
  for (size_t k = 0; k < count; ++k)
    if (!std::isfinite(h[k]) || (positive && !(h[k] > 0.0)))
      return fail(PGO_EINVAL, std::string(what) + " entry " + std::to_string(k) +
                                  (positive ? " must be finite and > 0" : " must be finite"));
  return PGO_OK;
}

}  // namespace

namespace {

hipError_t state_io(pgo_graph* g, double* buf, int to_device) {
  if (g->chordal)
    return g->opt.precision == PGO_FP64
               ? launch_state_io_c<double>(viewc<double>(g), buf, to_device, g->stream)
               : launch_state_io_c<float>(viewc<float>(g), buf, to_device, g->stream);
  return g->opt.precision == PGO_FP64
             ? launch_state_io<double>(view<double>(g), buf, to_device, g->stream)
             : launch_state_io<float>(view<float>(g), buf, to_device, g->stream);
}

pgo_status quaternion_only(pgo_graph* g, const char* what) {
  if (!g->chordal && !g->aniso) return PGO_OK;
  return fail(PGO_ESTATE, std::string(what) + " exists for the isotropic quaternion model only");
}

}  // namespace

extern "C" {

void pgo_default_options(pgo_options* o) {
  if (!o) return;
  o->h1 = 1.0;
  o->h2 = 1e-3;
  o->h3 = 1e-3;
  o->h4 = 1e-3;
  o->precision = PGO_FP64;
  o->schedule = PGO_SCHED_AUTO;
  o->block = 0;
  o->device = 0;
  o->model = PGO_MODEL_QUAT;
}

const char* pgo_last_error(void) { return g_err.c_str(); }

pgo_status pgo_create(pgo_graph** out, int32_t n, const double* R0, const double* t0, int64_t m,
                      const int32_t* ei, const int32_t* ej, const double* Rm, const double* tm,
                      const double* kappa, const double* tau, const pgo_options* opt) {
  if (n < 1) return fail(PGO_EINVAL, "n must be >= 1");
  if (m < 0) return fail(PGO_EINVAL, "m must be >= 0");
  const int64_t voff[2] = {0, n}, eoff[2] = {0, m};
  return create_impl(out, 1, voff, eoff, R0, t0, ei, ej, Rm, tm, kappa, tau, opt);
}

pgo_status pgo_create_batched(pgo_graph** out, int32_t G, const int64_t* voff,
                              const int64_t* eoff, const double* R0, const double* t0,
                              const int32_t* ei, const int32_t* ej, const double* Rm,
                              const double* tm, const double* kappa, const double* tau,
                              const pgo_options* opt) {
  return create_impl(out, G, voff, eoff, R0, t0, ei, ej, Rm, tm, kappa, tau, opt);
}

pgo_status pgo_create_info(pgo_graph** out, int32_t G, const int64_t* voff, const int64_t* eoff,
                           const double* R0, const double* t0, const int32_t* ei,
                           const int32_t* ej, const double* Rm, const double* tm,
                           const double* kappa, const double* info, const pgo_options* opt) {
  if (!out) return fail(PGO_EINVAL, "out must not be NULL");
  *out = nullptr;
  if (G < 1 || !voff || !eoff) return fail(PGO_EINVAL, "need G >= 1 and offsets");
  const int64_t m = eoff[G];
  if (m > 0 && !info) return fail(PGO_EINVAL, "info must not be NULL");
  // each S_e: finite, symmetric, positive definite; c_e = trace / 3 stands in for tau
  std::vector<double> c(static_cast<size_t>(std::max<int64_t>(m, 0)));
  for (int64_t e = 0; e < m; ++e) {
    const double* S = info + 9 * e;
    double big = 0.0;
    for (int k = 0; k < 9; ++k) {
      if (!std::isfinite(S[k]))
        return fail(PGO_EINVAL, "info of edge " + std::to_string(e) + " is not finite");
      big = std::max(big, std::fabs(S[k]));
    }
    if (std::fabs(S[1] - S[3]) > 1e-12 * big || std::fabs(S[2] - S[6]) > 1e-12 * big ||
        std::fabs(S[5] - S[7]) > 1e-12 * big)
      return fail(PGO_EINVAL, "info of edge " + std::to_string(e) + " is not symmetric");
    const double l11 = S[0] > 0 ? std::sqrt(S[0]) : 0.0;
    const double l21 = l11 > 0 ? S[3] / l11 : 0.0, l31 = l11 > 0 ? S[6] / l11 : 0.0;
    const double d2 = S[4] - l21 * l21;
    const double l22 = d2 > 0 ? std::sqrt(d2) : 0.0;
    const double l32 = l22 > 0 ? (S[7] - l31 * l21) / l22 : 0.0;
    const double d3 = S[8] - l31 * l31 - l32 * l32;
    if (!(l11 > 0 && d2 > 0 && d3 > 0))
      return fail(PGO_EINVAL, "info of edge " + std::to_string(e) + " is not positive definite");
    c[size_t(e)] = (S[0] + S[4] + S[8]) / 3.0;
  }
  static const double no_edges[9] = {};
  return create_impl(out, G, voff, eoff, R0, t0, ei, ej, Rm, tm, kappa, c.data(), opt,
                     info ? info : no_edges);
}

pgo_status pgo_set_stream(pgo_graph* g, void* hip_stream) {
  if (!g) return fail(PGO_EINVAL, "handle is NULL");
  g->stream = hip_stream ? static_cast<hipStream_t>(hip_stream) : g->own_stream;
  return PGO_OK;
}

pgo_status pgo_iterate(pgo_graph* g, int32_t k, double beta, double gamma) {
  if (!g) return fail(PGO_EINVAL, "handle is NULL");
  if (k < 0) return fail(PGO_EINVAL, "k must be >= 0");
  if (!(std::isfinite(beta) && beta > 0.0)) return fail(PGO_EINVAL, "beta must be finite and > 0");
  if (!(gamma > 0.0 && gamma < 2.0)) return fail(PGO_EINVAL, "gamma must lie in (0, 2)");
  if (k == 0) return PGO_OK;
  HIPCHK(hipSetDevice(g->device));
  const int block = g->sched == PGO_SCHED_GRAPH ? g->block_graph : g->block_phase;
  return iterate_with(g, k, beta, gamma, g->sched, block);
}

pgo_status pgo_iterate_graphs(pgo_graph* g, int32_t k, const double* beta, double gamma) {
  if (!g || !beta) return fail(PGO_EINVAL, "NULL argument");
  if (k < 0) return fail(PGO_EINVAL, "k must be >= 0");
  for (int32_t j = 0; j < g->G; ++j)
    if (!(std::isfinite(beta[j]) && beta[j] > 0.0))
      return fail(PGO_EINVAL, "beta of graph " + std::to_string(j) + " must be finite and > 0");
  if (!(gamma > 0.0 && gamma < 2.0)) return fail(PGO_EINVAL, "gamma must lie in (0, 2)");
  if (k == 0) return PGO_OK;
  HIPCHK(hipSetDevice(g->device));
  const int block = g->sched == PGO_SCHED_GRAPH ? g->block_graph : g->block_phase;
  return iterate_with(g, k, beta[0], gamma, g->sched, block, beta);
}

pgo_status pgo_merit(pgo_graph* g, double* out) {
  if (!g || !out) return fail(PGO_EINVAL, "NULL argument");
  return pgo_evaluate(g, nullptr, nullptr, out);
}

pgo_status pgo_iterate_until(pgo_graph* g, int32_t max_sweeps, int32_t check_every,
                             const double* beta, double gamma, double tol, int32_t* sweeps_done) {
  if (!g || !beta || !sweeps_done) return fail(PGO_EINVAL, "NULL argument");
  if (check_every < 1 || max_sweeps < 0 || max_sweeps % check_every != 0)
    return fail(PGO_EINVAL, "need check_every >= 1 and max_sweeps a multiple of check_every");
  if (!(gamma > 0.0 && gamma < 2.0)) return fail(PGO_EINVAL, "gamma must lie in (0, 2)");
  if (!std::isfinite(tol)) return fail(PGO_EINVAL, "tol must be finite");
  const int32_t G = g->G;
  for (int32_t j = 0; j < G; ++j)
    if (!(std::isfinite(beta[j]) && beta[j] > 0.0))
      return fail(PGO_EINVAL, "beta of graph " + std::to_string(j) + " must be finite and > 0");
  pgo_status s = PGO_OK;
  std::fill(sweeps_done, sweeps_done + G, 0);
  if (max_sweeps == 0) return PGO_OK;
  HIPCHK(hipSetDevice(g->device));
  if (g->sched == PGO_SCHED_GRAPH && !g->chordal && !g->aniso) {  // the rule inside the kernel
    if (!g->done_dev && (s = dalloc(g, &g->done_dev, size_t(G))) != PGO_OK) return s;
    HIPCHK(hipMemcpyAsync(g->beta_dev, beta, sizeof(double) * G, hipMemcpyHostToDevice,
                          g->stream));
    SweepParams sp{beta[0], gamma, g->opt.h1, g->opt.h2, g->opt.h3, g->opt.h4, g->beta_dev,
                   nullptr};
    sp.tol = tol;
    sp.check_every = check_every;
    sp.done = g->done_dev;
    const hipError_t he =
        g->opt.precision == PGO_FP64
            ? launch_graph_sweeps_stop<double>(view<double>(g), g->voff32, g->order, G,
                                               max_sweeps, sp, g->block_graph, g->max_n,
                                               g->graph_lds, g->stream)
            : launch_graph_sweeps_stop<float>(view<float>(g), g->voff32, g->order, G,
                                              max_sweeps, sp, g->block_graph, g->max_n,
                                              g->graph_lds, g->stream);
    if (he != hipSuccess) return hip_fail(he, "per-graph sweeps with stopping");
    HIPCHK(hipMemcpyAsync(sweeps_done, g->done_dev, sizeof(int32_t) * G, hipMemcpyDeviceToHost,
                          g->stream));
    HIPCHK(hipStreamSynchronize(g->stream));
  } else {  // chunks of check_every sweeps and an FP64 reduction after each
    std::vector<int32_t> active(size_t(G), 1);
    std::vector<double> r;
    const int block = g->sched == PGO_SCHED_GRAPH ? g->block_graph : g->block_phase;
    for (int32_t done = 0; done < max_sweeps; done += check_every) {
      if ((s = iterate_with(g, check_every, beta[0], gamma, g->sched, block, beta,
                            active.data())) != PGO_OK)
        return s;
      if ((s = reduce(g, r, false, g->active_dev)) != PGO_OK) return s;
      bool any = false;
      for (int32_t j = 0; j < G; ++j) {
        if (!active[size_t(j)]) continue;
        sweeps_done[j] += check_every;
        const double* v = &r[size_t(kRedVals) * j];
        const double e = (v[kDL2] + v[kDZ2]) / beta[j] + beta[j] * (v[kDQ2] + v[kDT2]);
        if (e < tol) active[size_t(j)] = 0;
        any = any || active[size_t(j)];
      }
      if (!any) break;
    }
  }
  g->have_prev = true;
  g->last_gamma = gamma;
  g->beta_h.assign(beta, beta + G);
  return PGO_OK;
}

pgo_status pgo_solve(pgo_graph* g, int32_t max_sweeps, int32_t check_every, double gamma,
                     double tol, double beta_growth, double* beta, int32_t* sweeps_done,
                     int32_t* converged) {
  if (!g || !beta) return fail(PGO_EINVAL, "NULL argument");
  if (check_every < 1 || max_sweeps < 0 || max_sweeps % check_every != 0)
    return fail(PGO_EINVAL, "need check_every >= 1 and max_sweeps a multiple of check_every");
  if (!(gamma > 0.0 && gamma < 2.0)) return fail(PGO_EINVAL, "gamma must lie in (0, 2)");
  if (!(beta_growth >= 1.0) || !std::isfinite(beta_growth) || !std::isfinite(tol))
    return fail(PGO_EINVAL, "beta_growth must be >= 1 and tol finite");
  const int32_t G = g->G;
  for (int32_t j = 0; j < G; ++j)
    if (!(std::isfinite(beta[j]) && beta[j] > 0.0))
      return fail(PGO_EINVAL, "beta of graph " + std::to_string(j) + " must be finite and > 0");
  HIPCHK(hipSetDevice(g->device));
  const bool adapt = beta_growth > 1.0;
  constexpr int kMaxRejects = 40;
  constexpr double kBetaMax = 1e30;  // a penalty stays representable in FP32
  // A chunk counts as a rise of the merit only beyond the rounding noise of
  // the state it is evaluated on.  Rounding a stored rotation moves it off
  // its manifold by a few ulps, which changes L_beta to first order by the
  // size of the vertex's update direction, at most ~(beta + w) per vertex
  // (w the mean diagonal weight): noise <= 8 eps (beta + w) n per graph.
  const double eps = g->opt.precision == PGO_FP32 ? 0x1p-24 : 0x1p-53;
  std::vector<int32_t> active(size_t(G), 1), done(size_t(G), 0), conv(size_t(G), 0),
      rejects(size_t(G), 0), flags(size_t(G), 0);
  std::vector<double> r, r_acc;
  pgo_status s = reduce(g, r_acc);  // values at the start: the accepted reference
  if (s != PGO_OK) return s;
  const int block = g->sched == PGO_SCHED_GRAPH ? g->block_graph : g->block_phase;
  g->last_gamma = gamma;
  for (;;) {
    bool any = false;
    for (int32_t j = 0; j < G; ++j) {
      if (done[size_t(j)] >= max_sweeps) active[size_t(j)] = 0;
      any = any || active[size_t(j)];
    }
    if (!any) break;
    // snapshots and reductions cover the running graphs only
    HIPCHK(hipMemcpyAsync(g->active_dev, active.data(), sizeof(int32_t) * G,
                          hipMemcpyHostToDevice, g->stream));
    if (adapt && (s = snapshot(g, g->active_dev)) != PGO_OK) return s;
    if ((s = iterate_with(g, check_every, beta[0], gamma, g->sched, block, beta, active.data())) !=
        PGO_OK)
      return s;
    if ((s = reduce(g, r, true, g->active_dev)) != PGO_OK) return s;
    bool any_restore = false;
    for (int32_t j = 0; j < G; ++j) {
      flags[size_t(j)] = 0;
      if (!active[size_t(j)]) {
        std::copy(&r[size_t(kRedVals) * j], &r[size_t(kRedVals) * (j + 1)],
                  &r_acc[size_t(kRedVals) * j]);
        continue;
      }
      const double* v = &r[size_t(kRedVals) * j];
      const bool finite = finite_graph(r, j);
      double L1, psi1, L0, psi0;
      merit_of(v, beta[j], gamma, &L1, &psi1);
      merit_of(&r_acc[size_t(kRedVals) * j], beta[j], gamma, &L0, &psi0);
      const double ng = double(g->voff_h[size_t(j) + 1] - g->voff_h[size_t(j)]);
      const double noise = 8.0 * eps * (beta[j] + g->wbar_h[size_t(j)]) * ng;
      const bool rose = !finite || psi1 > psi0 + 1e-12 * std::fabs(psi0) + noise;
      const bool can_raise = rejects[size_t(j)] < kMaxRejects && beta[j] * beta_growth <= kBetaMax;
      if (!finite && !(adapt && can_raise))
        return fail(PGO_ENUMERIC, "graph " + std::to_string(j) +
                                      " reached a non-finite state (penalty too small)");
      if (adapt && rose && can_raise) {
        flags[size_t(j)] = 1;  // undo this graph's chunk and raise its penalty
        any_restore = true;
        beta[j] *= beta_growth;
        ++rejects[size_t(j)];
        continue;
      }
      std::copy(v, v + kRedVals, &r_acc[size_t(kRedVals) * j]);
      done[size_t(j)] += check_every;
      const double b = beta[j];
      const double e = (v[kDL2] + v[kDZ2]) / b + b * (v[kDQ2] + v[kDT2]);
      if (tol > 0.0 && e < tol) {
        conv[size_t(j)] = 1;
        active[size_t(j)] = 0;
      }
    }
    if (any_restore && (s = restore_flagged(g, flags)) != PGO_OK) return s;
  }
  g->beta_h.assign(beta, beta + G);
  if (sweeps_done) std::copy(done.begin(), done.end(), sweeps_done);
  if (converged) std::copy(conv.begin(), conv.end(), converged);
  return PGO_OK;
}

pgo_status pgo_cost(pgo_graph* g, double* F) {
  if (!g || !F) return fail(PGO_EINVAL, "NULL argument");
  return pgo_evaluate(g, F, nullptr, nullptr);
}

pgo_status pgo_residuals(pgo_graph* g, double* out) {
  if (!g || !out) return fail(PGO_EINVAL, "NULL argument");
  return pgo_evaluate(g, nullptr, out, nullptr);
}

pgo_status pgo_evaluate(pgo_graph* g, double* F, double* res, double* merit) {
  if (!g) return fail(PGO_EINVAL, "NULL argument");
  std::vector<double> r;
  pgo_status s = reduce(g, r);
  if (s != PGO_OK) return s;
  for (int32_t k = 0; k < g->G; ++k) {
    const double b = g->beta_h[size_t(k)];
    const double* v = &r[size_t(kRedVals) * k];
    if (F) F[k] = v[kCost];
    if (res) {
      double* o = res + 6 * size_t(k);
      o[0] = std::sqrt(v[kPQ2]);
      o[1] = std::sqrt(v[kTS2]);
      o[2] = (v[kDL2] + v[kDZ2]) / b + b * (v[kDQ2] + v[kDT2]);
      o[3] = b * std::sqrt(v[kDQ2]);
      o[4] = b * std::sqrt(v[kDS2]);
      o[5] = v[kCost];
    }
    if (merit) merit_of(v, b, g->last_gamma, &merit[2 * size_t(k)], &merit[2 * size_t(k) + 1]);
  }
  return PGO_OK;
}

pgo_status pgo_evaluate_noalloc(pgo_graph* g, const double* beta_dev, double gamma,
                                double* out_dev) {
  if (!g || !beta_dev || !out_dev) return fail(PGO_EINVAL, "NULL argument");
  if (g->chordal)
    return fail(PGO_ESTATE, "pgo_evaluate_noalloc exists for the quaternion models only");
  if (!(gamma > 0.0 && gamma < 2.0)) return fail(PGO_EINVAL, "gamma must lie in (0, 2)");
  const size_t need = size_t(kEdgeVals) * g->n_ech + size_t(kVertVals) * g->n_vch +
                      size_t(kRedVals) * size_t(g->G);
  if (need > kScratchDoubles)
    return fail(PGO_EINVAL, "the handle's reductions need " + std::to_string(need) +
                                " doubles of the static scratch, which holds " +
                                std::to_string(kScratchDoubles) + " (use pgo_evaluate)");
  HIPCHK(hipSetDevice(g->device));
  double* scr = nullptr;
  HIPCHK(scratch_address(g->device, &scr));
  EdgeF64 e{g->ei, g->ej, g->qe, g->tm, g->kappa, g->tau, g->R9, g->S9};
  const hipError_t he =
      g->opt.precision == PGO_FP64
          ? launch_evaluate_noalloc<double>(view<double>(g), e, g->have_prev, g->ec_gid, g->ec_beg,
                                            g->ec_end, g->n_ech, g->vc_gid, g->vc_beg, g->vc_end,
                                            g->n_vch, g->g_ec_off, g->g_vc_off, g->G, scr,
                                            beta_dev, gamma, out_dev, g->stream)
          : launch_evaluate_noalloc<float>(view<float>(g), e, g->have_prev, g->ec_gid, g->ec_beg,
                                           g->ec_end, g->n_ech, g->vc_gid, g->vc_beg, g->vc_end,
                                           g->n_vch, g->g_ec_off, g->g_vc_off, g->G, scr,
                                           beta_dev, gamma, out_dev, g->stream);
  if (he != hipSuccess) return hip_fail(he, "evaluate_noalloc");
  return PGO_OK;
}

pgo_status pgo_get_poses(pgo_graph* g, double* R, double* t) {
  if (!g) return fail(PGO_EINVAL, "handle is NULL");
  if (!R && !t) return PGO_OK;
  HIPCHK(hipSetDevice(g->device));
  pgo_status s = ensure_iobuf(g);
  if (s != PGO_OK) return s;
  double* dR = R ? g->iobuf : nullptr;
  double* dt = t ? g->iobuf + 9 * g->n : nullptr;
  hipError_t he;
  if (g->chordal)
    he = g->opt.precision == PGO_FP64 ? launch_poses_c<double>(viewc<double>(g), dR, dt, g->stream)
                                      : launch_poses_c<float>(viewc<float>(g), dR, dt, g->stream);
  else
    he = g->opt.precision == PGO_FP64 ? launch_poses<double>(view<double>(g), dR, dt, g->stream)
                                      : launch_poses<float>(view<float>(g), dR, dt, g->stream);
  if (he != hipSuccess) return hip_fail(he, "poses");
  if (R) HIPCHK(hipMemcpyAsync(R, dR, sizeof(double) * 9 * g->n, hipMemcpyDeviceToHost, g->stream));
  if (t) HIPCHK(hipMemcpyAsync(t, dt, sizeof(double) * 3 * g->n, hipMemcpyDeviceToHost, g->stream));
  HIPCHK(hipStreamSynchronize(g->stream));
  return PGO_OK;
}

pgo_status pgo_get_state(pgo_graph* g, double* state) {
  if (!g || !state) return fail(PGO_EINVAL, "NULL argument");
  HIPCHK(hipSetDevice(g->device));
  pgo_status s = ensure_iobuf(g);
  if (s != PGO_OK) return s;
  hipError_t he = state_io(g, g->iobuf, 0);
  if (he != hipSuccess) return hip_fail(he, "state_io");
  HIPCHK(hipMemcpyAsync(state, g->iobuf, sizeof(double) * state_width(g) * g->n,
                        hipMemcpyDeviceToHost, g->stream));
  HIPCHK(hipStreamSynchronize(g->stream));
  return PGO_OK;
}

pgo_status pgo_set_state(pgo_graph* g, const double* state) {
  if (!g || !state) return fail(PGO_EINVAL, "NULL argument");
  HIPCHK(hipSetDevice(g->device));
  pgo_status s = ensure_iobuf(g);
  if (s != PGO_OK) return s;
  HIPCHK(hipMemcpyAsync(g->iobuf, state, sizeof(double) * state_width(g) * g->n,
                        hipMemcpyHostToDevice, g->stream));
  hipError_t he = state_io(g, g->iobuf, 1);
  if (he != hipSuccess) return hip_fail(he, "state_io");
  HIPCHK(hipStreamSynchronize(g->stream));
  g->have_prev = false;
  return PGO_OK;
}

pgo_status pgo_get_prepared(pgo_graph* g, double* edge_quat, double* vertex_quat0) {
  if (!g) return fail(PGO_EINVAL, "handle is NULL");
  HIPCHK(hipSetDevice(g->device));
  const size_t w = g->chordal ? 9 : 4;
  const void* e_src = g->chordal ? static_cast<const void*>(g->R9) : g->qe;
  const void* v_src = g->chordal ? static_cast<const void*>(g->P0) : g->p0;
  if (edge_quat && g->m)
    HIPCHK(hipMemcpyAsync(edge_quat, e_src, sizeof(double) * w * g->m, hipMemcpyDeviceToHost,
                          g->stream));
  if (vertex_quat0)
    HIPCHK(hipMemcpyAsync(vertex_quat0, v_src, sizeof(double) * w * g->n, hipMemcpyDeviceToHost,
                          g->stream));
  HIPCHK(hipStreamSynchronize(g->stream));
  return PGO_OK;
}

pgo_status pgo_info(pgo_graph* g, int64_t* n, int64_t* m, int32_t* G, int32_t* precision,
                    int32_t* schedule, int32_t* block, int32_t* model, int32_t* lds) {
  if (!g) return fail(PGO_EINVAL, "handle is NULL");
  if (n) *n = g->n;
  if (m) *m = g->m;
  if (G) *G = g->G;
  if (precision) *precision = g->opt.precision;
  if (schedule) *schedule = g->sched;
  if (block) *block = g->sched == PGO_SCHED_GRAPH ? g->block_graph : g->block_phase;
  if (model) *model = g->opt.model;
  if (lds) *lds = (g->sched == PGO_SCHED_GRAPH && g->graph_lds) ? 1 : 0;
  return PGO_OK;
}

pgo_status pgo_autotune(pgo_graph* g, double beta, double gamma, int32_t sweeps) {
  if (!g) return fail(PGO_EINVAL, "handle is NULL");
  if (sweeps < 1) return fail(PGO_EINVAL, "sweeps must be >= 1");
  if (!(std::isfinite(beta) && beta > 0.0)) return fail(PGO_EINVAL, "beta must be finite and > 0");
  if (!(gamma > 0.0 && gamma < 2.0)) return fail(PGO_EINVAL, "gamma must lie in (0, 2)");
  HIPCHK(hipSetDevice(g->device));
  std::vector<double> saved(size_t(state_width(g)) * g->n);
  pgo_status s = pgo_get_state(g, saved.data());
  if (s != PGO_OK) return s;
  // the candidates' runs overwrite the penalties, gamma and the residual
  // history (values before the last sweep) that pgo_merit, pgo_residuals
  // and pgo_evaluate use: keep them and put them back
  const std::vector<double> beta_keep = g->beta_h;
  const double gamma_keep = g->last_gamma;
  const bool prev_keep = g->have_prev;
  size_t vb[6];
  state_array_bytes(g, vb);
  void* prev[5] = {g->q_prev, g->lam_prev, g->t_prev, g->s_prev, g->z_prev};
  const size_t prev_bytes[5] = {vb[1], vb[2], vb[3], vb[4], vb[5]};
  void* hist[5] = {};
  auto release = [&]() {
    for (void* p : hist) dfree(g, p);
  };
  for (int k = 0; k < 5 && prev_keep; ++k) {
    if ((s = dalloc_bytes(g, &hist[k], prev_bytes[k] * size_t(g->n))) != PGO_OK) {
      release();
      return s;
    }
    HIPCHK(launch_copy(hist[k], prev[k], prev_bytes[k] * size_t(g->n), g->stream));
  }
  struct Cand {
    int sched, block, lds;
  };
  std::vector<Cand> cands;
  const int bmax = g->aniso ? 256 : 1024, bmax_graph = g->aniso ? 512 : 1024;
  for (int b : {64, 128, 256, 512})
    if (b <= bmax) cands.push_back({PGO_SCHED_PHASE, b, 0});
  if (!g->chordal && !g->aniso)
    for (int b : {128, 256, 512, 1024}) cands.push_back({PGO_SCHED_COOP, b, 0});
  if (g->max_n <= PGO_GRAPH_SCHED_MAX_N)
    for (int b : {128, 256, 512, 1024}) {
      if (b > bmax_graph) continue;
      cands.push_back({PGO_SCHED_GRAPH, b, 0});
      cands.push_back({PGO_SCHED_GRAPH, b, 1});
    }
  hipEvent_t e0, e1;
  HIPCHK(hipEventCreate(&e0));
  HIPCHK(hipEventCreate(&e1));
  float best = 1e30f;
  Cand pick{g->sched, g->sched == PGO_SCHED_GRAPH ? g->block_graph : g->block_phase,
            g->graph_lds};
  const int lds_before = g->graph_lds;
  for (const Cand& c : cands) {
    g->graph_lds = c.lds;
    if ((s = pgo_set_state(g, saved.data())) != PGO_OK) break;
    if ((s = iterate_with(g, sweeps, beta, gamma, c.sched, c.block)) != PGO_OK) break;  // warm-up
    if ((s = pgo_set_state(g, saved.data())) != PGO_OK) break;
    (void)hipEventRecord(e0, g->stream);
    if ((s = iterate_with(g, sweeps, beta, gamma, c.sched, c.block)) != PGO_OK) break;
    (void)hipEventRecord(e1, g->stream);
    (void)hipEventSynchronize(e1);
    float ms = 0.f;
    (void)hipEventElapsedTime(&ms, e0, e1);
    if (ms < best) {
      best = ms;
      pick = c;
    }
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  g->graph_lds = lds_before;
  if (s != PGO_OK) {
    release();
    return s;
  }
  g->sched = pick.sched;
  if (pick.sched == PGO_SCHED_GRAPH) g->graph_lds = pick.lds;
  if (pick.sched == PGO_SCHED_GRAPH)
    g->block_graph = pick.block;
  else
    g->block_phase = pick.block;
  s = pgo_set_state(g, saved.data());
  if (s == PGO_OK && prev_keep) {
    for (int k = 0; k < 5; ++k)
      HIPCHK(launch_copy(prev[k], hist[k], prev_bytes[k] * size_t(g->n), g->stream));
    HIPCHK(hipStreamSynchronize(g->stream));
  }
  release();
  g->beta_h = beta_keep;
  g->last_gamma = gamma_keep;
  g->have_prev = prev_keep;
  return s;
}

pgo_status pgo_set_edge_params(pgo_graph* g, const double* kappa, const double* tau,
                               const double* tm, const double* omega) {
  if (!g) return fail(PGO_EINVAL, "handle is NULL");
  pgo_status s = quaternion_only(g, "pgo_set_edge_params");
  if (s != PGO_OK) return s;
  HIPCHK(hipSetDevice(g->device));
  const size_t m = size_t(g->m);
  if (kappa && (s = check_device_values(g, kappa, m, true, "kappa")) != PGO_OK) return s;
  if (tau && (s = check_device_values(g, tau, m, true, "tau")) != PGO_OK) return s;
  if (tm && (s = check_device_values(g, tm, 3 * m, false, "tm")) != PGO_OK) return s;
  if (omega && (s = check_device_values(g, omega, 3 * m, false, "omega")) != PGO_OK) return s;
  if (m == 0) return PGO_OK;
  if (kappa) HIPCHK(launch_copy(g->kappa, kappa, 8 * m, g->stream));
  if (tau) HIPCHK(launch_copy(g->tau, tau, 8 * m, g->stream));
  if (tm) HIPCHK(launch_copy(g->tm, tm, 24 * m, g->stream));
  if (omega) {
    HIPCHK(launch_copy(g->omega, omega, 24 * m, g->stream));
    HIPCHK(launch_perturb(g->m, g->qe0, g->omega, g->qe, g->stream));
  }
  s = g->opt.precision == PGO_FP64 ? refill_edges<double>(g) : refill_edges<float>(g);
  if (s != PGO_OK) return s;
  g->rec_K = -1;  // a recorded forward pass no longer matches the edges
  HIPCHK(hipStreamSynchronize(g->stream));
  return PGO_OK;
}

pgo_status pgo_reset_state(pgo_graph* g) {
  if (!g) return fail(PGO_EINVAL, "handle is NULL");
  HIPCHK(hipSetDevice(g->device));
  hipError_t he;
  if (g->chordal)
    he = g->opt.precision == PGO_FP64
             ? launch_init_state_c<double>(viewc<double>(g), g->P0, g->t0dev, g->stream)
             : launch_init_state_c<float>(viewc<float>(g), g->P0, g->t0dev, g->stream);
  else
    he = g->opt.precision == PGO_FP64
             ? launch_init_state<double>(view<double>(g), g->p0, g->t0dev, g->stream)
             : launch_init_state<float>(view<float>(g), g->p0, g->t0dev, g->stream);
  if (he != hipSuccess) return hip_fail(he, "reset_state");
  HIPCHK(hipStreamSynchronize(g->stream));
  g->have_prev = false;
  g->rec_K = -1;
  return PGO_OK;
}

pgo_status pgo_chordal_init(pgo_graph* g, int32_t max_iters, double tol, int32_t* iters) {
  if (!g) return fail(PGO_EINVAL, "handle is NULL");
  if (max_iters < 1) return fail(PGO_EINVAL, "max_iters must be >= 1");
  if (!(std::isfinite(tol) && tol > 0.0 && tol < 1.0))
    return fail(PGO_EINVAL, "tol must lie in (0, 1)");
  HIPCHK(hipSetDevice(g->device));
  const int64_t n = g->n, m = g->m;
  const int32_t G = g->G;
  hipStream_t st = g->stream;
  // one anchor per connected component: its lowest-index vertex
  std::vector<int32_t> hei(static_cast<size_t>(m)), hej(static_cast<size_t>(m));
  if (m) {
    HIPCHK(hipMemcpyAsync(hei.data(), g->ei, 4 * size_t(m), hipMemcpyDeviceToHost, st));
    HIPCHK(hipMemcpyAsync(hej.data(), g->ej, 4 * size_t(m), hipMemcpyDeviceToHost, st));
    HIPCHK(hipStreamSynchronize(st));
  }
  std::vector<int32_t> parent(static_cast<size_t>(n));
  std::iota(parent.begin(), parent.end(), 0);
  auto find = [&](int32_t x) {
    while (parent[size_t(x)] != x) {
      parent[size_t(x)] = parent[size_t(parent[size_t(x)])];
      x = parent[size_t(x)];
    }
    return x;
  };
  for (int64_t e = 0; e < m; ++e) {  // union by smaller root index
    const int32_t a = find(hei[size_t(e)]), b = find(hej[size_t(e)]);
    if (a != b) parent[size_t(std::max(a, b))] = std::min(a, b);
  }
  std::vector<uint8_t> anchor(static_cast<size_t>(n));
  for (int64_t v = 0; v < n; ++v) anchor[size_t(v)] = find(int32_t(v)) == v ? 1 : 0;
  // conjugate-gradient chunks: <= 1024 vertices, never straddling graphs
  constexpr int64_t kCgChunk = 1024;
  std::vector<int64_t> cb, ce;
  std::vector<int32_t> cgr, goff(static_cast<size_t>(G) + 1, 0);
  for (int32_t k = 0; k < G; ++k) {
    for (int64_t a = g->voff_h[size_t(k)]; a < g->voff_h[size_t(k) + 1]; a += kCgChunk) {
      cb.push_back(a);
      ce.push_back(std::min(a + kCgChunk, g->voff_h[size_t(k) + 1]));
      cgr.push_back(k);
    }
    goff[size_t(k) + 1] = int32_t(cb.size());
  }
  std::vector<void*> tmp;
  auto talloc = [&](void** ptr, size_t bytes) {
    pgo_status s = dalloc_bytes(g, ptr, bytes);
    if (s == PGO_OK) tmp.push_back(*ptr);
    return s;
  };
  auto cleanup = [&](pgo_status s) {
    (void)hipStreamSynchronize(st);
    for (void* q : tmp) dfree(g, q);
    return s;
  };
  pgo_status s;
  uint8_t* d_anchor = nullptr;
  int64_t *d_cb = nullptr, *d_ce = nullptr;
  int32_t *d_cgr = nullptr, *d_goff = nullptr;
  double *R9 = nullptr, *given = nullptr, *Rp = nullptr, *rhs = nullptr, *diag = nullptr,
         *part = nullptr;
  double* vec[5] = {};
  double* sc[4] = {};
  int32_t *act = nullptr, *its = nullptr;
  if ((s = upload(g, &d_anchor, anchor.data(), anchor.size())) != PGO_OK) return s;
  tmp.push_back(d_anchor);
  if ((s = upload(g, &d_cb, cb.data(), cb.size())) != PGO_OK) return cleanup(s);
  tmp.push_back(d_cb);
  if ((s = upload(g, &d_ce, ce.data(), ce.size())) != PGO_OK) return cleanup(s);
  tmp.push_back(d_ce);
  if ((s = upload(g, &d_cgr, cgr.data(), cgr.size())) != PGO_OK) return cleanup(s);
  tmp.push_back(d_cgr);
  if ((s = upload(g, &d_goff, goff.data(), goff.size())) != PGO_OK) return cleanup(s);
  tmp.push_back(d_goff);
  const size_t nn = size_t(std::max<int64_t>(n, 1)), mm = size_t(std::max<int64_t>(m, 1));
  if ((s = talloc(reinterpret_cast<void**>(&given), 72 * nn)) != PGO_OK) return cleanup(s);
  if ((s = talloc(reinterpret_cast<void**>(&Rp), 72 * nn)) != PGO_OK) return cleanup(s);
  if ((s = talloc(reinterpret_cast<void**>(&rhs), 24 * nn)) != PGO_OK) return cleanup(s);
  if ((s = talloc(reinterpret_cast<void**>(&diag), 8 * nn)) != PGO_OK) return cleanup(s);
  if ((s = talloc(reinterpret_cast<void**>(&part), 8 * std::max<size_t>(cb.size(), 1))) != PGO_OK)
    return cleanup(s);
  for (double*& v : vec)
    if ((s = talloc(reinterpret_cast<void**>(&v), 72 * nn)) != PGO_OK) return cleanup(s);
  for (double*& v : sc)
    if ((s = talloc(reinterpret_cast<void**>(&v), 8 * size_t(G))) != PGO_OK) return cleanup(s);
  if ((s = talloc(reinterpret_cast<void**>(&act), 4 * size_t(G))) != PGO_OK) return cleanup(s);
  if ((s = talloc(reinterpret_cast<void**>(&its), 4 * size_t(G))) != PGO_OK) return cleanup(s);
  // measured rotations (caller order) and the given, projected rotations
  if (g->chordal) {
    R9 = g->R9;
    HIPCHK(launch_copy(given, g->P0, 72 * size_t(n), st));
  } else {
    if ((s = talloc(reinterpret_cast<void**>(&R9), 72 * mm)) != PGO_OK) return cleanup(s);
    HIPCHK(launch_cinit_qmat(m, g->qe, R9, st));
    HIPCHK(launch_cinit_qmat(n, g->p0, given, st));
  }
  double *o_wR = nullptr, *i_wR = nullptr, *o_w = nullptr, *i_w = nullptr;
  if ((s = talloc(reinterpret_cast<void**>(&o_wR), 72 * mm)) != PGO_OK) return cleanup(s);
  if ((s = talloc(reinterpret_cast<void**>(&i_wR), 72 * mm)) != PGO_OK) return cleanup(s);
  if ((s = talloc(reinterpret_cast<void**>(&o_w), 8 * mm)) != PGO_OK) return cleanup(s);
  if ((s = talloc(reinterpret_cast<void**>(&i_w), 8 * mm)) != PGO_OK) return cleanup(s);
  CinitGraph c{g->o_ptr, g->o_nbr, g->o_perm, g->i_ptr, g->i_nbr, g->i_perm, g->kappa, R9,
               g->tm, diag, d_anchor, o_wR, i_wR, o_w, i_w};
  CinitVec v{vec[0], vec[1], vec[2], vec[3], vec[4]};
  CinitChunks ch{d_cb, d_ce, d_cgr, d_goff, int(cb.size()), part};
  CinitScalars S{sc[0], sc[1], sc[2], sc[3], act, its};
  std::vector<int32_t> hact(static_cast<size_t>(G));
  // 1. relaxed rotations from the given ones
  HIPCHK(launch_copy(v.x, given, 72 * size_t(n), st));
  HIPCHK(launch_cinit_diag(c, int32_t(n), st));
  HIPCHK(launch_cinit_edges(c, m, 9, st));
  hipError_t he = launch_cinit_cg(c, v, ch, 9, nullptr, max_iters, 32, tol, S, G, hact.data(), st);
  if (he != hipSuccess) return cleanup(hip_fail(he, "chordal init (rotations)"));
  std::vector<int32_t> h1(static_cast<size_t>(G));
  HIPCHK(hipMemcpyAsync(h1.data(), its, 4 * size_t(G), hipMemcpyDeviceToHost, st));
  // 2. projection onto SO(3)
  HIPCHK(launch_cinit_project(int32_t(n), d_anchor, v.x, given, Rp, st));
  // 3. translations from the given ones
  c.wt = g->tau;
  HIPCHK(launch_copy(v.x, g->t0dev, 24 * size_t(n), st));
  HIPCHK(launch_cinit_diag(c, int32_t(n), st));
  HIPCHK(launch_cinit_edges(c, m, 3, st));
  HIPCHK(launch_cinit_rhs_t(c, int32_t(n), Rp, rhs, st));
  he = launch_cinit_cg(c, v, ch, 3, rhs, max_iters, 32, tol, S, G, hact.data(), st);
  if (he != hipSuccess) return cleanup(hip_fail(he, "chordal init (translations)"));
  std::vector<int32_t> h2(static_cast<size_t>(G));
  HIPCHK(hipMemcpyAsync(h2.data(), its, 4 * size_t(G), hipMemcpyDeviceToHost, st));
  HIPCHK(hipStreamSynchronize(st));
  // install the new initial point
  HIPCHK(launch_copy(g->t0dev, v.x, 24 * size_t(n), st));
  if (g->chordal) {
    HIPCHK(launch_copy(g->P0, Rp, 72 * size_t(n), st));
  } else {
    uint8_t* bad = nullptr;
    if ((s = talloc(reinterpret_cast<void**>(&bad), nn)) != PGO_OK) return cleanup(s);
    HIPCHK(launch_rot_to_quat(Rp, n, g->p0, 1, bad, st));
    HIPCHK(launch_align(g->p0, g->qe0, g->ei, g->ej, m, st));  // edge signs aligned against the new p^0
    if (m) HIPCHK(launch_perturb(m, g->qe0, g->omega, g->qe, st));
    s = g->opt.precision == PGO_FP64 ? refill_edges<double>(g) : refill_edges<float>(g);
    if (s != PGO_OK) return cleanup(s);
  }
  s = cleanup(PGO_OK);
  if (s != PGO_OK) return s;
  if ((s = pgo_reset_state(g)) != PGO_OK) return s;
  std::vector<double> r;
  if ((s = reduce(g, r)) != PGO_OK) return s;  // non-finite result -> PGO_ENUMERIC
  if (iters)
    for (int32_t k = 0; k < G; ++k) {
      iters[2 * size_t(k)] = h1[size_t(k)];
      iters[2 * size_t(k) + 1] = h2[size_t(k)];
    }
  return PGO_OK;
}

pgo_status pgo_get_state_dev(pgo_graph* g, double* state_dev) {
  if (!g || !state_dev) return fail(PGO_EINVAL, "NULL argument");
  HIPCHK(hipSetDevice(g->device));
  hipError_t he = state_io(g, state_dev, 0);
  if (he != hipSuccess) return hip_fail(he, "state_io");
  return PGO_OK;
}

pgo_status pgo_forward_record(pgo_graph* g, int32_t K, double beta, double gamma, int32_t C) {
  if (!g) return fail(PGO_EINVAL, "handle is NULL");
  pgo_status qs = quaternion_only(g, "pgo_forward_record");
  if (qs != PGO_OK) return qs;
  if (K < 1 || C < 1) return fail(PGO_EINVAL, "K and C must be >= 1");
  if (!(std::isfinite(beta) && beta > 0.0)) return fail(PGO_EINVAL, "beta must be finite and > 0");
  if (!(gamma > 0.0 && gamma < 2.0)) return fail(PGO_EINVAL, "gamma must lie in (0, 2)");
  HIPCHK(hipSetDevice(g->device));
  const int nseg = (K + C - 1) / C;
  // checkpoints 0..nseg (the last is x^K), then C+1 segment snapshots
  pgo_status s = ensure_sets(g, size_t(nseg + 1) + size_t(C) + 1);
  if (s != PGO_OK) return s;
  void* cur[6];
  state_ptrs(g, cur);
  const int block = g->sched == PGO_SCHED_GRAPH ? g->block_graph : g->block_phase;
  for (int seg = 0; seg < nseg; ++seg) {
    if ((s = copy_state(g, &g->sets[6 * size_t(seg)], cur)) != PGO_OK) return s;
    const int L = std::min(K, (seg + 1) * C) - seg * C;
    if ((s = iterate_with(g, L, beta, gamma, g->sched, block)) != PGO_OK) return s;
  }
  if ((s = copy_state(g, &g->sets[6 * size_t(nseg)], cur)) != PGO_OK) return s;
  g->rec_K = K;
  g->rec_C = C;
  g->rec_beta = beta;
  g->rec_gamma = gamma;
  ++g->rec_id;
  return PGO_OK;
}

pgo_status pgo_record_id(pgo_graph* g, int64_t* id) {
  if (!g || !id) return fail(PGO_EINVAL, "NULL argument");
  *id = g->rec_K >= 1 ? g->rec_id : -1;
  return PGO_OK;
}

pgo_status pgo_adjoint(pgo_graph* g, const double* dL_dstate, double* g_kappa, double* g_tau,
                       double* g_tm, double* g_omega, double* dL_dstate0) {
  if (!g || !dL_dstate) return fail(PGO_EINVAL, "NULL argument");
  pgo_status qs = quaternion_only(g, "pgo_adjoint");
  if (qs != PGO_OK) return qs;
  if (g->rec_K < 1) return fail(PGO_ESTATE, "no recorded forward pass (call pgo_forward_record)");
  HIPCHK(hipSetDevice(g->device));
  pgo_status s = ensure_adjoint_buffers(g);
  if (s != PGO_OK) return s;
  return g->opt.precision == PGO_FP64
             ? adjoint_impl<double>(g, dL_dstate, g_kappa, g_tau, g_tm, g_omega, dL_dstate0)
             : adjoint_impl<float>(g, dL_dstate, g_kappa, g_tau, g_tm, g_omega, dL_dstate0);
}

void pgo_destroy(pgo_graph* g) {
  if (!g) return;
  (void)hipSetDevice(g->device);
  if (g->stream) (void)hipStreamSynchronize(g->stream);
  if (g->gexec) (void)hipGraphExecDestroy(g->gexec);
  for (void* p : g->allocs) (void)hipFree(p);
  if (g->own_stream) (void)hipStreamDestroy(g->own_stream);
  delete g;
}

}  // extern "C"
