// Reverse mode through K unrolled sweeps (quaternion model): edge
// parameters on the device, the recorded forward pass with checkpoints, and
// the hand-written adjoint.
#include "handle.hpp"

using namespace pgo;
using namespace pgo::host;

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

extern "C" {

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

}  // extern "C"
