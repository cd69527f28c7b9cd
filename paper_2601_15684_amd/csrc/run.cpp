// Running sweeps: the dispatch to each model's kernels in each schedule
// (the per-phase sequence captured once into a HIP graph), per-graph
// penalties and run masks, the stopping rule, the merit-checked solve with
// per-graph undo, and the autotuner.
#include "handle.hpp"

using namespace pgo;
using namespace pgo::host;

namespace {

template <typename T>
pgo_status run_sweeps(pgo_graph* g, int32_t k, double beta, double gamma, int sched, int block,
                      bool per_graph, bool masked, bool snap_in_launch) {
  SweepParams sp{beta, gamma, g->opt.h1, g->opt.h2, g->opt.h3, g->opt.h4,
                 per_graph ? g->beta_dev : nullptr, masked ? g->active_dev : nullptr};
  if (snap_in_launch) {
    if (sched != PGO_SCHED_GRAPH || g->chordal || g->aniso)
      return fail(PGO_EINVAL, "snapshot in the launch: per-graph quaternion sweeps only");
    for (int a = 0; a < 6; ++a) sp.snap[a] = g->snap[a];
  }
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

// The snapshot arrays (allocated on first use), one per state array.
pgo_status snapshot_alloc(pgo_graph* g) {
  size_t vb[6];
  state_array_bytes(g, vb);
  for (int k = 0; k < 6; ++k)
    if (!g->snap[k]) {
      pgo_status s = dalloc_bytes(g, &g->snap[k], vb[k] * size_t(g->n));
      if (s != PGO_OK) return s;
    }
  return PGO_OK;
}

// Copies the state into the snapshot arrays: every vertex, or (active, G
// device flags) the vertices of the flagged graphs only.
pgo_status snapshot(pgo_graph* g, const int32_t* active) {
  size_t vb[6];
  state_array_bytes(g, vb);
  void* cur[6] = {g->p, g->q, g->lam, g->t, g->s, g->z};
  pgo_status s = snapshot_alloc(g);
  if (s != PGO_OK) return s;
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

namespace pgo {
namespace host {

pgo_status iterate_with(pgo_graph* g, int32_t k, double beta, double gamma, int sched, int block,
                        const double* beta_g, const int32_t* active, bool snap_in_launch) {
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
          ? run_sweeps<double>(g, k, beta, gamma, sched, block, per_graph, masked, snap_in_launch)
          : run_sweeps<float>(g, k, beta, gamma, sched, block, per_graph, masked, snap_in_launch);
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

// bytes per vertex of the six state arrays (p, q, lambda, t, s, z)
void state_array_bytes(const pgo_graph* g, size_t out[6]) {
  const size_t w = g->opt.precision == PGO_FP64 ? 8 : 4;
  for (int k = 0; k < 3; ++k) out[k] = size_t(rot_words(g)) * w;
  for (int k = 3; k < 6; ++k) out[k] = 3 * w;
}

}  // namespace host
}  // namespace pgo

extern "C" {

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
  const bool fused_snap = g->sched == PGO_SCHED_GRAPH && !g->chordal && !g->aniso;
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
    // the per-graph quaternion kernel takes the snapshot itself as it
    // starts each running graph (the state is read there anyway)
    if (adapt && (s = fused_snap ? snapshot_alloc(g) : snapshot(g, g->active_dev)) != PGO_OK)
      return s;
    if ((s = iterate_with(g, check_every, beta[0], gamma, g->sched, block, beta, active.data(),
                          adapt && fused_snap)) != PGO_OK)
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

}  // extern "C"
