// Handle creation and options: argument checking, device allocation, the
// boundary preparation sequence (projection, conversion, sign alignment,
// CSR/CSC build, per-vertex constants), schedule defaults, and teardown.
#include "handle.hpp"

using namespace pgo;
using namespace pgo::host;

namespace {

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
  // cQ for every model; cT, cS for the quaternion model's reverse sweeps
  void** c1[] = {&g->cQ, &g->cT, &g->cS};
  for (void** v : c1) {
    if (g->chordal && v != &g->cQ) continue;
    if ((s = dalloc_bytes(g, v, sizeof(T) * n)) != PGO_OK) return s;
  }
  if (g->aniso) {
    void** es[] = {&g->o_Sa, &g->o_Sb, &g->i_Sa, &g->i_Sb};
    for (void** v : es)
      if ((s = dalloc_bytes(g, v, 3 * sizeof(T) * m)) != PGO_OK) return s;
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
    HIPCHK(launch_vertex_consts_c<T>(int32_t(g->n), g->o_ptr, g->o_perm, g->kappa,
                                     static_cast<T*>(g->cQ), st));
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
  if ((s = reduction_edges(g)) != PGO_OK) return bail(s);
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

const char* pgo_last_error(void) { return last_error(); }

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
