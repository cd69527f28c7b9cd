// Host side of the chordal initialisation: per-graph conjugate-gradient
// control over the kernels of cinit.hip, then the new initial point.
#include "handle.hpp"

using namespace pgo;
using namespace pgo::host;

extern "C" {

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

}  // extern "C"
