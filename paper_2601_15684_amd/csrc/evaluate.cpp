// The FP64 per-graph reductions (cost, residuals, L_beta and merit) and
// their entry points, the no-allocation one included.
#include "handle.hpp"

using namespace pgo;
using namespace pgo::host;

namespace pgo {
namespace host {

namespace {

// the reductions read the out-ordered copy of the FP64 edges: a chunk's
// edges then gather their tails' state in order
EdgeF64 reduction_view(const pgo_graph* g) {
  return EdgeF64{g->r_ei, g->r_ej,  g->r_qe, g->r_tm, g->r_kappa, g->r_tau,
                 g->chordal ? g->r_X9 : nullptr, g->aniso ? g->r_X9 : nullptr};
}

}  // namespace

// Per-graph reduction values (RedIdx order).  Unless allow_nonfinite, a
// non-finite value anywhere is reported as PGO_ENUMERIC.
// active (device, G flags) restricts the work to the graphs flagged 1; the
// others report zeros.
pgo_status reduce(pgo_graph* g, std::vector<double>& out, bool allow_nonfinite,
                  const int32_t* active) {
  HIPCHK(hipSetDevice(g->device));
  const EdgeF64 e = reduction_view(g);
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

// L_beta (PRADMM section) and the merit of Theorem 1 without its unknown
// proximal-difference terms, from one graph's reduction values.
void merit_of(const double* v, double beta, double gamma, double* L, double* psi) {
  const double a1 = std::fabs(1.0 - gamma) / (1.0 - std::fabs(1.0 - gamma));
  *L = v[kSplit] - v[kLamPQ] + 0.5 * beta * v[kPQ2] - v[kZTS] + 0.5 * beta * v[kTS2];
  *psi = *L + a1 / (gamma * beta) * v[kDL2];
}

}  // namespace host
}  // namespace pgo

extern "C" {

pgo_status pgo_merit(pgo_graph* g, double* out) {
  if (!g || !out) return fail(PGO_EINVAL, "NULL argument");
  return pgo_evaluate(g, nullptr, nullptr, out);
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
  const EdgeF64 e = reduction_view(g);
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

}  // extern "C"
