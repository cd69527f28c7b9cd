// Error reporting and device allocation owned by the handle.
#include "handle.hpp"

using namespace pgo;
using namespace pgo::host;

namespace {

thread_local std::string g_err;

}  // namespace

namespace pgo {
namespace host {

pgo_status fail(pgo_status s, const std::string& msg) {
  g_err = msg;
  return s;
}

pgo_status hip_fail(hipError_t e, const char* what) {
  return fail(e == hipErrorOutOfMemory ? PGO_ENOMEM : PGO_EDEVICE,
              std::string(what) + ": " + hipGetErrorString(e));
}

const char* last_error() { return g_err.c_str(); }

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

bool finite_all(const double* a, size_t k) {
  for (size_t i = 0; i < k; ++i)
    if (!std::isfinite(a[i])) return false;
  return true;
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

pgo_status reduction_edges(pgo_graph* g) {
  const int64_t m = g->m;
  if (m <= 0) return PGO_OK;
  const double* X9 = g->chordal ? g->R9 : (g->aniso ? g->S9 : nullptr);
  if (!g->r_ei) {
    pgo_status s;
    if ((s = dalloc(g, &g->r_ei, size_t(m))) != PGO_OK) return s;
    if ((s = dalloc(g, &g->r_ej, size_t(m))) != PGO_OK) return s;
    if (g->qe && (s = dalloc(g, &g->r_qe, size_t(m))) != PGO_OK) return s;
    if ((s = dalloc(g, &g->r_tm, size_t(3 * m))) != PGO_OK) return s;
    if ((s = dalloc(g, &g->r_kappa, size_t(m))) != PGO_OK) return s;
    if ((s = dalloc(g, &g->r_tau, size_t(m))) != PGO_OK) return s;
    if (X9 && (s = dalloc(g, &g->r_X9, size_t(9 * m))) != PGO_OK) return s;
  }
  HIPCHK(launch_gather_edges_f64(g->o_perm, m, g->ei, g->ej, g->qe, g->tm, g->kappa, g->tau, X9,
                                 g->r_ei, g->r_ej, g->r_qe, g->r_tm, g->r_kappa, g->r_tau,
                                 g->r_X9, g->stream));
  return PGO_OK;
}

}  // namespace host
}  // namespace pgo
