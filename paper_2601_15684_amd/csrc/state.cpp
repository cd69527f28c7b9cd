// State transfer between the caller and the device: poses, the raw state,
// the prepared edge and vertex quaternions, and state resets.
#include "handle.hpp"

using namespace pgo;
using namespace pgo::host;

namespace pgo {
namespace host {

pgo_status ensure_iobuf(pgo_graph* g) {
  if (g->iobuf) return PGO_OK;
  return dalloc(g, &g->iobuf, size_t(state_width(g)) * g->n);
}

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

}  // namespace host
}  // namespace pgo

extern "C" {

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

pgo_status pgo_get_state_dev(pgo_graph* g, double* state_dev) {
  if (!g || !state_dev) return fail(PGO_EINVAL, "NULL argument");
  HIPCHK(hipSetDevice(g->device));
  hipError_t he = state_io(g, state_dev, 0);
  if (he != hipSuccess) return hip_fail(he, "state_io");
  return PGO_OK;
}

}  // extern "C"
