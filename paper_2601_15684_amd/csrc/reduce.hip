// FP64 reductions per graph: the cost of model (1) at (p, t) (or the
// chordal cost at (P, t)) and the residual sums behind App. E.1's iteration
// residual.  Work is cut into
// chunks that never straddle two graphs; each workgroup reduces one chunk
// with a fixed-shape tree, then one thread per graph adds its chunks in
// order.  No atomics, so every run gives the same bits.
//
// Multiply-adds are not contracted here: the device form of the residuals
// and the merit (pgo_evaluate_noalloc) rounds as the host's.
#pragma clang fp contract(off)
#include <mutex>

#include "internal.hpp"

namespace pgo {

namespace {

constexpr int kRB = 256;

template <int K>
__device__ void block_sum(double (&v)[K], double (*sh)[kRB]) {
  for (int k = 0; k < K; ++k) sh[k][threadIdx.x] = v[k];
  __syncthreads();
  for (int w = kRB / 2; w > 0; w >>= 1) {
    if (threadIdx.x < w)
      for (int k = 0; k < K; ++k) sh[k][threadIdx.x] += sh[k][threadIdx.x + w];
    __syncthreads();
  }
  for (int k = 0; k < K; ++k) v[k] = sh[k][0];
}

// |r|^2_{Sigma1} of a translation residual r = (r0, r1, r2, r3): tau |r|^2,
// or with a full information matrix c r0^2 + r_v^T S r_v (c = trace(S) / 3)
__device__ __forceinline__ double weighted_r(const EdgeF64& E, int64_t e, double r0, double r1,
                                             double r2, double r3) {
  if (!E.S9) return E.tau[e] * (r0 * r0 + r1 * r1 + r2 * r2 + r3 * r3);
  const double* S = E.S9 + 9 * e;
  const double c = (S[0] + S[4] + S[8]) / 3.0;
  return c * r0 * r0 + r1 * (S[0] * r1 + S[1] * r2 + S[2] * r3) +
         r2 * (S[3] * r1 + S[4] * r2 + S[5] * r3) + r3 * (S[6] * r1 + S[7] * r2 + S[8] * r3);
}

// cost term of edge e (model (1), Sigma1 = tau I_4 or diag(c, S), Sigma2 = kappa I_4)
template <typename T>
__device__ double edge_cost(const DevGraph<T>& g, const EdgeF64& E, int64_t e) {
  const int i = E.ei[e], j = E.ej[e];
  const Q4<double> pi = cvt<double>(g.p[i]), pj = cvt<double>(g.p[j]);
  const V3<T> ti = g.t[i], tj = g.t[j];
  const V3<double> tt = {E.tm[3 * e], E.tm[3 * e + 1], E.tm[3 * e + 2]};
  const Q4<double> rot = qmul(qmul_vp(pi, tt), qconj(pi));  // p_i [0, t~] p_i^*
  const double r0 = -rot.w;
  const double r1 = (double(tj.x) - double(ti.x)) - rot.x;
  const double r2 = (double(tj.y) - double(ti.y)) - rot.y;
  const double r3 = (double(tj.z) - double(ti.z)) - rot.z;
  const Q4<double> a = qmul(qmul(qconj(pj), pi), E.q[e]);  // p_j^* p_i q~
  const double a0 = a.w - 1.0;
  return weighted_r(E, e, r0, r1, r2, r3) +
         E.kappa[e] * (a0 * a0 + a.x * a.x + a.y * a.y + a.z * a.z);
}

// f + g of the split model (eq. 2) for edge e = (i -> j):
// tau |[0, t_j - s_i] - q_i [0, t~] p_i^*|^2 + kappa |p_j^* q_i q~ - 1|^2
template <typename T>
__device__ double edge_split(const DevGraph<T>& g, const EdgeF64& E, int64_t e) {
  const int i = E.ei[e], j = E.ej[e];
  const Q4<double> pi = cvt<double>(g.p[i]), qi = cvt<double>(g.q[i]), pj = cvt<double>(g.p[j]);
  const V3<T> si = g.s[i], tj = g.t[j];
  const V3<double> tt = {E.tm[3 * e], E.tm[3 * e + 1], E.tm[3 * e + 2]};
  const Q4<double> rot = qmul(qmul_vp(qi, tt), qconj(pi));  // q_i [0, t~] p_i^*
  const double r0 = -rot.w;
  const double r1 = (double(tj.x) - double(si.x)) - rot.x;
  const double r2 = (double(tj.y) - double(si.y)) - rot.y;
  const double r3 = (double(tj.z) - double(si.z)) - rot.z;
  const Q4<double> a = qmul(qmul(qconj(pj), qi), E.q[e]);
  const double a0 = a.w - 1.0;
  return weighted_r(E, e, r0, r1, r2, r3) +
         E.kappa[e] * (a0 * a0 + a.x * a.x + a.y * a.y + a.z * a.z);
}

// Chunks of graphs whose flag is 0 skip their work (partials 0), when
// active is given; chunk c belongs to graph gid[c].
struct ChunkMask {
  const int32_t* gid;
  const int32_t* active;
  __device__ __forceinline__ bool skip(int c) const { return active && !active[gid[c]]; }
};

template <typename T>
__global__ void __launch_bounds__(kRB) k_red_edges(DevGraph<T> g, EdgeF64 E,
                                                    const int64_t* __restrict__ beg,
                                                    const int64_t* __restrict__ end,
                                                    ChunkMask mask, double* __restrict__ partial) {
  __shared__ double sh[kEdgeVals][kRB];
  double v[kEdgeVals] = {0.0, 0.0};
  const int c = blockIdx.x;
  const int64_t stop = mask.skip(c) ? beg[c] : end[c];
  int64_t e = beg[c] + threadIdx.x;
  for (; e + kRB < stop; e += 2 * kRB) {  // two edges' loads in flight, added in order
    const double c0 = edge_cost(g, E, e), s0 = edge_split(g, E, e);
    const double c1 = edge_cost(g, E, e + kRB), s1 = edge_split(g, E, e + kRB);
    v[0] += c0;
    v[1] += s0;
    v[0] += c1;
    v[1] += s1;
  }
  for (; e < stop; e += kRB) {
    v[0] += edge_cost(g, E, e);
    v[1] += edge_split(g, E, e);
  }
  block_sum<kEdgeVals>(v, sh);
  if (threadIdx.x == 0)
    for (int k = 0; k < kEdgeVals; ++k) partial[kEdgeVals * int64_t(c) + k] = v[k];
}

template <typename T, typename V>
__device__ __forceinline__ double d2(const V& a, const V& b) {
  const double x = double(a.x) - double(b.x), y = double(a.y) - double(b.y),
               z = double(a.z) - double(b.z);
  return x * x + y * y + z * z;
}

template <typename T>
__device__ __forceinline__ double d2q(const Q4<T>& a, const Q4<T>& b) {
  const double w = double(a.w) - double(b.w);
  return w * w + d2<T, Q4<T>>(a, b);
}

// <l, a - b> for 4-vectors and 3-vectors
template <typename T>
__device__ __forceinline__ double dotq(const Q4<T>& l, const Q4<T>& a, const Q4<T>& b) {
  return double(l.w) * (double(a.w) - double(b.w)) + double(l.x) * (double(a.x) - double(b.x)) +
         double(l.y) * (double(a.y) - double(b.y)) + double(l.z) * (double(a.z) - double(b.z));
}

template <typename V>
__device__ __forceinline__ double dot3(const V& l, const V& a, const V& b) {
  return double(l.x) * (double(a.x) - double(b.x)) + double(l.y) * (double(a.y) - double(b.y)) +
         double(l.z) * (double(a.z) - double(b.z));
}

template <typename T>
__global__ void __launch_bounds__(kRB) k_red_vertices(DevGraph<T> g, int have_prev,
                                                       const int64_t* __restrict__ beg,
                                                       const int64_t* __restrict__ end,
                                                       ChunkMask mask,
                                                       double* __restrict__ partial) {
  __shared__ double sh[kVertVals][kRB];
  double v[kVertVals] = {0, 0, 0, 0, 0, 0, 0, 0, 0};
  const int c = blockIdx.x;
  const int64_t stop = mask.skip(c) ? beg[c] : end[c];
  for (int64_t i = beg[c] + threadIdx.x; i < stop; i += kRB) {
    v[0] += d2q(g.p[i], g.q[i]);
    v[1] += d2<T, V3<T>>(g.t[i], g.s[i]);
    v[7] += dotq(g.lam[i], g.p[i], g.q[i]);
    v[8] += dot3(g.z[i], g.t[i], g.s[i]);
    if (have_prev) {
      v[2] += d2q(g.lam[i], g.lam_prev[i]);
      v[3] += d2<T, V3<T>>(g.z[i], g.z_prev[i]);
      v[4] += d2q(g.q[i], g.q_prev[i]);
      v[5] += d2<T, V3<T>>(g.t[i], g.t_prev[i]);
      v[6] += d2<T, V3<T>>(g.s[i], g.s_prev[i]);
    }
  }
  block_sum<kVertVals>(v, sh);
  if (threadIdx.x == 0)
    for (int k = 0; k < kVertVals; ++k) partial[kVertVals * int64_t(c) + k] = v[k];
}

__global__ void k_red_finish(const double* __restrict__ pe, const double* __restrict__ pv,
                             const int32_t* __restrict__ g_ec_off,
                             const int32_t* __restrict__ g_vc_off, int G, double* __restrict__ out) {
  const int gr = blockIdx.x * blockDim.x + threadIdx.x;
  if (gr >= G) return;
  double c[kEdgeVals] = {0.0, 0.0};
  for (int k = g_ec_off[gr]; k < g_ec_off[gr + 1]; ++k)
    for (int q = 0; q < kEdgeVals; ++q) c[q] += pe[kEdgeVals * int64_t(k) + q];
  double v[kVertVals] = {0, 0, 0, 0, 0, 0, 0, 0, 0};
  for (int k = g_vc_off[gr]; k < g_vc_off[gr + 1]; ++k)
    for (int q = 0; q < kVertVals; ++q) v[q] += pv[kVertVals * int64_t(k) + q];
  for (int q = 0; q < kEdgeVals; ++q) out[kRedVals * int64_t(gr) + q] = c[q];
  for (int q = 0; q < kVertVals; ++q) out[kRedVals * int64_t(gr) + kEdgeVals + q] = v[q];
}

// --- chordal model -----------------------------------------------------------
template <typename T>
__device__ __forceinline__ void rowsd(const R3<T>& m, double o[9]) {
  for (int r = 0; r < 3; ++r) {
    o[3 * r] = double(m.r[r].x);
    o[3 * r + 1] = double(m.r[r].y);
    o[3 * r + 2] = double(m.r[r].z);
  }
}

// tau |a_j - b_i - A_i t~|^2 + kappa |B_i R~ - P_j|_F^2: the cost with
// (A, B, b) = (P, P, t), the split f + g with (A, B, b) = (P, Q, s).
template <typename T>
__device__ double edge_chordal(const EdgeF64& E, int64_t e, const R3<T>& Ai_, const R3<T>& Bi_,
                               const R3<T>& Pj_, const V3<T>& bi, const V3<T>& tj) {
  double A[9], B[9], Pj[9];
  rowsd(Ai_, A);
  rowsd(Bi_, B);
  rowsd(Pj_, Pj);
  const double* Rm = E.R9 + 9 * e;
  const double u[3] = {E.tm[3 * e], E.tm[3 * e + 1], E.tm[3 * e + 2]};
  const double d[3] = {double(tj.x) - double(bi.x), double(tj.y) - double(bi.y),
                       double(tj.z) - double(bi.z)};
  double rt = 0.0, rr = 0.0;
  for (int r = 0; r < 3; ++r) {
    const double x = d[r] - (A[3 * r] * u[0] + A[3 * r + 1] * u[1] + A[3 * r + 2] * u[2]);
    rt += x * x;
    for (int c = 0; c < 3; ++c) {
      const double y = B[3 * r] * Rm[c] + B[3 * r + 1] * Rm[3 + c] + B[3 * r + 2] * Rm[6 + c] -
                       Pj[3 * r + c];
      rr += y * y;
    }
  }
  return E.tau[e] * rt + E.kappa[e] * rr;
}

template <typename T>
__global__ void __launch_bounds__(kRB) k_red_edges_c(DevChordal<T> g, EdgeF64 E,
                                                      const int64_t* __restrict__ beg,
                                                      const int64_t* __restrict__ end,
                                                      ChunkMask mask,
                                                      double* __restrict__ partial) {
  __shared__ double sh[kEdgeVals][kRB];
  double v[kEdgeVals] = {0.0, 0.0};
  const int c = blockIdx.x;
  const int64_t stop = mask.skip(c) ? beg[c] : end[c];
  auto both = [&](int64_t e, double& f, double& fs) {
    const int i = E.ei[e], j = E.ej[e];
    const R3<T> Pi = g.P[i], Pj = g.P[j];
    f = edge_chordal(E, e, Pi, Pi, Pj, g.t[i], g.t[j]);
    fs = edge_chordal(E, e, Pi, g.Q[i], Pj, g.s[i], g.t[j]);
  };
  int64_t e = beg[c] + threadIdx.x;
  for (; e + kRB < stop; e += 2 * kRB) {  // two edges' loads in flight, added in order
    double c0, s0, c1, s1;
    both(e, c0, s0);
    both(e + kRB, c1, s1);
    v[0] += c0;
    v[1] += s0;
    v[0] += c1;
    v[1] += s1;
  }
  for (; e < stop; e += kRB) {
    double c0, s0;
    both(e, c0, s0);
    v[0] += c0;
    v[1] += s0;
  }
  block_sum<kEdgeVals>(v, sh);
  if (threadIdx.x == 0)
    for (int k = 0; k < kEdgeVals; ++k) partial[kEdgeVals * int64_t(c) + k] = v[k];
}

template <typename T>
__device__ __forceinline__ double d2m(const R3<T>& a, const R3<T>& b) {
  double s = 0.0;
  for (int r = 0; r < 3; ++r) s += d2<T, V3<T>>(a.r[r], b.r[r]);
  return s;
}

template <typename T>
__device__ __forceinline__ double dotm(const R3<T>& l, const R3<T>& a, const R3<T>& b) {
  double s = 0.0;
  for (int r = 0; r < 3; ++r) s += dot3(l.r[r], a.r[r], b.r[r]);
  return s;
}

template <typename T>
__global__ void __launch_bounds__(kRB) k_red_vertices_c(DevChordal<T> g, int have_prev,
                                                         const int64_t* __restrict__ beg,
                                                         const int64_t* __restrict__ end,
                                                         ChunkMask mask,
                                                         double* __restrict__ partial) {
  __shared__ double sh[kVertVals][kRB];
  double v[kVertVals] = {0, 0, 0, 0, 0, 0, 0, 0, 0};
  const int c = blockIdx.x;
  const int64_t stop = mask.skip(c) ? beg[c] : end[c];
  for (int64_t i = beg[c] + threadIdx.x; i < stop; i += kRB) {
    v[0] += d2m(g.P[i], g.Q[i]);
    v[1] += d2<T, V3<T>>(g.t[i], g.s[i]);
    v[7] += dotm(g.L[i], g.P[i], g.Q[i]);
    v[8] += dot3(g.z[i], g.t[i], g.s[i]);
    if (have_prev) {
      v[2] += d2m(g.L[i], g.L_prev[i]);
      v[3] += d2<T, V3<T>>(g.z[i], g.z_prev[i]);
      v[4] += d2m(g.Q[i], g.Q_prev[i]);
      v[5] += d2<T, V3<T>>(g.t[i], g.t_prev[i]);
      v[6] += d2<T, V3<T>>(g.s[i], g.s_prev[i]);
    }
  }
  block_sum<kVertVals>(v, sh);
  if (threadIdx.x == 0)
    for (int k = 0; k < kVertVals; ++k) partial[kVertVals * int64_t(c) + k] = v[k];
}

}  // namespace

template <typename T>
hipError_t launch_reduce_c(const DevChordal<T>& g, const EdgeF64& e, int have_prev,
                           const int32_t* ec_graph, const int64_t* ec_beg, const int64_t* ec_end,
                           int n_echunks, const int32_t* vc_graph, const int64_t* vc_beg,
                           const int64_t* vc_end, int n_vchunks, double* partial_e,
                           double* partial_v, const int32_t* g_ec_off, const int32_t* g_vc_off,
                           int G, double* out, const int32_t* active, hipStream_t st) {
  if (n_echunks > 0)
    hipLaunchKernelGGL((k_red_edges_c<T>), dim3(n_echunks), dim3(kRB), 0, st, g, e, ec_beg, ec_end,
                       ChunkMask{ec_graph, active}, partial_e);
  if (n_vchunks > 0)
    hipLaunchKernelGGL((k_red_vertices_c<T>), dim3(n_vchunks), dim3(kRB), 0, st, g, have_prev,
                       vc_beg, vc_end, ChunkMask{vc_graph, active}, partial_v);
  hipLaunchKernelGGL(k_red_finish, dim3((G + 255) / 256), dim3(256), 0, st, partial_e, partial_v,
                     g_ec_off, g_vc_off, G, out);
  return hipGetLastError();
}

template hipError_t launch_reduce_c<float>(const DevChordal<float>&, const EdgeF64&, int,
                                           const int32_t*, const int64_t*, const int64_t*, int,
                                           const int32_t*, const int64_t*, const int64_t*, int,
                                           double*, double*, const int32_t*, const int32_t*, int,
                                           double*, const int32_t*, hipStream_t);
template hipError_t launch_reduce_c<double>(const DevChordal<double>&, const EdgeF64&, int,
                                            const int32_t*, const int64_t*, const int64_t*, int,
                                            const int32_t*, const int64_t*, const int64_t*, int,
                                            double*, double*, const int32_t*, const int32_t*, int,
                                            double*, const int32_t*, hipStream_t);

template <typename T>
hipError_t launch_reduce(const DevGraph<T>& g, const EdgeF64& e, int have_prev,
                         const int32_t* ec_graph, const int64_t* ec_beg, const int64_t* ec_end,
                         int n_echunks, const int32_t* vc_graph, const int64_t* vc_beg,
                         const int64_t* vc_end, int n_vchunks, double* partial_e,
                         double* partial_v, const int32_t* g_ec_off, const int32_t* g_vc_off,
                         int G, double* out, const int32_t* active, hipStream_t st) {
  if (n_echunks > 0)
    hipLaunchKernelGGL((k_red_edges<T>), dim3(n_echunks), dim3(kRB), 0, st, g, e, ec_beg, ec_end,
                       ChunkMask{ec_graph, active}, partial_e);
  if (n_vchunks > 0)
    hipLaunchKernelGGL((k_red_vertices<T>), dim3(n_vchunks), dim3(kRB), 0, st, g, have_prev,
                       vc_beg, vc_end, ChunkMask{vc_graph, active}, partial_v);
  hipLaunchKernelGGL(k_red_finish, dim3((G + 255) / 256), dim3(256), 0, st, partial_e, partial_v,
                     g_ec_off, g_vc_off, G, out);
  return hipGetLastError();
}

template hipError_t launch_reduce<float>(const DevGraph<float>&, const EdgeF64&, int,
                                         const int32_t*, const int64_t*, const int64_t*, int,
                                         const int32_t*, const int64_t*, const int64_t*, int,
                                         double*, double*, const int32_t*, const int32_t*, int,
                                         double*, const int32_t*, hipStream_t);
template hipError_t launch_reduce<double>(const DevGraph<double>&, const EdgeF64&, int,
                                          const int32_t*, const int64_t*, const int64_t*, int,
                                          const int32_t*, const int64_t*, const int64_t*, int,
                                          double*, double*, const int32_t*, const int32_t*, int,
                                          double*, const int32_t*, hipStream_t);

// ---------------------------------------------------------------------------
// The reductions with their partial sums and per-graph values in a static
// device array (for callers that cannot allocate; see pgo_evaluate_noalloc):
// `scratch` lives on every device the library runs on until the process
// ends.  Every chunk writes its own partials and every graph its own values,
// so nothing needs clearing between calls; calls that overlap on one device
// race on the array.
// ---------------------------------------------------------------------------
__device__ __align__(256) double scratch[kScratchDoubles];

namespace {

// L_beta and the merit (as merit_of on the host, the same operations in the
// same order) and the residuals of one graph's reduction values
__global__ void k_eval_finish(const double* __restrict__ red, const double* __restrict__ beta,
                              double gamma, int G, double* __restrict__ out) {
  const int gr = blockIdx.x * blockDim.x + threadIdx.x;
  if (gr >= G) return;
  const double* v = red + kRedVals * int64_t(gr);
  const double b = beta[gr];
  double* o = out + kEvalVals * int64_t(gr);
  o[0] = v[kCost];
  o[1] = sqrt(v[kPQ2]);
  o[2] = sqrt(v[kTS2]);
  o[3] = (v[kDL2] + v[kDZ2]) / b + b * (v[kDQ2] + v[kDT2]);
  o[4] = b * sqrt(v[kDQ2]);
  o[5] = b * sqrt(v[kDS2]);
  const double a1 = fabs(1.0 - gamma) / (1.0 - fabs(1.0 - gamma));
  const double L = v[kSplit] - v[kLamPQ] + 0.5 * b * v[kPQ2] - v[kZTS] + 0.5 * b * v[kTS2];
  o[6] = L;
  o[7] = L + a1 / (gamma * b) * v[kDL2];
}

std::mutex g_scratch_mu;
double* g_scratch_ptr[64] = {};

}  // namespace

hipError_t scratch_address(int device, double** ptr) {
  if (device < 0 || device >= 64) return hipErrorInvalidDevice;
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_ptr[device]) {
    int cur = 0;
    hipError_t e = hipGetDevice(&cur);
    if (e != hipSuccess) return e;
    if (cur != device && (e = hipSetDevice(device)) != hipSuccess) return e;
    void* p = nullptr;
    e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (cur != device) (void)hipSetDevice(cur);
    if (e != hipSuccess) return e;
    g_scratch_ptr[device] = static_cast<double*>(p);
  }
  *ptr = g_scratch_ptr[device];
  return hipSuccess;
}

template <typename T>
hipError_t launch_evaluate_noalloc(const DevGraph<T>& g, const EdgeF64& e, int have_prev,
                                   const int32_t* ec_graph, const int64_t* ec_beg,
                                   const int64_t* ec_end, int n_echunks, const int32_t* vc_graph,
                                   const int64_t* vc_beg, const int64_t* vc_end, int n_vchunks,
                                   const int32_t* g_ec_off, const int32_t* g_vc_off, int G,
                                   double* scr, const double* beta, double gamma, double* out,
                                   hipStream_t st) {
  double* pe = scr;
  double* pv = pe + size_t(kEdgeVals) * n_echunks;
  double* red = pv + size_t(kVertVals) * n_vchunks;
  const hipError_t err = launch_reduce<T>(g, e, have_prev, ec_graph, ec_beg, ec_end, n_echunks,
                                          vc_graph, vc_beg, vc_end, n_vchunks, pe, pv, g_ec_off,
                                          g_vc_off, G, red, nullptr, st);
  if (err != hipSuccess) return err;
  hipLaunchKernelGGL(k_eval_finish, dim3((G + 255) / 256), dim3(256), 0, st, red, beta, gamma, G,
                     out);
  return hipGetLastError();
}

template hipError_t launch_evaluate_noalloc<float>(const DevGraph<float>&, const EdgeF64&, int,
                                                   const int32_t*, const int64_t*,
                                                   const int64_t*, int, const int32_t*,
                                                   const int64_t*, const int64_t*, int,
                                                   const int32_t*, const int32_t*, int, double*,
                                                   const double*, double, double*, hipStream_t);
template hipError_t launch_evaluate_noalloc<double>(const DevGraph<double>&, const EdgeF64&, int,
                                                    const int32_t*, const int64_t*,
                                                    const int64_t*, int, const int32_t*,
                                                    const int64_t*, const int64_t*, int,
                                                    const int32_t*, const int32_t*, int, double*,
                                                    const double*, double, double*, hipStream_t);

}  // namespace pgo
