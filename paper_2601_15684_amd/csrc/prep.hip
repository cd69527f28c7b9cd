// Boundary preparation, once per handle (FP64 throughout):
//  * every input rotation is checked (det > 0, ||R^T R - I||_F <= 1e-2),
//    projected onto SO(3) by its polar factor U V^T from a register-resident
//    one-sided Jacobi SVD, and converted to a unit quaternion (Shepperd's
//    branch on the largest diagonal combination) with the convention of
//    App. A.2, R v = Im(q [0, v] q^*);
//  * vertex quaternions get a canonical sign (first component of magnitude
//    > 1e-6 positive); edge quaternions are flipped where
//    <p_i^0 q~_e, p_j^0> < 0 so the initial poses are consistent with them;
//  * edges are sorted by tail and by head (stable radix sort, so each
//    vertex's edges keep the caller's order), CSR/CSC offsets come from a
//    lower-bound search of the sorted keys, and the SoA edge records and
//    the per-vertex constants are written in the handle's precision;
//  * the state starts at q = p^0, s = t^0, lambda = z = 0.
#include <hipcub/hipcub.hpp>

#include <algorithm>

#include "internal.hpp"
#include "polar.hpp"

namespace pgo {

namespace {

__device__ Q4<double> quat_of_rot(const double r[9]) {
  const double tr = r[0] + r[4] + r[8];
  Q4<double> q;
  if (tr >= r[0] && tr >= r[4] && tr >= r[8]) {
    const double w = 0.5 * sqrt(fmax(1.0 + tr, 0.0)), f = 0.25 / w;
    q = {w, (r[7] - r[5]) * f, (r[2] - r[6]) * f, (r[3] - r[1]) * f};
  } else if (r[0] >= r[4] && r[0] >= r[8]) {
    const double x = 0.5 * sqrt(fmax(1.0 + r[0] - r[4] - r[8], 0.0)), f = 0.25 / x;
    q = {(r[7] - r[5]) * f, x, (r[1] + r[3]) * f, (r[2] + r[6]) * f};
  } else if (r[4] >= r[8]) {
    const double y = 0.5 * sqrt(fmax(1.0 - r[0] + r[4] - r[8], 0.0)), f = 0.25 / y;
    q = {(r[2] - r[6]) * f, (r[1] + r[3]) * f, y, (r[5] + r[7]) * f};
  } else {
    const double z = 0.5 * sqrt(fmax(1.0 - r[0] - r[4] + r[8], 0.0)), f = 0.25 / z;
    q = {(r[3] - r[1]) * f, (r[2] + r[6]) * f, (r[5] + r[7]) * f, z};
  }
  const double nrm = sqrt(q.w * q.w + q.x * q.x + q.y * q.y + q.z * q.z);
  return {q.w / nrm, q.x / nrm, q.y / nrm, q.z / nrm};
}

__global__ void k_rot_to_quat(const double* __restrict__ R, int64_t count,
                              Q4<double>* __restrict__ out, int canonical,
                              uint8_t* __restrict__ bad) {
  const int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i >= count) return;
  double a[9];
  for (int k = 0; k < 9; ++k) a[k] = R[9 * i + k];
  // validity: det > 0 and ||A^T A - I||_F <= 1e-2
  double dev = 0.0;
  for (int r = 0; r < 3; ++r)
    for (int s = 0; s < 3; ++s) {
      const double d = a[r] * a[s] + a[3 + r] * a[3 + s] + a[6 + r] * a[6 + s] - (r == s ? 1.0 : 0.0);
      dev += d * d;
    }
  const bool ok = det3<double>(a) > 0.0 && sqrt(dev) <= 1e-2;
  bad[i] = ok ? 0 : 1;
  if (!ok) {
    out[i] = Q4<double>{1.0, 0.0, 0.0, 0.0};
    return;
  }
  double rot[9], sig[3];
  polar3<double>(a, rot, sig);
  Q4<double> q = quat_of_rot(rot);
  if (canonical) {
    const double lead = fabs(q.w) > 1e-6 ? q.w : fabs(q.x) > 1e-6 ? q.x : fabs(q.y) > 1e-6 ? q.y : q.z;
    if (lead < 0.0) q = Q4<double>{-q.w, -q.x, -q.y, -q.z};
  }
  out[i] = q;
}

__global__ void k_align(const Q4<double>* __restrict__ pv, Q4<double>* __restrict__ qe,
                        const int32_t* __restrict__ ei, const int32_t* __restrict__ ej, int64_t m) {
  const int64_t e = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (e >= m) return;
  const Q4<double> a = qmul(pv[ei[e]], qe[e]);
  const Q4<double> b = pv[ej[e]];
  const double s = a.w * b.w + a.x * b.x + a.y * b.y + a.z * b.z;
  if (s < 0.0) {
    const Q4<double> q = qe[e];
    qe[e] = Q4<double>{-q.w, -q.x, -q.y, -q.z};
  }
}

__global__ void k_iota(int32_t* v, int64_t m) {
  const int64_t e = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (e < m) v[e] = int32_t(e);
}

__global__ void k_ptr(const int32_t* __restrict__ keys, int64_t m, int32_t n,
                      int32_t* __restrict__ ptr) {
  const int64_t v = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (v > n) return;
  int64_t lo = 0, hi = m;  // first position with key >= v
  while (lo < hi) {
    const int64_t mid = (lo + hi) >> 1;
    if (keys[mid] < v) lo = mid + 1; else hi = mid;
  }
  ptr[v] = int32_t(lo);
}

template <typename T>
__global__ void k_fill_edges(const int32_t* __restrict__ perm, const int32_t* __restrict__ nbr_src,
                             const Q4<double>* __restrict__ qe, const double* __restrict__ tm,
                             const double* __restrict__ kappa, const double* __restrict__ tau,
                             int64_t m, int32_t* __restrict__ nbr, P4<T>* __restrict__ tt,
                             Q4<T>* __restrict__ w) {
  const int64_t k = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (k >= m) return;
  const int32_t e = perm[k];
  nbr[k] = nbr_src[e];
  const double ta = tau[e], ka = kappa[e];
  tt[k] = P4<T>{T(ta * tm[3 * int64_t(e)]), T(ta * tm[3 * int64_t(e) + 1]),
                T(ta * tm[3 * int64_t(e) + 2]), T(ta)};
  const Q4<double> q = qe[e];
  w[k] = Q4<T>{T(ka * q.w), T(ka * q.x), T(ka * q.y), T(ka * q.z)};
}

template <typename T>
__global__ void k_vertex_consts(int32_t n, const int32_t* __restrict__ o_ptr,
                                const int32_t* __restrict__ o_perm,
                                const int32_t* __restrict__ i_ptr,
                                const int32_t* __restrict__ i_perm, const double* __restrict__ tm,
                                const double* __restrict__ kappa, const double* __restrict__ tau,
                                T* cQ, T* cT, T* cS) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  double q = 0.0, s = 0.0, t = 0.0;
  for (int k = o_ptr[i]; k < o_ptr[i + 1]; ++k) {
    const int64_t e = o_perm[k];
    const double x = tm[3 * e], y = tm[3 * e + 1], z = tm[3 * e + 2];
    q += 2.0 * (tau[e] * (x * x + y * y + z * z) + kappa[e]);
    s += 2.0 * tau[e];
  }
  for (int k = i_ptr[i]; k < i_ptr[i + 1]; ++k) t += 2.0 * tau[i_perm[k]];
  cQ[i] = T(q);
  cT[i] = T(t);
  cS[i] = T(s);
}

template <typename T>
__global__ void k_init_state(DevGraph<T> g, const Q4<double>* __restrict__ p0,
                             const double* __restrict__ t0) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= g.n) return;
  const Q4<T> p = cvt<T>(p0[i]);
  const V3<T> t = {T(t0[3 * int64_t(i)]), T(t0[3 * int64_t(i) + 1]), T(t0[3 * int64_t(i) + 2])};
  const Q4<T> zq = {T(0), T(0), T(0), T(0)};
  const V3<T> zv = {T(0), T(0), T(0)};
  g.p[i] = p;
  g.q[i] = p;
  g.t[i] = t;
  g.s[i] = t;
  g.lam[i] = zq;
  g.z[i] = zv;
  g.q_prev[i] = p;
  g.t_prev[i] = t;
  g.s_prev[i] = t;
  g.lam_prev[i] = zq;
  g.z_prev[i] = zv;
}

// state <-> packed n x 21 doubles (p q t s lambda z)
template <typename T>
__global__ void k_state_io(DevGraph<T> g, double* __restrict__ buf, int to_device) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= g.n) return;
  double* b = buf + 21 * int64_t(i);
  if (!to_device) {
    const Q4<T> p = g.p[i], q = g.q[i], l = g.lam[i];
    const V3<T> t = g.t[i], s = g.s[i], z = g.z[i];
    const double v[21] = {double(p.w), double(p.x), double(p.y), double(p.z),
                          double(q.w), double(q.x), double(q.y), double(q.z),
                          double(t.x), double(t.y), double(t.z),
                          double(s.x), double(s.y), double(s.z),
                          double(l.w), double(l.x), double(l.y), double(l.z),
                          double(z.x), double(z.y), double(z.z)};
    for (int k = 0; k < 21; ++k) b[k] = v[k];
  } else {
    g.p[i] = Q4<T>{T(b[0]), T(b[1]), T(b[2]), T(b[3])};
    g.q[i] = Q4<T>{T(b[4]), T(b[5]), T(b[6]), T(b[7])};
    g.t[i] = V3<T>{T(b[8]), T(b[9]), T(b[10])};
    g.s[i] = V3<T>{T(b[11]), T(b[12]), T(b[13])};
    g.lam[i] = Q4<T>{T(b[14]), T(b[15]), T(b[16]), T(b[17])};
    g.z[i] = V3<T>{T(b[18]), T(b[19]), T(b[20])};
    g.q_prev[i] = g.q[i];
    g.lam_prev[i] = g.lam[i];
    g.t_prev[i] = g.t[i];
    g.s_prev[i] = g.s[i];
    g.z_prev[i] = g.z[i];
  }
}

// R(p_i) row-major: column k of R is Im(p [0, e_k] p^*)
template <typename T>
__global__ void k_poses(DevGraph<T> g, double* __restrict__ R, double* __restrict__ t) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= g.n) return;
  const Q4<double> p = cvt<double>(g.p[i]);
  if (R) {
    for (int k = 0; k < 3; ++k) {
      const V3<double> e = {k == 0 ? 1.0 : 0.0, k == 1 ? 1.0 : 0.0, k == 2 ? 1.0 : 0.0};
      const V3<double> col = im_mul_conj(qmul_vp(p, e), p);
      R[9 * int64_t(i) + k] = col.x;
      R[9 * int64_t(i) + 3 + k] = col.y;
      R[9 * int64_t(i) + 6 + k] = col.z;
    }
  }
  if (t) {
    const V3<T> ti = g.t[i];
    t[3 * int64_t(i)] = double(ti.x);
    t[3 * int64_t(i) + 1] = double(ti.y);
    t[3 * int64_t(i) + 2] = double(ti.z);
  }
}

inline dim3 grid_for(int64_t count, int block) {
  return dim3(unsigned((count + block - 1) / block));
}

}  // namespace

hipError_t launch_rot_to_quat(const double* R, int64_t count, Q4<double>* out, int canonical,
                              uint8_t* bad, hipStream_t st) {
  if (count <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_rot_to_quat, grid_for(count, 256), dim3(256), 0, st, R, count, out,
                     canonical, bad);
  return hipGetLastError();
}

hipError_t launch_align(const Q4<double>* pv, Q4<double>* qe, const int32_t* ei,
                        const int32_t* ej, int64_t m, hipStream_t st) {
  if (m <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_align, grid_for(m, 256), dim3(256), 0, st, pv, qe, ei, ej, m);
  return hipGetLastError();
}

hipError_t sort_by_key(const int32_t* keys, int32_t* perm, int64_t m, int32_t n, int32_t* iota,
                       void* tmp, size_t* tmp_bytes, int32_t* keys_sorted, hipStream_t st) {
  // tmp == nullptr: size query only (writes *tmp_bytes)
  int bits = 1;
  while ((int64_t(1) << bits) < int64_t(n)) ++bits;
  if (tmp == nullptr)
    return hipcub::DeviceRadixSort::SortPairs(nullptr, *tmp_bytes, keys, keys_sorted, iota, perm,
                                              int(m), 0, bits, st);
  if (m <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_iota, grid_for(m, 256), dim3(256), 0, st, iota, m);
  return hipcub::DeviceRadixSort::SortPairs(tmp, *tmp_bytes, keys, keys_sorted, iota, perm, int(m),
                                            0, bits, st);
}

hipError_t launch_ptr_from_sorted(const int32_t* keys_sorted, int64_t m, int32_t n, int32_t* ptr,
                                  hipStream_t st) {
  hipLaunchKernelGGL(k_ptr, grid_for(int64_t(n) + 1, 256), dim3(256), 0, st, keys_sorted, m, n,
                     ptr);
  return hipGetLastError();
}

template <typename T>
hipError_t launch_fill_edges(const int32_t* perm, const int32_t* nbr_src, const Q4<double>* qe,
                             const double* tm, const double* kappa, const double* tau, int64_t m,
                             int32_t* nbr, P4<T>* tt, Q4<T>* w, hipStream_t st) {
  if (m <= 0) return hipSuccess;
  hipLaunchKernelGGL((k_fill_edges<T>), grid_for(m, 256), dim3(256), 0, st, perm, nbr_src, qe, tm,
                     kappa, tau, m, nbr, tt, w);
  return hipGetLastError();
}

template <typename T>
hipError_t launch_vertex_consts(int32_t n, const int32_t* o_ptr, const int32_t* o_perm,
                                const int32_t* i_ptr, const int32_t* i_perm, const double* tm,
                                const double* kappa, const double* tau, T* cQ, T* cT, T* cS,
                                hipStream_t st) {
  hipLaunchKernelGGL((k_vertex_consts<T>), grid_for(n, 256), dim3(256), 0, st, n, o_ptr, o_perm,
                     i_ptr, i_perm, tm, kappa, tau, cQ, cT, cS);
  return hipGetLastError();
}

template <typename T>
hipError_t launch_init_state(const DevGraph<T>& g, const Q4<double>* p0, const double* t0,
                             hipStream_t st) {
  hipLaunchKernelGGL((k_init_state<T>), grid_for(g.n, 256), dim3(256), 0, st, g, p0, t0);
  return hipGetLastError();
}

template <typename T>
hipError_t launch_state_io(const DevGraph<T>& g, double* buf, int to_device, hipStream_t st) {
  hipLaunchKernelGGL((k_state_io<T>), grid_for(g.n, 256), dim3(256), 0, st, g, buf, to_device);
  return hipGetLastError();
}

template <typename T>
hipError_t launch_poses(const DevGraph<T>& g, double* R, double* t, hipStream_t st) {
  hipLaunchKernelGGL((k_poses<T>), grid_for(g.n, 256), dim3(256), 0, st, g, R, t);
  return hipGetLastError();
}

#define PGO_INST(T)                                                                             \
  template hipError_t launch_fill_edges<T>(const int32_t*, const int32_t*, const Q4<double>*,  \
                                           const double*, const double*, const double*,       \
                                           int64_t, int32_t*, P4<T>*, Q4<T>*, hipStream_t);   \
  template hipError_t launch_vertex_consts<T>(int32_t, const int32_t*, const int32_t*,         \
                                              const int32_t*, const int32_t*, const double*,  \
                                              const double*, const double*, T*, T*, T*,       \
                                              hipStream_t);                                   \
  template hipError_t launch_init_state<T>(const DevGraph<T>&, const Q4<double>*,             \
                                           const double*, hipStream_t);                       \
  template hipError_t launch_state_io<T>(const DevGraph<T>&, double*, int, hipStream_t);      \
  template hipError_t launch_poses<T>(const DevGraph<T>&, double*, double*, hipStream_t);
PGO_INST(float)
PGO_INST(double)
#undef PGO_INST

// Device-to-device copy of 8-byte words as an ordinary kernel on the stream,
// so it is ordered with the sweep launches (plain or replayed graphs) exactly
// like every other kernel of the library.
template <typename W>
__global__ void k_copy_words(W* __restrict__ dst, const W* __restrict__ src, int64_t words) {
  const int64_t stride = int64_t(gridDim.x) * blockDim.x;
  for (int64_t k = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; k < words; k += stride)
    dst[k] = src[k];
}

__global__ void k_gather_edges_f64(const int32_t* __restrict__ perm, int64_t m,
                                   const int32_t* __restrict__ ei, const int32_t* __restrict__ ej,
                                   const Q4<double>* __restrict__ q, const double* __restrict__ tm,
                                   const double* __restrict__ kappa,
                                   const double* __restrict__ tau, const double* __restrict__ X9,
                                   int32_t* __restrict__ oi, int32_t* __restrict__ oj,
                                   Q4<double>* __restrict__ oq, double* __restrict__ otm,
                                   double* __restrict__ okappa, double* __restrict__ otau,
                                   double* __restrict__ oX9) {
  const int64_t k = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (k >= m) return;
  const int64_t e = perm[k];
  oi[k] = ei[e];
  oj[k] = ej[e];
  if (q) oq[k] = q[e];
  for (int c = 0; c < 3; ++c) otm[3 * k + c] = tm[3 * e + c];
  okappa[k] = kappa[e];
  otau[k] = tau[e];
  if (X9)
    for (int c = 0; c < 9; ++c) oX9[9 * k + c] = X9[9 * e + c];
}

hipError_t launch_gather_edges_f64(const int32_t* perm, int64_t m, const int32_t* ei,
                                   const int32_t* ej, const Q4<double>* q, const double* tm,
                                   const double* kappa, const double* tau, const double* X9,
                                   int32_t* oi, int32_t* oj, Q4<double>* oq, double* otm,
                                   double* okappa, double* otau, double* oX9, hipStream_t st) {
  if (m <= 0) return hipSuccess;
  if (!perm || !ei || !ej || !tm || !kappa || !tau || !oi || !oj || !otm || !okappa || !otau ||
      (q && !oq) || (X9 && !oX9))
    return hipErrorInvalidValue;
  hipLaunchKernelGGL(k_gather_edges_f64, grid_for(m, 256), dim3(256), 0, st, perm, m, ei, ej, q,
                     tm, kappa, tau, X9, oi, oj, oq, otm, okappa, otau, oX9);
  return hipGetLastError();
}

hipError_t launch_copy(void* dst, const void* src, size_t bytes, hipStream_t st) {
  if (bytes == 0) return hipSuccess;
  const uintptr_t a = reinterpret_cast<uintptr_t>(dst) | reinterpret_cast<uintptr_t>(src);
  if (bytes % 4 || a % 4) return hipErrorInvalidValue;
  if (bytes % 8 == 0 && a % 8 == 0) {
    const int64_t words = int64_t(bytes / 8);
    const int64_t blocks = std::min<int64_t>((words + 255) / 256, 8192);
    hipLaunchKernelGGL(k_copy_words<uint64_t>, dim3(unsigned(blocks)), dim3(256), 0, st,
                       static_cast<uint64_t*>(dst), static_cast<const uint64_t*>(src), words);
  } else {
    const int64_t words = int64_t(bytes / 4);
    const int64_t blocks = std::min<int64_t>((words + 255) / 256, 8192);
    hipLaunchKernelGGL(k_copy_words<uint32_t>, dim3(unsigned(blocks)), dim3(256), 0, st,
                       static_cast<uint32_t*>(dst), static_cast<const uint32_t*>(src), words);
  }
  return hipGetLastError();
}

struct RestoreArgs {
  uint32_t* dst[6];
  const uint32_t* src[6];
  int words[6];
};

__global__ void k_restore_words(int32_t n, const int32_t* __restrict__ gid,
                                const int32_t* __restrict__ flag, RestoreArgs a) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n || !flag[gid[i]]) return;
  for (int k = 0; k < 6; ++k) {
    const int w = a.words[k];
    for (int c = 0; c < w; ++c) a.dst[k][int64_t(i) * w + c] = a.src[k][int64_t(i) * w + c];
  }
}

hipError_t launch_restore_words(int32_t n, const int32_t* gid, const int32_t* flag,
                                void* const* dst, const void* const* src, const int* words,
                                hipStream_t st) {
  if (n <= 0) return hipSuccess;
  RestoreArgs a;
  for (int k = 0; k < 6; ++k) {
    if (words[k] < 0 || words[k] > 32) return hipErrorInvalidValue;
    a.dst[k] = static_cast<uint32_t*>(dst[k]);
    a.src[k] = static_cast<const uint32_t*>(src[k]);
    a.words[k] = words[k];
  }
  hipLaunchKernelGGL(k_restore_words, dim3((n + 255) / 256), dim3(256), 0, st, n, gid, flag, a);
  return hipGetLastError();
}

}  // namespace pgo
