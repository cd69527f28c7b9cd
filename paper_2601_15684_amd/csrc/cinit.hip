// Chordal initialisation on the device (the step before the path: the
// experiments start every method from a chordal initial point):
//
//   1. relaxed rotations  min sum_e kappa_e |R_i R~_e - R_j|_F^2  over free
//      3x3 blocks, one anchor per connected component held at its given
//      rotation.  Normal equations, for a free vertex i:
//        (A R)_i = d_i R_i - sum_out kappa R_j R~^T - sum_in kappa R_l R~ = 0,
//        d_i = sum_out kappa + sum_in kappa  (R~ R~^T = I);
//   2. R_i <- its SO(3) polar factor;
//   3. translations  min sum_e tau_e |t_j - t_i - R_i t~_e|^2 :
//        (A t)_i = d_i t_i - sum_out tau t_j - sum_in tau t_l
//                = sum_in tau R_l t~ - sum_out tau R_i t~,  d_i = sum tau.
//
// Both are solved per graph by Jacobi-preconditioned conjugate gradients in
// FP64, every graph of a batch with its own scalars.  Vectors hold the
// anchors' fixed values; search directions are zero there, so A applied to
// them is A_ff.  Work is cut into the reduction chunks of the handle (never
// straddling graphs); each workgroup owns one chunk, forms its partial dot
// product with a fixed-shape tree, and one thread per graph adds the
// partials in order: deterministic, no atomics.
#include "internal.hpp"
#include "polar.hpp"

namespace pgo {

namespace {

constexpr int kCB = 256;

__device__ double block_sum1(double v, double* sh) {
  sh[threadIdx.x] = v;
  __syncthreads();
  for (int w = kCB / 2; w > 0; w >>= 1) {
    if (threadIdx.x < w) sh[threadIdx.x] += sh[threadIdx.x + w];
    __syncthreads();
  }
  const double r = sh[0];
  __syncthreads();
  return r;
}

// y = (A x)_i for one vertex; W = 9 (rotation rows, R~ transforms) or 3.
template <int W>
__device__ void apply_A(const CinitGraph& c, int i, const double* __restrict__ x, double y[W]) {
  const double* xi = x + int64_t(W) * i;
  const double di = c.diag[i];
  for (int k = 0; k < W; ++k) y[k] = di * xi[k];
  for (int e = c.o_ptr[i]; e < c.o_ptr[i + 1]; ++e) {
    const double* xj = x + int64_t(W) * c.o_nbr[e];
    if (W == 9) {
      const double* Rm = c.o_wR + 9 * int64_t(e);  // x_j (w R~)^T: (r, q) -> sum_k x_j[r][k] wR~[q][k]
      for (int r = 0; r < 3; ++r)
        for (int q = 0; q < 3; ++q)
          y[3 * r + q] -= xj[3 * r] * Rm[3 * q] + xj[3 * r + 1] * Rm[3 * q + 1] +
                          xj[3 * r + 2] * Rm[3 * q + 2];
    } else {
      const double w = c.o_w[e];
      for (int k = 0; k < W; ++k) y[k] -= w * xj[k];
    }
  }
  for (int e = c.i_ptr[i]; e < c.i_ptr[i + 1]; ++e) {
    const double* xl = x + int64_t(W) * c.i_nbr[e];
    if (W == 9) {
      const double* Rm = c.i_wR + 9 * int64_t(e);  // x_l (w R~): (r, q) -> sum_k x_l[r][k] wR~[k][q]
      for (int r = 0; r < 3; ++r)
        for (int q = 0; q < 3; ++q)
          y[3 * r + q] -= xl[3 * r] * Rm[q] + xl[3 * r + 1] * Rm[3 + q] + xl[3 * r + 2] * Rm[6 + q];
    } else {
      const double w = c.i_w[e];
      for (int k = 0; k < W; ++k) y[k] -= w * xl[k];
    }
  }
}

// edge data of the operator in out- and in-order
__global__ void k_cinit_edges(CinitGraph c, int64_t m, int W) {
  const int64_t e = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (e >= m) return;
  const int64_t eo = c.o_perm[e], ei = c.i_perm[e];
  if (W == 9) {
    const double wo = c.wt[eo], wi = c.wt[ei];
    for (int k = 0; k < 9; ++k) {
      c.o_wR[9 * e + k] = wo * c.R9[9 * eo + k];
      c.i_wR[9 * e + k] = wi * c.R9[9 * ei + k];
    }
  } else {
    c.o_w[e] = c.wt[eo];
    c.i_w[e] = c.wt[ei];
  }
}

// diag_i = sum of the weights of every edge at i
__global__ void k_cinit_diag(CinitGraph c, int32_t n) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  double d = 0.0;
  for (int e = c.o_ptr[i]; e < c.o_ptr[i + 1]; ++e) d += c.wt[c.o_perm[e]];
  for (int e = c.i_ptr[i]; e < c.i_ptr[i + 1]; ++e) d += c.wt[c.i_perm[e]];
  c.diag[i] = d;
}

// translation right-hand side: sum_in tau R_l t~ - sum_out tau R_i t~
__global__ void k_cinit_rhs_t(CinitGraph c, int32_t n, const double* __restrict__ R,
                              double* __restrict__ rhs) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  double b[3] = {0.0, 0.0, 0.0};
  const double* Ri = R + 9 * int64_t(i);
  for (int e = c.o_ptr[i]; e < c.o_ptr[i + 1]; ++e) {
    const int64_t ed = c.o_perm[e];
    const double w = c.wt[ed], *u = c.tm + 3 * ed;
    for (int r = 0; r < 3; ++r) b[r] -= w * (Ri[3 * r] * u[0] + Ri[3 * r + 1] * u[1] + Ri[3 * r + 2] * u[2]);
  }
  for (int e = c.i_ptr[i]; e < c.i_ptr[i + 1]; ++e) {
    const int64_t ed = c.i_perm[e];
    const double w = c.wt[ed], *u = c.tm + 3 * ed;
    const double* Rl = R + 9 * int64_t(c.i_nbr[e]);
    for (int r = 0; r < 3; ++r) b[r] += w * (Rl[3 * r] * u[0] + Rl[3 * r + 1] * u[1] + Rl[3 * r + 2] * u[2]);
  }
  for (int r = 0; r < 3; ++r) rhs[3 * int64_t(i) + r] = b[r];
}

// r = b - A x (b may be null: 0), z = r / d, p = z on free vertices (0 on
// anchors); partial of <r, z> per chunk.
template <int W>
__global__ void __launch_bounds__(kCB) k_cinit_start(CinitGraph c, CinitVec v, const double* b,
                                                     const int64_t* __restrict__ beg,
                                                     const int64_t* __restrict__ end,
                                                     double* __restrict__ part) {
  __shared__ double sh[kCB];
  double acc = 0.0;
  const int ch = blockIdx.x;
  for (int64_t i = beg[ch] + threadIdx.x; i < end[ch]; i += kCB) {
    double y[W];
    apply_A<W>(c, int(i), v.x, y);
    const bool fr = !c.anchor[i];
    const double di = c.diag[i];
    for (int k = 0; k < W; ++k) {
      const double r = fr ? (b ? b[W * i + k] : 0.0) - y[k] : 0.0;
      const double z = (fr && di > 0.0) ? r / di : 0.0;
      v.r[W * i + k] = r;
      v.p[W * i + k] = z;
      acc += r * z;
    }
  }
  acc = block_sum1(acc, sh);
  if (threadIdx.x == 0) part[ch] = acc;
}

// ap = A p; partial of <p, ap> per chunk (graphs that stopped skip the work)
template <int W>
__global__ void __launch_bounds__(kCB) k_cinit_Ap(CinitGraph c, CinitVec v,
                                                  const int64_t* __restrict__ beg,
                                                  const int64_t* __restrict__ end,
                                                  const int32_t* __restrict__ cgraph,
                                                  const int32_t* __restrict__ active,
                                                  double* __restrict__ part) {
  __shared__ double sh[kCB];
  double acc = 0.0;
  const int ch = blockIdx.x;
  if (active[cgraph[ch]]) {
    for (int64_t i = beg[ch] + threadIdx.x; i < end[ch]; i += kCB) {
      double y[W];
      apply_A<W>(c, int(i), v.p, y);
      const bool fr = !c.anchor[i];  // rows of A_ff only
      for (int k = 0; k < W; ++k) {
        const double a = fr ? y[k] : 0.0;
        v.ap[W * i + k] = a;
        acc += v.p[W * i + k] * a;
      }
    }
  }
  acc = block_sum1(acc, sh);
  if (threadIdx.x == 0) part[ch] = acc;
}

// x += alpha p, r -= alpha ap, z = r / d; partial of <r, z>.  The chunk's
// W x (vertices) doubles are walked as one flat range, so consecutive
// threads touch consecutive doubles.
template <int W>
__global__ void __launch_bounds__(kCB) k_cinit_update(CinitGraph c, CinitVec v,
                                                      const int64_t* __restrict__ beg,
                                                      const int64_t* __restrict__ end,
                                                      const int32_t* __restrict__ cgraph,
                                                      const int32_t* __restrict__ active,
                                                      const double* __restrict__ alpha,
                                                      double* __restrict__ part) {
  __shared__ double sh[kCB];
  double acc = 0.0;
  const int ch = blockIdx.x;
  const int gr = cgraph[ch];
  if (active[gr]) {
    const double a = alpha[gr];
    for (int64_t q = W * beg[ch] + threadIdx.x; q < W * end[ch]; q += kCB) {
      const int64_t i = q / W;
      const double di = c.diag[i];
      const bool fr = !c.anchor[i];
      v.x[q] += a * v.p[q];
      const double r = v.r[q] - a * v.ap[q];
      v.r[q] = r;
      const double z = (fr && di > 0.0) ? r / di : 0.0;
      v.z[q] = z;
      acc += r * z;
    }
  }
  acc = block_sum1(acc, sh);
  if (threadIdx.x == 0) part[ch] = acc;
}

// p = z + beta p, over the chunk's doubles as one flat range
template <int W>
__global__ void __launch_bounds__(kCB) k_cinit_dir(CinitVec v, const int64_t* __restrict__ beg,
                                                   const int64_t* __restrict__ end,
                                                   const int32_t* __restrict__ cgraph,
                                                   const int32_t* __restrict__ active,
                                                   const double* __restrict__ beta) {
  const int ch = blockIdx.x;
  const int gr = cgraph[ch];
  if (!active[gr]) return;
  const double b = beta[gr];
  for (int64_t q = W * beg[ch] + threadIdx.x; q < W * end[ch]; q += kCB) v.p[q] = v.z[q] + b * v.p[q];
}

// per-graph scalars.  mode 0: rz0 = rz = sum, active = rz > 0.
// mode 1: alpha = rz / pAp.  mode 2: rz_new; stop when rz_new <= tol^2 rz0
// (or max iterations), else beta = rz_new / rz.
__global__ void k_cinit_scalars(int G, const double* __restrict__ part,
                                const int32_t* __restrict__ g_off, int mode, double tol2,
                                CinitScalars s) {
  const int gr = blockIdx.x * blockDim.x + threadIdx.x;
  if (gr >= G) return;
  double sum = 0.0;
  for (int k = g_off[gr]; k < g_off[gr + 1]; ++k) sum += part[k];
  if (mode == 0) {
    s.rz0[gr] = sum;
    s.rz[gr] = sum;
    s.active[gr] = sum > 0.0 ? 1 : 0;
    s.iters[gr] = 0;
    return;
  }
  if (!s.active[gr]) return;
  if (mode == 1) {
    s.alpha[gr] = sum > 0.0 ? s.rz[gr] / sum : 0.0;
    if (!(sum > 0.0)) s.active[gr] = 0;
    return;
  }
  s.iters[gr] += 1;
  s.beta[gr] = s.rz[gr] > 0.0 ? sum / s.rz[gr] : 0.0;
  s.rz[gr] = sum;
  if (!(sum > tol2 * s.rz0[gr])) s.active[gr] = 0;
}

__global__ void k_cinit_project(int32_t n, const uint8_t* __restrict__ anchor,
                                const double* __restrict__ X, const double* __restrict__ given,
                                double* __restrict__ R) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  double rot[9], sig[3];
  if (anchor[i]) {
    for (int k = 0; k < 9; ++k) rot[k] = given[9 * int64_t(i) + k];
  } else {
    double a[9];
    for (int k = 0; k < 9; ++k) a[k] = X[9 * int64_t(i) + k];
    polar3<double>(a, rot, sig);
  }
  for (int k = 0; k < 9; ++k) R[9 * int64_t(i) + k] = rot[k];
}

// quaternion -> rotation matrix (row-major), for the edges of the quaternion model
__global__ void k_cinit_qmat(int64_t m, const Q4<double>* __restrict__ q, double* __restrict__ R) {
  const int64_t e = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (e >= m) return;
  const Q4<double> a = q[e];
  const double w = a.w, x = a.x, y = a.y, z = a.z;
  double* r = R + 9 * e;
  r[0] = 1 - 2 * (y * y + z * z); r[1] = 2 * (x * y - w * z);     r[2] = 2 * (x * z + w * y);
  r[3] = 2 * (x * y + w * z);     r[4] = 1 - 2 * (x * x + z * z); r[5] = 2 * (y * z - w * x);
  r[6] = 2 * (x * z - w * y);     r[7] = 2 * (y * z + w * x);     r[8] = 1 - 2 * (x * x + y * y);
}

inline dim3 grid_of(int64_t count, int block) { return dim3(unsigned((count + block - 1) / block)); }

}  // namespace

hipError_t launch_cinit_edges(const CinitGraph& c, int64_t m, int W, hipStream_t st) {
  if (m <= 0) return hipSuccess;
  if (W != 9 && W != 3) return hipErrorInvalidValue;
  hipLaunchKernelGGL(k_cinit_edges, dim3(unsigned((m + 255) / 256)), dim3(256), 0, st, c, m, W);
  return hipGetLastError();
}

hipError_t launch_cinit_diag(const CinitGraph& c, int32_t n, hipStream_t st) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_cinit_diag, grid_of(n, 256), dim3(256), 0, st, c, n);
  return hipGetLastError();
}

hipError_t launch_cinit_rhs_t(const CinitGraph& c, int32_t n, const double* R, double* rhs,
                              hipStream_t st) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_cinit_rhs_t, grid_of(n, 256), dim3(256), 0, st, c, n, R, rhs);
  return hipGetLastError();
}

hipError_t launch_cinit_project(int32_t n, const uint8_t* anchor, const double* X,
                                const double* given, double* R, hipStream_t st) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_cinit_project, grid_of(n, 256), dim3(256), 0, st, n, anchor, X, given, R);
  return hipGetLastError();
}

hipError_t launch_cinit_qmat(int64_t m, const Q4<double>* q, double* R, hipStream_t st) {
  if (m <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_cinit_qmat, grid_of(m, 256), dim3(256), 0, st, m, q, R);
  return hipGetLastError();
}

hipError_t launch_cinit_cg(const CinitGraph& c, const CinitVec& v, const CinitChunks& ch, int W,
                           const double* b, int max_iters, int check_every, double tol,
                           const CinitScalars& s, int G, int32_t* host_active, hipStream_t st) {
  if (W != 9 && W != 3) return hipErrorInvalidValue;
  const int nc = ch.n_chunks;
  if (nc <= 0) return hipSuccess;
  const dim3 gs((G + 255) / 256);
  const double tol2 = tol * tol;
  if (W == 9)
    hipLaunchKernelGGL(k_cinit_start<9>, dim3(nc), dim3(kCB), 0, st, c, v, b, ch.beg, ch.end, ch.part);
  else
    hipLaunchKernelGGL(k_cinit_start<3>, dim3(nc), dim3(kCB), 0, st, c, v, b, ch.beg, ch.end, ch.part);
  hipLaunchKernelGGL(k_cinit_scalars, gs, dim3(256), 0, st, G, ch.part, ch.g_off, 0, tol2, s);
  for (int it = 0; it < max_iters; ++it) {
    if (W == 9) {
      hipLaunchKernelGGL(k_cinit_Ap<9>, dim3(nc), dim3(kCB), 0, st, c, v, ch.beg, ch.end, ch.cgraph,
                         s.active, ch.part);
    } else {
      hipLaunchKernelGGL(k_cinit_Ap<3>, dim3(nc), dim3(kCB), 0, st, c, v, ch.beg, ch.end, ch.cgraph,
                         s.active, ch.part);
    }
    hipLaunchKernelGGL(k_cinit_scalars, gs, dim3(256), 0, st, G, ch.part, ch.g_off, 1, tol2, s);
    if (W == 9) {
      hipLaunchKernelGGL(k_cinit_update<9>, dim3(nc), dim3(kCB), 0, st, c, v, ch.beg, ch.end,
                         ch.cgraph, s.active, s.alpha, ch.part);
    } else {
      hipLaunchKernelGGL(k_cinit_update<3>, dim3(nc), dim3(kCB), 0, st, c, v, ch.beg, ch.end,
                         ch.cgraph, s.active, s.alpha, ch.part);
    }
    hipLaunchKernelGGL(k_cinit_scalars, gs, dim3(256), 0, st, G, ch.part, ch.g_off, 2, tol2, s);
    if (W == 9) {
      hipLaunchKernelGGL(k_cinit_dir<9>, dim3(nc), dim3(kCB), 0, st, v, ch.beg, ch.end, ch.cgraph,
                         s.active, s.beta);
    } else {
      hipLaunchKernelGGL(k_cinit_dir<3>, dim3(nc), dim3(kCB), 0, st, v, ch.beg, ch.end, ch.cgraph,
                         s.active, s.beta);
    }
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    if ((it + 1) % check_every == 0 || it + 1 == max_iters) {
      e = hipMemcpyAsync(host_active, s.active, sizeof(int32_t) * G, hipMemcpyDeviceToHost, st);
      if (e != hipSuccess) return e;
      e = hipStreamSynchronize(st);
      if (e != hipSuccess) return e;
      bool any = false;
      for (int k = 0; k < G; ++k) any = any || host_active[k];
      if (!any) break;
    }
  }
  return hipGetLastError();
}

}  // namespace pgo
