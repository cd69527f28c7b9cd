// Polar factor of a 3x3 matrix, register resident, by one-sided Jacobi.
//
// Plane rotations multiply A from the right until its columns are
// orthogonal: A V = U S.  The rotation closest to A in the Frobenius norm
// (the maximiser of <R, A> over SO(3)) is R = U diag(1, 1, det(U V^T)) V^T:
// when U V^T is a reflection, the column of U with the smallest singular
// value changes sign.  Row-major in and out; sig returns the singular values
// (unsorted, matching the columns of U).
#pragma once
#include <hip/hip_runtime.h>

namespace pgo {

template <typename T>
__device__ __forceinline__ T det3(const T r[9]) {
  return r[0] * (r[4] * r[8] - r[5] * r[7]) - r[1] * (r[3] * r[8] - r[5] * r[6]) +
         r[2] * (r[3] * r[7] - r[4] * r[6]);
}

template <typename T>
__device__ void polar3(const T a_in[9], T R[9], T sig[3]) {
  // convergence threshold on the largest |cos| between two columns; FP32
  // rounding alone leaves ~1e-7, so the float threshold sits above it
  constexpr T kEps = sizeof(T) == 4 ? T(3e-7) : T(1e-15);
  // The factor does not depend on the scale of A: A is taken times 2^-e,
  // e the binary exponent of its largest entry (exact), so that the
  // products of squared column norms below stay finite in FP32 (entries of
  // 1e9 and more overflow them); the singular values are scaled back.
  T amax = T(0);
  for (int k = 0; k < 9; ++k) amax = fmax(amax, fabs(a_in[k]));
  int e = 0;
  if (amax > T(0) && amax <= T(3e38)) (void)frexp(amax, &e);
  T c[3][3], v[3][3];  // c[k] = column k of A V, v[k] = column k of V
  for (int k = 0; k < 3; ++k)
    for (int r = 0; r < 3; ++r) {
      c[k][r] = ldexp(a_in[3 * r + k], -e);
      v[k][r] = (k == r) ? T(1) : T(0);
    }
  const int P[3] = {0, 0, 1}, Qc[3] = {1, 2, 2};
  for (int sweep = 0; sweep < 20; ++sweep) {
    T off = T(0);
#pragma unroll
    for (int pr = 0; pr < 3; ++pr) {
      const int p = P[pr], q = Qc[pr];
      const T al = c[p][0] * c[p][0] + c[p][1] * c[p][1] + c[p][2] * c[p][2];
      const T be = c[q][0] * c[q][0] + c[q][1] * c[q][1] + c[q][2] * c[q][2];
      const T ga = c[p][0] * c[q][0] + c[p][1] * c[q][1] + c[p][2] * c[q][2];
      const T scale = sqrt(al * be);
      if (scale == T(0) || fabs(ga) <= T(0.1) * kEps * scale) continue;
      off = fmax(off, fabs(ga) / scale);
      const T zeta = (be - al) / (T(2) * ga);
      const T t = copysign(T(1), zeta) / (fabs(zeta) + sqrt(T(1) + zeta * zeta));
      const T cs = T(1) / sqrt(T(1) + t * t), sn = cs * t;
      for (int r = 0; r < 3; ++r) {
        const T cp = c[p][r], cq = c[q][r];
        c[p][r] = cs * cp - sn * cq;
        c[q][r] = sn * cp + cs * cq;
        const T vp = v[p][r], vq = v[q][r];
        v[p][r] = cs * vp - sn * vq;
        v[q][r] = sn * vp + cs * vq;
      }
    }
    if (off < kEps) break;
  }
  for (int k = 0; k < 3; ++k) {
    const T sk = sqrt(c[k][0] * c[k][0] + c[k][1] * c[k][1] + c[k][2] * c[k][2]);
    const T inv = sk > T(0) ? T(1) / sk : T(0);
    for (int r = 0; r < 3; ++r) c[k][r] *= inv;
    sig[k] = ldexp(sk, e);
  }
  for (int pass = 0; pass < 2; ++pass) {
    for (int r = 0; r < 3; ++r)
      for (int s = 0; s < 3; ++s)
        R[3 * r + s] = c[0][r] * v[0][s] + c[1][r] * v[1][s] + c[2][r] * v[2][s];
    if (det3(R) > T(0)) break;
    const int kmin = (sig[0] <= sig[1] && sig[0] <= sig[2]) ? 0 : (sig[1] <= sig[2] ? 1 : 2);
#pragma unroll
    for (int k = 0; k < 3; ++k)  // constant indices keep c in registers
      if (k == kmin)
        for (int r = 0; r < 3; ++r) c[k][r] = -c[k][r];
  }
}

}  // namespace pgo
