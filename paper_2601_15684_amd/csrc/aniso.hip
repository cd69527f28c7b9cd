// The quaternion sweep with a full translation information matrix per edge:
// Sigma1_e = diag(c_e, S_e) (Model section, S_e = Omega_e^{-1} symmetric
// positive definite, c_e = trace(S_e) / 3), Sigma2 = kappa_e I.  The blocks
// A_s of App. B are then full matrices:
//
//   P  A1 = 2 sum_out G1^T Sigma1 G1 + (2 sum_in kappa |q_l|^2 + beta + H1) I,
//      b1 = -2 sum_out G1^T Sigma1 [0, t_j - s_i] - 2 sum_in q_l (x) (kappa q~)
//           - beta q_i - lambda_i - H1 p_i,
//      p_i = argmin_{|p| = 1} 1/2 p^T A1 p + b1^T p   (Lemma 1; solved in FP64
//      from A1 = W diag(a) W^T by the secular equation of Lemma B.1 (ii):
//      Newton on 1/|x(lambda)| - 1 with bisection safeguards, x(lambda) =
//      -(A1 + lambda I)^{-1} b1, lambda > -a_min; in the hard case, of the
//      minimisers the one nearest p_i^k);
//   Q  A2 = 2 sum_out (G3^T Sigma1 G3 + kappa |p_j|^2 I) + (beta + H2) I,
//      b2 = 2 sum_out (G3^T Sigma1 [0, t_j - s_i] + p_j (x) (kappa q~)^*)
//           + beta p_i - lambda_i + H2 q_i,  q_i = A2^{-1} b2  (App. B.2);
//   T  (2 sum_in S + (beta + H3) I) t_i = 2 sum_in S (s_l + c_e) + beta s_i + z_i + H3 t_i;
//   S  (2 sum_out S + (beta + H4) I) s_i = 2 sum_out S (t_j - c_e) + beta t_i - z_i + H4 s_i;
//   multipliers as in the isotropic sweep.
// Here G1 x = q_i (x) [0, t~] (x) x^*, G3 x = x (x) [0, t~] (x) p_i^* (Lemma MW),
// c_e = Im(q (x) [0, t~] (x) p^*) of the edge's tail.  Schedules, fusion of S
// with the next P and determinism are those of the isotropic sweep.
#include <algorithm>

#include "internal.hpp"

namespace pgo {

namespace {

// edges in flight per thread in every edge loop: one in FP32 (the batch's
// per-graph launch: 103.5 ms with two, 101.7 with one, 108.6 with three),
// two in FP64
template <typename T>
constexpr int kUA = sizeof(T) == 4 ? 1 : 2;

template <typename A>
struct Sym3 {
  A xx, xy, xz, yy, yz, zz;
};

// from the two halves of the upper triangle, (xx, xy, xz) and (yy, yz, zz)
template <typename A, typename T>
__device__ __forceinline__ Sym3<A> sym3(const V3<T>& a, const V3<T>& b) {
  return {A(a.x), A(a.y), A(a.z), A(b.x), A(b.y), A(b.z)};
}

template <typename A>
__device__ __forceinline__ V3<A> smul(const Sym3<A>& S, const V3<A>& v) {
  return {S.xx * v.x + S.xy * v.y + S.xz * v.z, S.xy * v.x + S.yy * v.y + S.yz * v.z,
          S.xz * v.x + S.yz * v.y + S.zz * v.z};
}

template <typename A>
__device__ __forceinline__ A dot3v(const V3<A>& a, const V3<A>& b) {
  return a.x * b.x + a.y * b.y + a.z * b.z;
}

// columns k of a 4x4 map: c_k = u (x) e_k^* (G1, with u = q_i (x) [0, t~])
// or c_k = e_k (x) v (G3, with v = [0, t~] (x) p_i^*)
template <typename A>
__device__ __forceinline__ void cols_right(const Q4<A>& u, Q4<A> c[4]) {
  c[0] = u;                                              // u (x) 1
  c[1] = {u.x, -u.w, -u.z, u.y};                         // u (x) (-i)
  c[2] = {u.y, u.z, -u.w, -u.x};                         // u (x) (-j)
  c[3] = {u.z, -u.y, u.x, -u.w};                         // u (x) (-k)
}

template <typename A>
__device__ __forceinline__ void cols_left(const Q4<A>& v, Q4<A> c[4]) {
  c[0] = v;                                              // 1 (x) v
  c[1] = {-v.x, v.w, -v.z, v.y};                         // i (x) v
  c[2] = {-v.y, v.z, v.w, -v.x};                         // j (x) v
  c[3] = {-v.z, -v.y, v.x, v.w};                         // k (x) v
}

// acc (upper triangle of a 4x4, row-major 10 entries) += 2 C^T Sigma1 C,
// bacc += 2 C^T Sigma1 [0, r] for the columns C of one edge's map.
template <typename A>
__device__ __forceinline__ void add_quadratic(const Q4<A> c[4], A cw, const Sym3<A>& S,
                                              const V3<A>& Sr, A M[10], A bv[4], A sgn_b) {
  V3<A> Sc[4];
#pragma unroll
  for (int k = 0; k < 4; ++k) Sc[k] = smul(S, V3<A>{c[k].x, c[k].y, c[k].z});
  int idx = 0;
#pragma unroll
  for (int k = 0; k < 4; ++k)
#pragma unroll
    for (int l = k; l < 4; ++l) {
      M[idx++] += A(2) * (cw * c[k].w * c[l].w + c[k].x * Sc[l].x + c[k].y * Sc[l].y +
                          c[k].z * Sc[l].z);
    }
#pragma unroll
  for (int k = 0; k < 4; ++k) bv[k] += sgn_b * A(2) * (c[k].x * Sr.x + c[k].y * Sr.y + c[k].z * Sr.z);
}

__device__ __forceinline__ int uidx(int k, int l) {  // upper-triangle index, k <= l
  const int base[4] = {0, 4, 7, 9};
  return base[k] + (l - k);
}

// symmetric 4x4 eigen-decomposition by cyclic Jacobi rotations (FP64):
// A = V diag(w) V^T, columns of V the eigenvectors
__device__ void jacobi4(const double M[10], double w[4], double V[4][4]) {
  double a[4][4];
  for (int k = 0; k < 4; ++k)
    for (int l = k; l < 4; ++l) a[k][l] = a[l][k] = M[uidx(k, l)];
  for (int k = 0; k < 4; ++k)
    for (int l = 0; l < 4; ++l) V[k][l] = k == l ? 1.0 : 0.0;
  for (int sweep = 0; sweep < 16; ++sweep) {
    double off = 0.0, diag = 0.0;
    for (int k = 0; k < 4; ++k) {
      diag += a[k][k] * a[k][k];
      for (int l = k + 1; l < 4; ++l) off += a[k][l] * a[k][l];
    }
    if (off <= 1e-34 * diag || off == 0.0) break;
    for (int p = 0; p < 3; ++p)
      for (int q = p + 1; q < 4; ++q) {
        const double apq = a[p][q];
        if (apq == 0.0) continue;
        const double theta = (a[q][q] - a[p][p]) / (2.0 * apq);
        const double t = copysign(1.0, theta) / (fabs(theta) + sqrt(1.0 + theta * theta));
        const double c = 1.0 / sqrt(1.0 + t * t), s = t * c;
        for (int k = 0; k < 4; ++k) {  // columns p, q of A
          const double akp = a[k][p], akq = a[k][q];
          a[k][p] = c * akp - s * akq;
          a[k][q] = s * akp + c * akq;
        }
        for (int k = 0; k < 4; ++k) {  // rows p, q
          const double apk = a[p][k], aqk = a[q][k];
          a[p][k] = c * apk - s * aqk;
          a[q][k] = s * apk + c * aqk;
        }
        for (int k = 0; k < 4; ++k) {
          const double vkp = V[k][p], vkq = V[k][q];
          V[k][p] = c * vkp - s * vkq;
          V[k][q] = s * vkp + c * vkq;
        }
      }
  }
  for (int k = 0; k < 4; ++k) w[k] = a[k][k];
}

// LDL^T of A + lam I (A symmetric, upper triangle in M); false unless every
// pivot exceeds floor, i.e. unless A + lam I is safely positive definite.
__device__ __forceinline__ bool ldl4(const double M[10], double lam, double floor,
                                     double L[4][4], double dinv[4]) {
  double d[4];
#pragma unroll
  for (int j = 0; j < 4; ++j) {
    double dj = M[uidx(j, j)] + lam;
#pragma unroll
    for (int k = 0; k < j; ++k) dj -= L[j][k] * L[j][k] * d[k];
    if (!(dj > floor)) return false;
    d[j] = dj;
    dinv[j] = 1.0 / dj;
#pragma unroll
    for (int i = j + 1; i < 4; ++i) {
      double sij = M[uidx(j, i)];
#pragma unroll
      for (int k = 0; k < j; ++k) sij -= L[i][k] * L[j][k] * d[k];
      L[i][j] = sij * dinv[j];
    }
  }
  return true;
}

// The easy case of Lemma B.1 (ii) without an eigen-decomposition: Newton on
// phi(lambda) = 1/|x(lambda)| - 1, x(lambda) = -(A + lambda I)^{-1} b, each
// step from an LDL^T factorisation (phi' = x^T (A + lambda I)^{-1} x /
// |x|^3), started from the multiplier p^k would have (lambda = -p^T (A p + b)
// at p = p^k, exact at a fixed point) and kept in a bracket [lo, hi] of the
// root: lo = -min_k A_kk <= -a_min (a failed factorisation raises lo), hi =
// |b| - (Gershgorin lower bound of a_min), where |x| <= 1.  phi is concave
// and increasing on (-a_min, inf), so once left of the root Newton climbs to
// it monotonically.  Returns false (the caller then takes the eigen-
// decomposition path) on b = 0, a near-singular A + lambda I, or no
// convergence: the root is unique on (-a_min, inf), so both paths give the
// same point up to rounding.
__device__ bool trs4_ldl(const double M[10], const double b[4], const double pprev[4],
                         double x[4]) {
  const double nb = sqrt(b[0] * b[0] + b[1] * b[1] + b[2] * b[2] + b[3] * b[3]);
  if (!(nb > 0.0)) return false;
  double dmin = M[0], gmin = M[0], amax = fabs(M[0]);
#pragma unroll
  for (int k = 0; k < 4; ++k) {
    double off = 0.0;
#pragma unroll
    for (int l = 0; l < 4; ++l)
      if (l != k) off += fabs(M[uidx(k < l ? k : l, k < l ? l : k)]);
    const double dk = M[uidx(k, k)];
    dmin = fmin(dmin, dk);
    gmin = fmin(gmin, dk - off);
    amax = fmax(amax, fabs(dk) + off);
  }
  const double floor = 1e-10 * fmax(1.0, fmax(amax, nb));
  double lo = -dmin, hi = nb - gmin;
  double Ap[4];
#pragma unroll
  for (int k = 0; k < 4; ++k) {
    double sk = 0.0;
#pragma unroll
    for (int l = 0; l < 4; ++l) sk += M[uidx(k < l ? k : l, k < l ? l : k)] * pprev[l];
    Ap[k] = sk + b[k];
  }
  double lam = -(pprev[0] * Ap[0] + pprev[1] * Ap[1] + pprev[2] * Ap[2] + pprev[3] * Ap[3]);
  if (!(lam > lo && lam < hi)) lam = hi;
  for (int it = 0; it < 40; ++it) {
    double L[4][4], dinv[4];
    if (!ldl4(M, lam, floor, L, dinv)) {
      lo = lam;  // not positive definite: lambda <= -a_min + floor
      lam = 0.5 * (lo + hi);
      continue;
    }
    double y[4];
#pragma unroll
    for (int k = 0; k < 4; ++k) {  // L y = -b
      double yk = -b[k];
#pragma unroll
      for (int l = 0; l < k; ++l) yk -= L[k][l] * y[l];
      y[k] = yk;
    }
#pragma unroll
    for (int k = 3; k >= 0; --k) {  // L^T x = D^{-1} y
      double xk = y[k] * dinv[k];
#pragma unroll
      for (int l = k + 1; l < 4; ++l) xk -= L[l][k] * x[l];
      x[k] = xk;
    }
    double u[4], q = 0.0;
#pragma unroll
    for (int k = 0; k < 4; ++k) {  // L u = x, q = u^T D^{-1} u
      double uk = x[k];
#pragma unroll
      for (int l = 0; l < k; ++l) uk -= L[k][l] * u[l];
      u[k] = uk;
      q += uk * uk * dinv[k];
    }
    const double nx2 = x[0] * x[0] + x[1] * x[1] + x[2] * x[2] + x[3] * x[3];
    const double nx = sqrt(nx2);
    if (fabs(nx - 1.0) <= 1e-14) return true;
    if (nx > 1.0) lo = lam; else hi = lam;
    if (hi - lo <= 1e-15 * fmax(1.0, fabs(lam))) return false;
    double next = lam + (nx - 1.0) * nx2 / q;
    if (!(next > lo && next < hi)) next = 0.5 * (lo + hi);
    lam = next;
  }
  return false;
}

// argmin over |x| = 1 of 1/2 x^T A x + b^T x (Lemma 1 / Lemma B.1), FP64:
// the factorisation path above, else the eigen-decomposition of A (Newton
// on the same phi with g = W^T b), which also covers the hard case.
__device__ void trs4(const double M[10], const double b[4], const double pprev[4], double x[4]) {
  if (trs4_ldl(M, b, pprev, x)) return;
  double w[4], V[4][4];
  jacobi4(M, w, V);
  int kmin = 0;
  for (int k = 1; k < 4; ++k)
    if (w[k] < w[kmin]) kmin = k;
  const double wmin = w[kmin];
  double g[4], nb2 = 0.0, wabs = 0.0;
  for (int k = 0; k < 4; ++k) {
    g[k] = V[0][k] * b[0] + V[1][k] * b[1] + V[2][k] * b[2] + V[3][k] * b[3];
    nb2 += b[k] * b[k];
    wabs = fmax(wabs, fabs(w[k]));
  }
  const double nb = sqrt(nb2);
  const double scale = fmax(1.0, fmax(wabs, nb));
  bool low[4];
  double glow2 = 0.0;
  for (int k = 0; k < 4; ++k) {
    low[k] = fabs(w[k] - wmin) <= 1e-12 * scale;
    if (low[k]) glow2 += g[k] * g[k];
  }
  double rest0 = 0.0;  // |x|^2 at lambda = -wmin without the lowest eigenspace
  for (int k = 0; k < 4; ++k)
    if (!low[k]) rest0 += g[k] * g[k] / ((w[k] - wmin) * (w[k] - wmin));
  const bool hard = sqrt(glow2) <= 1e-14 * scale && rest0 <= 1.0;
  double lam;
  if (!hard) {
    // bracket [lo, hi] of the root of |x(lambda)| = 1 on (-wmin, inf)
    double lo = -wmin, hi = nb - wmin;
    lam = hi;
    for (int it = 0; it < 100; ++it) {
      double n2 = 0.0, d3 = 0.0;
      for (int k = 0; k < 4; ++k) {
        const double den = w[k] + lam;
        const double gk = g[k] / den;
        n2 += gk * gk;
        d3 += gk * gk / den;
      }
      const double nx = sqrt(n2);
      const double phi = 1.0 / nx - 1.0;  // increasing in lambda
      if (phi < 0.0) lo = lam; else hi = lam;
      if (fabs(phi) <= 1e-15 || hi - lo <= 1e-16 * fmax(1.0, fabs(lam))) break;
      const double dphi = d3 / (n2 * nx);  // d(1/|x|)/dlambda
      double next = lam - phi / dphi;
      if (!(next > lo && next < hi)) next = 0.5 * (lo + hi);
      lam = next;
    }
    for (int r = 0; r < 4; ++r) {
      double s = 0.0;
      for (int k = 0; k < 4; ++k) s += V[r][k] * (-g[k] / (w[k] + lam));
      x[r] = s;
    }
    return;
  }
  lam = -wmin;
  double n0 = 0.0;
  for (int r = 0; r < 4; ++r) x[r] = 0.0;
  for (int k = 0; k < 4; ++k)
    if (!low[k]) {
      const double ck = -g[k] / (w[k] + lam);
      n0 += ck * ck;
      for (int r = 0; r < 4; ++r) x[r] += V[r][k] * ck;
    }
  const double rem = sqrt(fmax(0.0, 1.0 - n0));
  // the minimisers are x + y, y in the lowest eigenspace with |y| = rem;
  // the one nearest p^k takes y along p^k's projection on that space
  double y[4] = {0.0, 0.0, 0.0, 0.0};
  for (int k = 0; k < 4; ++k)
    if (low[k]) {
      const double d = V[0][k] * pprev[0] + V[1][k] * pprev[1] + V[2][k] * pprev[2] +
                       V[3][k] * pprev[3];
      for (int r = 0; r < 4; ++r) y[r] += d * V[r][k];
    }
  const double ny = sqrt(y[0] * y[0] + y[1] * y[1] + y[2] * y[2] + y[3] * y[3]);
  for (int r = 0; r < 4; ++r) x[r] += rem * (ny > 0.0 ? y[r] / ny : V[r][kmin]);
}

// SPD solves by Cholesky (upper-triangle storage)
template <typename A>
__device__ void chol_solve4(const A M[10], const A b[4], A x[4]) {
  A L[4][4] = {};
  for (int j = 0; j < 4; ++j) {
    A s = M[uidx(j, j)];
    for (int k = 0; k < j; ++k) s -= L[j][k] * L[j][k];
    L[j][j] = sqrt(s);
    for (int i = j + 1; i < 4; ++i) {
      A t = M[uidx(j, i)];
      for (int k = 0; k < j; ++k) t -= L[i][k] * L[j][k];
      L[i][j] = t / L[j][j];
    }
  }
  A y[4];
  for (int i = 0; i < 4; ++i) {
    A s = b[i];
    for (int k = 0; k < i; ++k) s -= L[i][k] * y[k];
    y[i] = s / L[i][i];
  }
  for (int i = 3; i >= 0; --i) {
    A s = y[i];
    for (int k = i + 1; k < 4; ++k) s -= L[k][i] * x[k];
    x[i] = s / L[i][i];
  }
}

template <typename A>
__device__ V3<A> sym_solve3(const Sym3<A>& S, A add, const V3<A>& b) {
  const A a11 = S.xx + add, a22 = S.yy + add, a33 = S.zz + add;
  const A a12 = S.xy, a13 = S.xz, a23 = S.yz;
  const A c11 = a22 * a33 - a23 * a23, c12 = a13 * a23 - a12 * a33, c13 = a12 * a23 - a13 * a22;
  const A c22 = a11 * a33 - a13 * a13, c23 = a12 * a13 - a11 * a23, c33 = a11 * a22 - a12 * a12;
  const A det = a11 * c11 + a12 * c12 + a13 * c13;
  return {(c11 * b.x + c12 * b.y + c13 * b.z) / det, (c12 * b.x + c22 * b.y + c23 * b.z) / det,
          (c13 * b.x + c23 * b.y + c33 * b.z) / det};
}

template <typename T>
__device__ __forceinline__ Q4<T> qmul_pure_r(const Q4<T>& a, const V3<T>& b) {  // a (x) [0, b]
  return {-a.x * b.x - a.y * b.y - a.z * b.z, a.w * b.x + a.y * b.z - a.z * b.y,
          a.w * b.y - a.x * b.z + a.z * b.x, a.w * b.z + a.x * b.y - a.y * b.x};
}

// ---------------------------------------------------------------------------
// vertex updates
// ---------------------------------------------------------------------------
template <typename T>
__device__ void vertex_P_own(const DevAniso<T>& a, const State<T>& st, int i,
                             const SweepParams& sp, const Q4<T>& qi_, const V3<T>& si_,
                             const Q4<T>& pi_, const Q4<T>& li_) {
  const DevGraph<T>& g = a.g;
  using A = double;  // the sphere-constrained solve is conditioned by A1's spectrum
  const Q4<A> qi = cvt<A>(qi_);
  const V3<A> si = {A(si_.x), A(si_.y), A(si_.z)};
  A M[10] = {0, 0, 0, 0, 0, 0, 0, 0, 0, 0};
  A bv[4] = {0, 0, 0, 0};
  A diag = A(sp.beta) + A(sp.h1);
  struct OutE {
    P4<T> tt;
    V3<T> tj;
    V3<T> Sa, Sb;
  };
  edge_loop<kUA<T>>(
      g.o_ptr[i], g.o_ptr[i + 1],
      [&](int e) { return OutE{g.o_tt[e], st.t(g.o_nbr[e]), a.o_Sa[e], a.o_Sb[e]}; },
      [&](const OutE& d) {
        const Sym3<A> S = sym3<A>(d.Sa, d.Sb);
        const V3<A> tm = {A(d.tt.x), A(d.tt.y), A(d.tt.z)};
        const Q4<A> u = qmul_pure_r(qi, tm);  // q_i (x) [0, t~]
        Q4<A> c[4];
        cols_right(u, c);
        const V3<A> Sr = smul(S, V3<A>{A(d.tj.x) - si.x, A(d.tj.y) - si.y, A(d.tj.z) - si.z});
        add_quadratic(c, A(d.tt.u), S, Sr, M, bv, A(-1));
      });
  struct InE {
    Q4<T> ql, w;
  };
  edge_loop<kUA<T>>(
      g.i_ptr[i], g.i_ptr[i + 1], [&](int e) { return InE{st.q(g.i_nbr[e]), g.i_w[e]}; },
      [&](const InE& d) {
        const Q4<A> ql = cvt<A>(d.ql);
        const Q4<A> w = cvt<A>(d.w);
        const A kap = sqrt(w.w * w.w + w.x * w.x + w.y * w.y + w.z * w.z);
        diag += A(2) * kap * (ql.w * ql.w + ql.x * ql.x + ql.y * ql.y + ql.z * ql.z);
        const Q4<A> t = qmul(ql, w);
        bv[0] -= A(2) * t.w; bv[1] -= A(2) * t.x; bv[2] -= A(2) * t.y; bv[3] -= A(2) * t.z;
      });
  M[0] += diag; M[4] += diag; M[7] += diag; M[9] += diag;
  const Q4<A> li = cvt<A>(li_), pi = cvt<A>(pi_);
  const A b = A(sp.beta), h = A(sp.h1);
  bv[0] -= b * qi.w + li.w + h * pi.w;
  bv[1] -= b * qi.x + li.x + h * pi.x;
  bv[2] -= b * qi.y + li.y + h * pi.y;
  bv[3] -= b * qi.z + li.z + h * pi.z;
  const A pp[4] = {pi.w, pi.x, pi.y, pi.z};
  A x[4];
  trs4(M, bv, pp, x);
  // the solvers stop within ~1e-14 of the sphere; the update lies on it
  const A nx = sqrt(x[0] * x[0] + x[1] * x[1] + x[2] * x[2] + x[3] * x[3]);
  st.p(i) = Q4<T>{T(x[0] / nx), T(x[1] / nx), T(x[2] / nx), T(x[3] / nx)};
}

template <typename T>
__device__ __forceinline__ void vertex_Q(const DevAniso<T>& a, const State<T>& st, int i,
                                         const SweepParams& sp, bool save) {
  const DevGraph<T>& g = a.g;
  const Q4<T> pi = st.p(i), qi = st.q(i), li = st.lam(i);
  const V3<T> si = st.s(i);
  const Q4<T> pic = qconj(pi);
  T M[10] = {0, 0, 0, 0, 0, 0, 0, 0, 0, 0};
  T bv[4] = {0, 0, 0, 0};
  T diag = T(sp.beta) + T(sp.h2);
  struct OutE {
    P4<T> tt;
    V3<T> tj;
    V3<T> Sa, Sb;
    Q4<T> pj, w;
  };
  edge_loop<kUA<T>>(
      g.o_ptr[i], g.o_ptr[i + 1],
      [&](int e) {
        const int j = g.o_nbr[e];
        return OutE{g.o_tt[e], st.t(j), a.o_Sa[e], a.o_Sb[e], st.p(j), g.o_w[e]};
      },
      [&](const OutE& d) {
        const Sym3<T> S = sym3<T>(d.Sa, d.Sb);
        const Q4<T> v = qmul_pv(V3<T>{d.tt.x, d.tt.y, d.tt.z}, pic);  // [0, t~] (x) p_i^*
        Q4<T> c[4];
        cols_left(v, c);
        const V3<T> Sr = smul(S, V3<T>{d.tj.x - si.x, d.tj.y - si.y, d.tj.z - si.z});
        add_quadratic(c, d.tt.u, S, Sr, M, bv, T(1));
        const Q4<T> pj = d.pj, w = d.w;
        const T kap = sqrt(w.w * w.w + w.x * w.x + w.y * w.y + w.z * w.z);
        diag += T(2) * kap * (pj.w * pj.w + pj.x * pj.x + pj.y * pj.y + pj.z * pj.z);
        const Q4<T> t = qmul(pj, qconj(w));
        bv[0] += T(2) * t.w; bv[1] += T(2) * t.x; bv[2] += T(2) * t.y; bv[3] += T(2) * t.z;
      });
  M[0] += diag; M[4] += diag; M[7] += diag; M[9] += diag;
  const T b = T(sp.beta), h = T(sp.h2);
  bv[0] += b * pi.w - li.w + h * qi.w;
  bv[1] += b * pi.x - li.x + h * qi.x;
  bv[2] += b * pi.y - li.y + h * qi.y;
  bv[3] += b * pi.z - li.z + h * qi.z;
  T x[4];
  chol_solve4(M, bv, x);
  const Q4<T> qn = {x[0], x[1], x[2], x[3]};
  const T gb = T(sp.gamma * sp.beta);
  if (save) {
    g.q_prev[i] = qi;
    g.lam_prev[i] = li;
  }
  st.q(i) = qn;
  st.lam(i) = Q4<T>{li.w - gb * (pi.w - qn.w), li.x - gb * (pi.x - qn.x), li.y - gb * (pi.y - qn.y),
              li.z - gb * (pi.z - qn.z)};
}

template <typename T>
__device__ __forceinline__ void vertex_T(const DevAniso<T>& a, const State<T>& st, int i,
                                         const SweepParams& sp, bool save) {
  const DevGraph<T>& g = a.g;
  V3<T> acc = {T(0), T(0), T(0)};
  // sum_in S_e (half the system matrix's constant part), formed from the
  // records the pass streams instead of loaded per vertex
  V3<T> sa = {T(0), T(0), T(0)}, sb = {T(0), T(0), T(0)};
  struct InE {
    P4<T> tt;
    V3<T> sl;
    V3<T> Sa, Sb;
    Q4<T> ql, pl;
  };
  edge_loop<kUA<T>>(
      g.i_ptr[i], g.i_ptr[i + 1],
      [&](int e) {
        const int l = g.i_nbr[e];
        return InE{g.i_tt[e], st.s(l), a.i_Sa[e], a.i_Sb[e], st.q(l), st.p(l)};
      },
      [&](const InE& d) {
        const V3<T> c = im_mul_conj(qmul_vp(d.ql, V3<T>{d.tt.x, d.tt.y, d.tt.z}), d.pl);
        const V3<T> y =
            smul(sym3<T>(d.Sa, d.Sb), V3<T>{d.sl.x + c.x, d.sl.y + c.y, d.sl.z + c.z});
        acc.x += y.x; acc.y += y.y; acc.z += y.z;
        sa.x += d.Sa.x; sa.y += d.Sa.y; sa.z += d.Sa.z;
        sb.x += d.Sb.x; sb.y += d.Sb.y; sb.z += d.Sb.z;
      });
  const V3<T> ti = st.t(i), si = st.s(i);
  const V3<T> zi = st.z(i);
  const T b = T(sp.beta), h = T(sp.h3);
  const V3<T> rhs = {T(2) * acc.x + b * si.x + zi.x + h * ti.x, T(2) * acc.y + b * si.y + zi.y + h * ti.y,
                     T(2) * acc.z + b * si.z + zi.z + h * ti.z};
  if (save) g.t_prev[i] = ti;
  st.t(i) = sym_solve3(sym3<T>(V3<T>{T(2) * sa.x, T(2) * sa.y, T(2) * sa.z},
                               V3<T>{T(2) * sb.x, T(2) * sb.y, T(2) * sb.z}),
                       b + h, rhs);
}

template <typename T>
__device__ __forceinline__ void vertex_S(const DevAniso<T>& a, const State<T>& st, int i,
                                         const SweepParams& sp, bool save,
                                         Q4<T>* p_out = nullptr, Q4<T>* q_out = nullptr,
                                         V3<T>* s_out = nullptr) {
  const DevGraph<T>& g = a.g;
  const Q4<T> pi = st.p(i), qi = st.q(i);
  V3<T> acc = {T(0), T(0), T(0)};
  V3<T> sa = {T(0), T(0), T(0)}, sb = {T(0), T(0), T(0)};  // sum_out S_e, as in T
  struct OutE {
    P4<T> tt;
    V3<T> tj;
    V3<T> Sa, Sb;
  };
  edge_loop<kUA<T>>(
      g.o_ptr[i], g.o_ptr[i + 1],
      [&](int e) { return OutE{g.o_tt[e], st.t(g.o_nbr[e]), a.o_Sa[e], a.o_Sb[e]}; },
      [&](const OutE& d) {
        const V3<T> c = im_mul_conj(qmul_vp(qi, V3<T>{d.tt.x, d.tt.y, d.tt.z}), pi);
        const V3<T> y =
            smul(sym3<T>(d.Sa, d.Sb), V3<T>{d.tj.x - c.x, d.tj.y - c.y, d.tj.z - c.z});
        acc.x += y.x; acc.y += y.y; acc.z += y.z;
        sa.x += d.Sa.x; sa.y += d.Sa.y; sa.z += d.Sa.z;
        sb.x += d.Sb.x; sb.y += d.Sb.y; sb.z += d.Sb.z;
      });
  const V3<T> ti = st.t(i), si = st.s(i);
  const V3<T> zi = st.z(i);
  const T b = T(sp.beta), h = T(sp.h4);
  const V3<T> rhs = {T(2) * acc.x + b * ti.x - zi.x + h * si.x, T(2) * acc.y + b * ti.y - zi.y + h * si.y,
                     T(2) * acc.z + b * ti.z - zi.z + h * si.z};
  const V3<T> sn = sym_solve3(sym3<T>(V3<T>{T(2) * sa.x, T(2) * sa.y, T(2) * sa.z},
                                      V3<T>{T(2) * sb.x, T(2) * sb.y, T(2) * sb.z}),
                              b + h, rhs);
  const T gb = T(sp.gamma * sp.beta);
  if (save) {
    g.s_prev[i] = si;
    g.z_prev[i] = zi;
  }
  st.s(i) = sn;
  st.z(i) = (V3<T>{zi.x - gb * (ti.x - sn.x), zi.y - gb * (ti.y - sn.y),
                       zi.z - gb * (ti.z - sn.z)});
  if (p_out) {
    *p_out = pi;
    *q_out = qi;
    *s_out = sn;
  }
}

template <int PH, typename T>
__device__ __forceinline__ void phase_a(const DevAniso<T>& a, const State<T>& st, int i,
                                        const SweepParams& sp, bool save) {
  if (PH == 0) vertex_P_own(a, st, i, sp, st.q(i), st.s(i), st.p(i), st.lam(i));
  if (PH == 1) vertex_Q(a, st, i, sp, save);
  if (PH == 2) vertex_T(a, st, i, sp, save);
  if (PH == 3) vertex_S(a, st, i, sp, save);
  if (PH == 4) {  // S of this sweep + P of the next
    Q4<T> pi, qi;
    V3<T> si;
    vertex_S(a, st, i, sp, false, &pi, &qi, &si);
    vertex_P_own(a, st, i, sp, qi, si, pi, st.lam(i));
  }
}

constexpr int kXcds = 8;

__device__ __forceinline__ int xcd_block() {
  const int b = blockIdx.x, nb = gridDim.x;
  const int xcd = b % kXcds, local = b / kXcds;
  const int per = nb / kXcds, rem = nb % kXcds;
  return xcd < rem ? xcd * (per + 1) + local : rem * (per + 1) + (xcd - rem) * per + local;
}

// At most 256 threads per workgroup: the FP64 sphere-constrained solve of the
// P update needs more than the 128 registers a 1024-thread group leaves.
constexpr int kMaxBlockA = 256;

template <int PH, typename T>
__global__ void __launch_bounds__(kMaxBlockA) k_phase_a(DevAniso<T> a, SweepParams sp, int save) {
  const int i = xcd_block() * blockDim.x + threadIdx.x;
  if (i >= a.g.n) return;
  if (sp.active && !sp.active[a.g.gid[i]]) return;
  if (sp.beta_g) sp.beta = sp.beta_g[a.g.gid[i]];
  phase_a<PH, T>(a, global_state(a.g), i, sp, save != 0);
}

// One persistent workgroup per graph with the LDS residency of the
// quaternion sweep: a graph keeps the first k of p, q, t, s, lambda, z in
// LDS for the whole launch, k the most whose slots fit.  Up to 512 threads:
// the P update's registers allow eight waves per CU, so one 512-thread
// workgroup with all of the CU's LDS runs as many waves as two 256-thread
// ones would.
constexpr int kMaxBlockGraphA = 512;

template <int kSlots, typename T>
__device__ __forceinline__ void graph_sweeps_a(const DevAniso<T>& a, int v0, int v1, int k,
                                               const SweepParams& sp, unsigned char* lds) {
  const State<T> st = state_load<kSlots>(a.g, v0, v1, lds);
  for (int i = v0 + threadIdx.x; i < v1; i += blockDim.x) phase_a<0, T>(a, st, i, sp, false);
  __syncthreads();
  for (int it = 0; it < k; ++it) {
    const bool save = it == k - 1;
    for (int i = v0 + threadIdx.x; i < v1; i += blockDim.x) phase_a<1, T>(a, st, i, sp, save);
    __syncthreads();
    for (int i = v0 + threadIdx.x; i < v1; i += blockDim.x) phase_a<2, T>(a, st, i, sp, save);
    __syncthreads();
    if (save) {
      for (int i = v0 + threadIdx.x; i < v1; i += blockDim.x) phase_a<3, T>(a, st, i, sp, true);
    } else {
      for (int i = v0 + threadIdx.x; i < v1; i += blockDim.x) phase_a<4, T>(a, st, i, sp, false);
    }
    __syncthreads();
  }
  state_store<kSlots>(a.g, st, v0, v1);
}

template <typename T>
__global__ void __launch_bounds__(kMaxBlockGraphA) k_graph_sweeps_a(
    DevAniso<T> a, const int32_t* __restrict__ voff, const int32_t* __restrict__ order, int k,
    SweepParams sp, int lds_bytes) {
  extern __shared__ unsigned char lds_raw[];
  const int gr = order[blockIdx.x];
  const int v0 = voff[gr], v1 = voff[gr + 1];
  if (sp.active && !sp.active[gr]) return;
  if (sp.beta_g) sp.beta = sp.beta_g[gr];
  const size_t n = size_t(v1 - v0);
  int slots = 0;
  while (slots < 6 && state_lds_bytes<T>(slots + 1, n) <= size_t(lds_bytes)) ++slots;
  switch (slots) {
    case 6: graph_sweeps_a<6, T>(a, v0, v1, k, sp, lds_raw); break;
    case 5: graph_sweeps_a<5, T>(a, v0, v1, k, sp, lds_raw); break;
    case 4: graph_sweeps_a<4, T>(a, v0, v1, k, sp, lds_raw); break;
    case 3: graph_sweeps_a<3, T>(a, v0, v1, k, sp, lds_raw); break;
    case 2: graph_sweeps_a<2, T>(a, v0, v1, k, sp, lds_raw); break;
    case 1: graph_sweeps_a<1, T>(a, v0, v1, k, sp, lds_raw); break;
    default: graph_sweeps_a<0, T>(a, v0, v1, k, sp, lds_raw); break;
  }
}

// edge records: tt = (t~, c_e), S_e as (xx, xy, xz), (yy, yz, zz)
template <typename T>
__global__ void k_fill_edges_a(const int32_t* __restrict__ perm, const double* __restrict__ tm,
                               const double* __restrict__ S9, int64_t m, P4<T>* __restrict__ tt,
                               V3<T>* __restrict__ Sa, V3<T>* __restrict__ Sb) {
  const int64_t k = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (k >= m) return;
  const int64_t e = perm[k];
  const double* S = S9 + 9 * e;
  const double c = (S[0] + S[4] + S[8]) / 3.0;
  tt[k] = P4<T>{T(tm[3 * e]), T(tm[3 * e + 1]), T(tm[3 * e + 2]), T(c)};
  Sa[k] = V3<T>{T(S[0]), T(S[1]), T(S[2])};
  Sb[k] = V3<T>{T(S[4]), T(S[5]), T(S[8])};
}

inline dim3 grid_of(int64_t count, int block) { return dim3(unsigned((count + block - 1) / block)); }

}  // namespace

template <typename T>
hipError_t launch_phase_sweeps_a(const DevAniso<T>& a, int k, const SweepParams& sp, int block,
                                 hipStream_t st) {
  if (a.g.n <= 0 || k <= 0) return hipSuccess;
  if (block <= 0 || block > kMaxBlockA || block % 64) return hipErrorInvalidValue;
  const int nb = (a.g.n + block - 1) / block;
  hipLaunchKernelGGL((k_phase_a<0, T>), dim3(nb), dim3(block), 0, st, a, sp, 0);
  for (int it = 0; it < k; ++it) {
    const int save = it == k - 1;
    hipLaunchKernelGGL((k_phase_a<1, T>), dim3(nb), dim3(block), 0, st, a, sp, save);
    hipLaunchKernelGGL((k_phase_a<2, T>), dim3(nb), dim3(block), 0, st, a, sp, save);
    if (save)
      hipLaunchKernelGGL((k_phase_a<3, T>), dim3(nb), dim3(block), 0, st, a, sp, 1);
    else
      hipLaunchKernelGGL((k_phase_a<4, T>), dim3(nb), dim3(block), 0, st, a, sp, 0);
    const hipError_t err = hipGetLastError();
    if (err != hipSuccess) return err;
  }
  return hipSuccess;
}

template <typename T>
hipError_t launch_graph_sweeps_a(const DevAniso<T>& a, const int32_t* voff, const int32_t* order,
                                 int G, int k, const SweepParams& sp, int block, int max_n, int lds,
                                 hipStream_t st) {
  if (G <= 0 || k <= 0) return hipSuccess;
  if (block <= 0 || block > kMaxBlockGraphA || block % 64) return hipErrorInvalidValue;
  // all six arrays of the largest graph, within the 160 KiB of a CU
  constexpr size_t kLds = 160 * 1024;
  size_t bytes = lds ? std::min(kLds, state_lds_bytes<T>(6, size_t(max_n))) : 0;
  if (bytes && hipFuncSetAttribute(reinterpret_cast<const void*>(&k_graph_sweeps_a<T>),
                                   hipFuncAttributeMaxDynamicSharedMemorySize,
                                   int(bytes)) != hipSuccess) {
    (void)hipGetLastError();  // clear a refused request; run without LDS residency
    bytes = 0;
  }
  hipLaunchKernelGGL((k_graph_sweeps_a<T>), dim3(G), dim3(block), bytes, st, a, voff, order, k,
                     sp, int(bytes));
  return hipGetLastError();
}

template <typename T>
hipError_t launch_fill_edges_a(const int32_t* perm, const double* tm, const double* S9, int64_t m,
                               P4<T>* tt, V3<T>* Sa, V3<T>* Sb, hipStream_t st) {
  if (m <= 0) return hipSuccess;
  hipLaunchKernelGGL((k_fill_edges_a<T>), grid_of(m, 256), dim3(256), 0, st, perm, tm, S9, m, tt,
                     Sa, Sb);
  return hipGetLastError();
}

#define PGO_ANISO_INST(T)                                                                         \
  template hipError_t launch_phase_sweeps_a<T>(const DevAniso<T>&, int, const SweepParams&, int,  \
                                               hipStream_t);                                      \
  template hipError_t launch_graph_sweeps_a<T>(const DevAniso<T>&, const int32_t*,               \
                                               const int32_t*, int, int, const SweepParams&,      \
                                               int, int, int, hipStream_t);                       \
  template hipError_t launch_fill_edges_a<T>(const int32_t*, const double*, const double*,       \
                                             int64_t, P4<T>*, V3<T>*, V3<T>*, hipStream_t);

PGO_ANISO_INST(float)
PGO_ANISO_INST(double)

}  // namespace pgo
