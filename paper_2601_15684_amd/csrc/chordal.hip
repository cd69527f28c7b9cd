// The PRADMM splitting applied to the chordal pose-graph cost: rotations as
// 3x3 matrices, the chordal distance of App. A.4 on every rotation
// measurement, translations as in model (1):
//
//   F(R, t) = sum_e tau_e |t_j - t_i - R_i t~_e|^2 + kappa_e |R_i R~_e - R_j|_F^2
//
// with duplicates P = Q (P_i in SO(3), Q_i a free 3x3 block), t = s and the
// multipliers Lambda (3x3) and z.  Every block update of the sweep is closed
// form; the P update is a 3x3 polar factor per vertex:
//
//   P  M_i = 2 sum_out (t_j - s_i)(tau t~_e)^T + 2 sum_in Q_l (kappa R~_e)
//          + beta Q_i + Lambda_i + H1 P_i,
//      P_i = argmax_{R in SO(3)} <R, M_i> = U diag(1, 1, det(U V^T)) V^T
//      (|P t~| = |t~| and |P|_F^2 = 3 make f, g and the penalty linear in P);
//   Q  Q_i = (2 sum_out P_j (kappa R~_e)^T + beta P_i - Lambda_i + H2 Q_i)
//            / (cQ_i + beta + H2),   Lambda_i -= gamma beta (P_i - Q_i);
//   T  t_i = (2 sum_in (tau s_l + P_l (tau t~_e)) + beta s_i + z_i + H3 t_i)
//            / (cT_i + beta + H3);
//   S  s_i = (2 sum_out (tau t_j - P_i (tau t~_e)) + beta t_i - z_i + H4 s_i)
//            / (cS_i + beta + H4),   z_i -= gamma beta (t_i - s_i).
//
// The schedule is the quaternion model's: P, then per sweep Q, T and S fused
// with the next sweep's P (P reads neighbours' t and Q only, both final
// before S starts), one thread per vertex, in-place and race-free, sums in
// edge order without atomics (bitwise identical across schedules).
//
// FP32 path: M_i is summed in float and its polar factor taken in float;
// when the factor is ill-conditioned relative to the size of the terms
// (gap = sigma_2 + sign(det M) sigma_3 below 1e-2 of the L1 size of all
// terms), M_i is summed again in double from the stored float values and
// factored in double.
//
// Multiply-adds are not contracted in this file: M_i is summed by two code
// paths (alone at the start of a launch, fused with S inside it) that must
// round identically, and the compiler's choice of fused multiply-adds
// depends on the code around an expression.
#pragma clang fp contract(off)
#include <algorithm>

#include "internal.hpp"
#include "polar.hpp"

namespace pgo {

namespace {

template <typename A, typename T>
__device__ __forceinline__ void ld9(const R3<T>& m, A out[9]) {
#pragma unroll
  for (int r = 0; r < 3; ++r) {
    const V3<T> row = m.r[r];
    out[3 * r] = A(row.x);
    out[3 * r + 1] = A(row.y);
    out[3 * r + 2] = A(row.z);
  }
}

template <typename T, typename A>
__device__ __forceinline__ R3<T> st9(const A m[9]) {
  R3<T> o;
#pragma unroll
  for (int r = 0; r < 3; ++r) o.r[r] = V3<T>{T(m[3 * r]), T(m[3 * r + 1]), T(m[3 * r + 2])};
  return o;
}

template <typename A>
__device__ __forceinline__ A l1_9(const A m[9]) {
  A s = A(0);
#pragma unroll
  for (int k = 0; k < 9; ++k) s += fabs(m[k]);
  return s;
}

// Where the state of the vertices being updated lives: each array either
// in global memory (base 0) or, in the per-graph kernel, in LDS for the
// graph's vertices v0.. (base v0); element j of an array is x[j - xb].
template <typename T>
struct StateC {
  R3<T>* P_;
  R3<T>* Q_;
  R3<T>* L_;
  V3<T>* t_;
  V3<T>* s_;
  V3<T>* z_;
  int Pb, Qb, Lb, tb, sb, zb;
  __device__ __forceinline__ R3<T>& P(int j) const { return P_[j - Pb]; }
  __device__ __forceinline__ R3<T>& Q(int j) const { return Q_[j - Qb]; }
  __device__ __forceinline__ R3<T>& L(int j) const { return L_[j - Lb]; }
  __device__ __forceinline__ V3<T>& t(int j) const { return t_[j - tb]; }
  __device__ __forceinline__ V3<T>& s(int j) const { return s_[j - sb]; }
  __device__ __forceinline__ V3<T>& z(int j) const { return z_[j - zb]; }
};

template <typename T>
__device__ __forceinline__ StateC<T> global_state(const DevChordal<T>& g) {
  return {g.P, g.Q, g.L, g.t, g.s, g.z, 0, 0, 0, 0, 0, 0};
}

// Out-edge part of M_i.  Each term (t_j - s_i) u_e^T (u_e = tau t~_e) is
// linear in s_i, so the sum over the out-edges is
//   sum (t_j - t_i) u_e^T + (t_i - s_i) (sum u_e)^T,
// and the first sum needs no s_i: the S update of the same vertex gathers it
// in its own pass over the out-edges, and P finishes it once the new s_i is
// known.  Both brackets are differences of nearby positions, which keeps
// FP32's relative accuracy where coordinates are large.
template <typename A>
struct MOut {
  A acc[9], u[3], mag;
};

template <typename A>
__device__ __forceinline__ void m_out_zero(MOut<A>& mo) {
#pragma unroll
  for (int k = 0; k < 9; ++k) mo.acc[k] = A(0);
  mo.u[0] = mo.u[1] = mo.u[2] = A(0);
  mo.mag = A(0);
}

template <typename A, bool kMag, typename T>
__device__ __forceinline__ void m_out_add(MOut<A>& mo, const A ti[3], const V3<T>& tj,
                                          const P4<T>& u) {
  const A d[3] = {A(tj.x) - ti[0], A(tj.y) - ti[1], A(tj.z) - ti[2]};
  const A uu[3] = {A(u.x), A(u.y), A(u.z)};
#pragma unroll
  for (int r = 0; r < 3; ++r)
#pragma unroll
    for (int c = 0; c < 3; ++c) mo.acc[3 * r + c] += d[r] * uu[c];
#pragma unroll
  for (int c = 0; c < 3; ++c) mo.u[c] += uu[c];
  if (kMag)
    mo.mag += (fabs(d[0]) + fabs(d[1]) + fabs(d[2])) * (fabs(uu[0]) + fabs(uu[1]) + fabs(uu[2]));
}

// M_i of the P update in accumulation type A from the state in type T; the
// out-edge part is taken from pre when the caller gathered it already.
// mag collects the L1 size of every term (FP32 conditioning check only).
template <typename A, typename T, bool kMag>
__device__ void p_matrix(const DevChordal<T>& g, const StateC<T>& st, int i, const SweepParams& sp,
                         const R3<T>& Qi_,
                         const V3<T>& ti_, const V3<T>& si_, const R3<T>& Pi_, const R3<T>& Li_,
                         A M[9], A& mag, const MOut<A>* pre = nullptr) {
  const A ti[3] = {A(ti_.x), A(ti_.y), A(ti_.z)};
  MOut<A> mo;
  if (pre) {
    mo = *pre;
  } else {
    m_out_zero(mo);
    struct OutE {
      V3<T> tj;
      P4<T> u;
    };
    edge_loop(
        g.o_ptr[i], g.o_ptr[i + 1], [&](int e) { return OutE{st.t(g.o_nbr[e]), g.o_tt[e]}; },
        [&](const OutE& x) { m_out_add<A, kMag>(mo, ti, x.tj, x.u); });
  }
  const A ds[3] = {ti[0] - A(si_.x), ti[1] - A(si_.y), ti[2] - A(si_.z)};  // t_i - s_i
  A acc[9];
#pragma unroll
  for (int a = 0; a < 3; ++a)
#pragma unroll
    for (int c = 0; c < 3; ++c) acc[3 * a + c] = ds[a] * mo.u[c] + mo.acc[3 * a + c];
  if (kMag)
    mag += mo.mag + (fabs(ds[0]) + fabs(ds[1]) + fabs(ds[2])) *
                        (fabs(mo.u[0]) + fabs(mo.u[1]) + fabs(mo.u[2]));
  struct InE {
    R3<T> Ql, W;
  };
  // FP32: two 3x3 pairs in flight here and in Q (95.6 -> 93.5 ms per 50
  // sweeps of the 4096-graph batch, no spills); FP64: one (two cost 7%)
  edge_loop<sizeof(T) == 4 ? 2 : 1>(
      g.i_ptr[i], g.i_ptr[i + 1], [&](int e) { return InE{st.Q(g.i_nbr[e]), g.i_R[e]}; },
      [&](const InE& x) {
        A Ql[9], W[9];
        ld9<A>(x.Ql, Ql);
        ld9<A>(x.W, W);
#pragma unroll
        for (int r = 0; r < 3; ++r)
#pragma unroll
          for (int c = 0; c < 3; ++c)
            acc[3 * r + c] += Ql[3 * r] * W[c] + Ql[3 * r + 1] * W[3 + c] + Ql[3 * r + 2] * W[6 + c];
        if (kMag) mag += l1_9(Ql) * l1_9(W);
      });
  A Qi[9], Pi[9], Li[9];
  ld9<A>(Qi_, Qi);
  ld9<A>(Pi_, Pi);
  ld9<A>(Li_, Li);
  const A b = A(sp.beta), h = A(sp.h1);
#pragma unroll
  for (int k = 0; k < 9; ++k) M[k] = A(2) * acc[k] + b * Qi[k] + Li[k] + h * Pi[k];
  if (kMag) mag = A(2) * mag + b * l1_9(Qi) + l1_9(Li) + h * l1_9(Pi);
}

// sigma_2 + sign(det M) sigma_3 with the singular values sorted descending:
// the smallest denominator in the derivative of the SO(3) factor.
template <typename A>
__device__ __forceinline__ A polar_gap(const A M[9], const A sig[3]) {
  A a = sig[0], b = sig[1], c = sig[2];
  if (a < b) { const A t = a; a = b; b = t; }
  if (b < c) { const A t = b; b = c; c = t; }
  if (a < b) { const A t = a; a = b; b = t; }
  return det3<A>(M) >= A(0) ? b + c : b - c;
}

// P update of vertex i from its own values (passed in, as the fused S+P
// phase has them in registers).  P_i is kept when M_i = 0.
template <typename T>
__device__ void vertex_P_own(const DevChordal<T>& g, const StateC<T>& st, int i,
                             const SweepParams& sp, const R3<T>& Qi, const V3<T>& ti,
                             const V3<T>& si, const R3<T>& Pi, const R3<T>& Li,
                             const MOut<T>* pre = nullptr) {
  constexpr bool kF32 = sizeof(T) == 4;
  T M[9], R[9], sig[3], mag = T(0);
  p_matrix<T, T, kF32>(g, st, i, sp, Qi, ti, si, Pi, Li, M, mag, pre);
  polar3<T>(M, R, sig);
  if (kF32 && !(polar_gap<T>(M, sig) >= T(1e-2) * mag)) {
    double Md[9], Rd[9], sd[3], dm = 0.0;
    p_matrix<double, T, false>(g, st, i, sp, Qi, ti, si, Pi, Li, Md, dm);
    polar3<double>(Md, Rd, sd);
    if (sd[0] > 0.0 || sd[1] > 0.0 || sd[2] > 0.0) st.P(i) = st9<T, double>(Rd);
    return;
  }
  if (sig[0] > T(0) || sig[1] > T(0) || sig[2] > T(0)) st.P(i) = st9<T, T>(R);
}

template <typename T>
__device__ __forceinline__ void vertex_Q(const DevChordal<T>& g, const StateC<T>& st, int i,
                                         const SweepParams& sp, bool save) {
  T acc[9];
#pragma unroll
  for (int k = 0; k < 9; ++k) acc[k] = T(0);
  struct OutE {
    R3<T> Pj, W;
  };
  edge_loop<sizeof(T) == 4 ? 2 : 1>(
      g.o_ptr[i], g.o_ptr[i + 1], [&](int e) { return OutE{st.P(g.o_nbr[e]), g.o_R[e]}; },
      [&](const OutE& x) {
        T Pj[9], W[9];
        ld9<T>(x.Pj, Pj);
        ld9<T>(x.W, W);
#pragma unroll
        for (int r = 0; r < 3; ++r)
#pragma unroll
          for (int c = 0; c < 3; ++c)  // (P_j W^T)[r][c] = sum_k P_j[r][k] W[c][k]
            acc[3 * r + c] += Pj[3 * r] * W[3 * c] + Pj[3 * r + 1] * W[3 * c + 1] +
                              Pj[3 * r + 2] * W[3 * c + 2];
      });
  T Pi[9], Qi[9], Li[9], Qn[9], Ln[9];
  const R3<T> Qold = st.Q(i), lam = st.L(i);
  ld9<T>(st.P(i), Pi);
  ld9<T>(Qold, Qi);
  ld9<T>(lam, Li);
  const T b = T(sp.beta), h = T(sp.h2);
  const T a = g.cQ[i] + b + h;
  const T gb = T(sp.gamma * sp.beta);
#pragma unroll
  for (int k = 0; k < 9; ++k) {
    Qn[k] = (T(2) * acc[k] + b * Pi[k] - Li[k] + h * Qi[k]) / a;
    Ln[k] = Li[k] - gb * (Pi[k] - Qn[k]);
  }
  if (save) {
    g.Q_prev[i] = Qold;
    g.L_prev[i] = lam;
  }
  st.Q(i) = st9<T, T>(Qn);
  st.L(i) = st9<T, T>(Ln);
}

template <typename T>
__device__ __forceinline__ V3<T> mat_vec(const R3<T>& m, const P4<T>& v) {
  return {m.r[0].x * v.x + m.r[0].y * v.y + m.r[0].z * v.z,
          m.r[1].x * v.x + m.r[1].y * v.y + m.r[1].z * v.z,
          m.r[2].x * v.x + m.r[2].y * v.y + m.r[2].z * v.z};
}

template <typename T>
__device__ __forceinline__ void vertex_T(const DevChordal<T>& g, const StateC<T>& st, int i,
                                         const SweepParams& sp, bool save) {
  V3<T> acc = {T(0), T(0), T(0)};
  T tau_in = T(0);  // sum_in tau: cT_i / 2, formed here instead of loaded
  struct InE {
    P4<T> u;
    V3<T> sl;
    R3<T> Pl;
  };
  edge_loop(
      g.i_ptr[i], g.i_ptr[i + 1],
      [&](int e) {
        const int l = g.i_nbr[e];
        return InE{g.i_tt[e], st.s(l), st.P(l)};
      },
      [&](const InE& x) {
        const V3<T> c = mat_vec(x.Pl, x.u);  // P_l (tau t~)
        acc.x += x.u.u * x.sl.x + c.x;
        acc.y += x.u.u * x.sl.y + c.y;
        acc.z += x.u.u * x.sl.z + c.z;
        tau_in += x.u.u;
      });
  const V3<T> ti = st.t(i), si = st.s(i);
  const V3<T> zi = st.z(i);
  const T b = T(sp.beta), h = T(sp.h3);
  const T a = T(2) * tau_in + b + h;
  if (save) g.t_prev[i] = ti;
  st.t(i) = V3<T>{(T(2) * acc.x + b * si.x + zi.x + h * ti.x) / a,
                  (T(2) * acc.y + b * si.y + zi.y + h * ti.y) / a,
                  (T(2) * acc.z + b * si.z + zi.z + h * ti.z) / a};
}

template <typename T>
__device__ __forceinline__ void vertex_S(const DevChordal<T>& g, const StateC<T>& st, int i,
                                         const SweepParams& sp, bool save,
                                         R3<T>* P_out = nullptr, R3<T>* Q_out = nullptr,
                                         V3<T>* t_out = nullptr, V3<T>* s_out = nullptr,
                                         MOut<T>* mo = nullptr) {
  constexpr bool kF32 = sizeof(T) == 4;
  const R3<T> Pi = st.P(i);
  const V3<T> ti = st.t(i), si = st.s(i);
  const T tiv[3] = {ti.x, ti.y, ti.z};
  V3<T> acc = {T(0), T(0), T(0)};
  T tau_out = T(0);  // sum_out tau: cS_i / 2, formed here instead of loaded
  struct OutE {
    P4<T> u;
    V3<T> tj;
  };
  edge_loop(
      g.o_ptr[i], g.o_ptr[i + 1], [&](int e) { return OutE{g.o_tt[e], st.t(g.o_nbr[e])}; },
      [&](const OutE& x) {
        const V3<T> c = mat_vec(Pi, x.u);  // P_i (tau t~)
        acc.x += x.u.u * x.tj.x - c.x;
        acc.y += x.u.u * x.tj.y - c.y;
        acc.z += x.u.u * x.tj.z - c.z;
        tau_out += x.u.u;
        if (mo) m_out_add<T, kF32>(*mo, tiv, x.tj, x.u);  // the next P's out-edge sum
      });
  const V3<T> zi = st.z(i);
  const T b = T(sp.beta), h = T(sp.h4);
  const T a = T(2) * tau_out + b + h;
  const V3<T> sn = {(T(2) * acc.x + b * ti.x - zi.x + h * si.x) / a,
                    (T(2) * acc.y + b * ti.y - zi.y + h * si.y) / a,
                    (T(2) * acc.z + b * ti.z - zi.z + h * si.z) / a};
  const T gb = T(sp.gamma * sp.beta);
  if (save) {
    g.s_prev[i] = si;
    g.z_prev[i] = zi;
  }
  st.s(i) = sn;
  st.z(i) = V3<T>{zi.x - gb * (ti.x - sn.x), zi.y - gb * (ti.y - sn.y), zi.z - gb * (ti.z - sn.z)};
  if (P_out) {
    *P_out = Pi;
    *Q_out = st.Q(i);
    *t_out = ti;
    *s_out = sn;
  }
}

template <int PH, typename T>
__device__ __forceinline__ void phase_c(const DevChordal<T>& g, const StateC<T>& st, int i,
                                        const SweepParams& sp, bool save) {
  if (PH == 0) vertex_P_own(g, st, i, sp, st.Q(i), st.t(i), st.s(i), st.P(i), st.L(i));
  if (PH == 1) vertex_Q(g, st, i, sp, save);
  if (PH == 2) vertex_T(g, st, i, sp, save);
  if (PH == 3) vertex_S(g, st, i, sp, save);
  if (PH == 4) {  // S of this sweep + P of the next
    R3<T> Pi, Qi;
    V3<T> ti, si;
    MOut<T> mo;
    m_out_zero(mo);
    vertex_S(g, st, i, sp, false, &Pi, &Qi, &ti, &si, &mo);
    vertex_P_own(g, st, i, sp, Qi, ti, si, Pi, st.L(i), &mo);
  }
}

constexpr int kXcds = 8;

// XCD-aware block renumbering (see the quaternion sweep): each XCD walks one
// contiguous range of vertices.
__device__ __forceinline__ int xcd_block() {
  const int b = blockIdx.x, nb = gridDim.x;
  const int xcd = b % kXcds, local = b / kXcds;
  const int per = nb / kXcds, rem = nb % kXcds;
  return xcd < rem ? xcd * (per + 1) + local : rem * (per + 1) + (xcd - rem) * per + local;
}

template <int PH, typename T>
__global__ void k_phase_c(DevChordal<T> g, SweepParams sp, int save) {
  const int i = xcd_block() * blockDim.x + threadIdx.x;
  if (i >= g.n) return;
  if (sp.active && !sp.active[g.gid[i]]) return;
  if (sp.beta_g) sp.beta = sp.beta_g[g.gid[i]];
  phase_c<PH, T>(g, global_state(g), i, sp, save != 0);
}

// One persistent workgroup per graph, as in the quaternion sweep, with the
// part of the graph's state that fits the launch's LDS held there for all k
// sweeps.  The arrays go to LDS in the order of what a byte saves per
// sweep: s and P are read and written by their owner and gathered by
// neighbours (s in T; P in Q and T), t and Q likewise with fewer reads, z and
// Lambda only by their owner.  A graph keeps the first kArrays of
// s, P, t, Q, z, Lambda whose slots fit.
// Each array starts on a 16-byte boundary, which keeps the wide loads of
// its records aligned.
__device__ __forceinline__ size_t align16(size_t b) { return (b + 15) & ~size_t(15); }

template <typename T>
__device__ __forceinline__ size_t lds_prefix_c(int k, size_t n) {
  // LDS bytes of the first k arrays of s, P, t, Q, z, Lambda for n vertices
  const size_t v = align16(sizeof(V3<T>) * n), r = align16(sizeof(R3<T>) * n);
  const size_t c[7] = {0, v, v + r, 2 * v + r, 2 * v + 2 * r, 3 * v + 2 * r, 3 * v + 3 * r};
  return c[k];
}

template <int kArrays, typename T>
__device__ __forceinline__ void graph_sweeps_c(const DevChordal<T>& g, int v0, int v1, int k,
                                               const SweepParams& sp, unsigned char* lds) {
  const int n = v1 - v0;
  StateC<T> st = global_state(g);
  unsigned char* at = lds;
  const size_t vb = align16(sizeof(V3<T>) * n), rb = align16(sizeof(R3<T>) * n);
  if (kArrays >= 1) st.s_ = reinterpret_cast<V3<T>*>(at), st.sb = v0, at += vb;
  if (kArrays >= 2) st.P_ = reinterpret_cast<R3<T>*>(at), st.Pb = v0, at += rb;
  if (kArrays >= 3) st.t_ = reinterpret_cast<V3<T>*>(at), st.tb = v0, at += vb;
  if (kArrays >= 4) st.Q_ = reinterpret_cast<R3<T>*>(at), st.Qb = v0, at += rb;
  if (kArrays >= 5) st.z_ = reinterpret_cast<V3<T>*>(at), st.zb = v0, at += vb;
  if (kArrays >= 6) st.L_ = reinterpret_cast<R3<T>*>(at), st.Lb = v0;
  if (kArrays >= 1) {
    for (int i = v0 + threadIdx.x; i < v1; i += blockDim.x) {
      st.s(i) = g.s[i];
      if (kArrays >= 2) st.P(i) = g.P[i];
      if (kArrays >= 3) st.t(i) = g.t[i];
      if (kArrays >= 4) st.Q(i) = g.Q[i];
      if (kArrays >= 5) st.z(i) = g.z[i];
      if (kArrays >= 6) st.L(i) = g.L[i];
    }
    __syncthreads();
  }
  for (int i = v0 + threadIdx.x; i < v1; i += blockDim.x) phase_c<0, T>(g, st, i, sp, false);
  __syncthreads();
  for (int it = 0; it < k; ++it) {
    const bool save = it == k - 1;
    for (int i = v0 + threadIdx.x; i < v1; i += blockDim.x) phase_c<1, T>(g, st, i, sp, save);
    __syncthreads();
    for (int i = v0 + threadIdx.x; i < v1; i += blockDim.x) phase_c<2, T>(g, st, i, sp, save);
    __syncthreads();
    if (save) {
      for (int i = v0 + threadIdx.x; i < v1; i += blockDim.x) phase_c<3, T>(g, st, i, sp, true);
    } else {
      for (int i = v0 + threadIdx.x; i < v1; i += blockDim.x) phase_c<4, T>(g, st, i, sp, false);
    }
    __syncthreads();
  }
  if (kArrays >= 1) {  // each thread writes back the slots only it wrote
    for (int i = v0 + threadIdx.x; i < v1; i += blockDim.x) {
      g.s[i] = st.s(i);
      if (kArrays >= 2) g.P[i] = st.P(i);
      if (kArrays >= 3) g.t[i] = st.t(i);
      if (kArrays >= 4) g.Q[i] = st.Q(i);
      if (kArrays >= 5) g.z[i] = st.z(i);
      if (kArrays >= 6) g.L[i] = st.L(i);
    }
  }
}

template <typename T>
__global__ void k_graph_sweeps_c(DevChordal<T> g, const int32_t* __restrict__ voff,
                                 const int32_t* __restrict__ order, int k, SweepParams sp,
                                 int lds_bytes) {
  extern __shared__ unsigned char lds_raw[];
  const int gr = order[blockIdx.x];
  const int v0 = voff[gr], v1 = voff[gr + 1];
  if (sp.active && !sp.active[gr]) return;
  if (sp.beta_g) sp.beta = sp.beta_g[gr];
  const size_t n = size_t(v1 - v0);
  int arrays = 0;
  while (arrays < 6 && lds_prefix_c<T>(arrays + 1, n) <= size_t(lds_bytes)) ++arrays;
  switch (arrays) {
    case 6: graph_sweeps_c<6, T>(g, v0, v1, k, sp, lds_raw); break;
    case 5: graph_sweeps_c<5, T>(g, v0, v1, k, sp, lds_raw); break;
    case 4: graph_sweeps_c<4, T>(g, v0, v1, k, sp, lds_raw); break;
    case 3: graph_sweeps_c<3, T>(g, v0, v1, k, sp, lds_raw); break;
    case 2: graph_sweeps_c<2, T>(g, v0, v1, k, sp, lds_raw); break;
    case 1: graph_sweeps_c<1, T>(g, v0, v1, k, sp, lds_raw); break;
    default: graph_sweeps_c<0, T>(g, v0, v1, k, sp, lds_raw); break;
  }
}

// ---------------------------------------------------------------------------
// preparation and state transfer
// ---------------------------------------------------------------------------
__global__ void k_project_rot(const double* __restrict__ R, int64_t count, double* __restrict__ out,
                              uint8_t* __restrict__ bad) {
  const int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i >= count) return;
  double a[9];
  for (int k = 0; k < 9; ++k) a[k] = R[9 * i + k];
  double dev = 0.0;
  for (int r = 0; r < 3; ++r)
    for (int s = 0; s < 3; ++s) {
      const double d = a[r] * a[s] + a[3 + r] * a[3 + s] + a[6 + r] * a[6 + s] - (r == s ? 1.0 : 0.0);
      dev += d * d;
    }
  const bool ok = det3<double>(a) > 0.0 && sqrt(dev) <= 1e-2;
  bad[i] = ok ? 0 : 1;
  double rot[9], sig[3];
  if (ok) {
    polar3<double>(a, rot, sig);
  } else {
    for (int k = 0; k < 9; ++k) rot[k] = (k % 4 == 0) ? 1.0 : 0.0;
  }
  for (int k = 0; k < 9; ++k) out[9 * i + k] = rot[k];
}

template <typename T>
__global__ void k_fill_edges_c(const int32_t* __restrict__ perm, const int32_t* __restrict__ nbr_src,
                               const double* __restrict__ R9, const double* __restrict__ tm,
                               const double* __restrict__ kappa, const double* __restrict__ tau,
                               int64_t m, int32_t* __restrict__ nbr, P4<T>* __restrict__ tt,
                               R3<T>* __restrict__ Rw) {
  const int64_t k = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (k >= m) return;
  const int64_t e = perm[k];
  nbr[k] = nbr_src[e];
  const double ta = tau[e], ka = kappa[e];
  tt[k] = P4<T>{T(ta * tm[3 * e]), T(ta * tm[3 * e + 1]), T(ta * tm[3 * e + 2]), T(ta)};
  double w[9];
  for (int c = 0; c < 9; ++c) w[c] = ka * R9[9 * e + c];
  Rw[k] = st9<T, double>(w);
}

// cQ_i = 2 sum_out kappa (FP64 sum); T and S form their sums of tau from
// the edge records they stream
template <typename T>
__global__ void k_vertex_consts_c(int32_t n, const int32_t* __restrict__ o_ptr,
                                  const int32_t* __restrict__ o_perm,
                                  const double* __restrict__ kappa, T* __restrict__ cQ) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  double q = 0.0;
  for (int k = o_ptr[i]; k < o_ptr[i + 1]; ++k) q += kappa[o_perm[k]];
  cQ[i] = T(2.0 * q);
}

template <typename T>
__global__ void k_init_state_c(DevChordal<T> g, const double* __restrict__ P0,
                               const double* __restrict__ t0) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= g.n) return;
  const R3<T> P = st9<T, double>(P0 + 9 * int64_t(i));
  const V3<T> t = V3<T>{T(t0[3 * i]), T(t0[3 * i + 1]), T(t0[3 * i + 2])};
  const R3<T> Z = {{V3<T>{T(0), T(0), T(0)}, V3<T>{T(0), T(0), T(0)},
                    V3<T>{T(0), T(0), T(0)}}};
  const V3<T> z3 = V3<T>{T(0), T(0), T(0)};
  g.P[i] = P;
  g.Q[i] = P;
  g.L[i] = Z;
  g.t[i] = t;
  g.s[i] = t;
  g.z[i] = z3;
  g.Q_prev[i] = P;
  g.L_prev[i] = Z;
  g.t_prev[i] = t;
  g.s_prev[i] = t;
  g.z_prev[i] = z3;
}

template <typename T>
__global__ void k_state_io_c(DevChordal<T> g, double* __restrict__ buf, int to_device) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= g.n) return;
  double* b = buf + 36 * int64_t(i);
  if (to_device) {
    g.P[i] = st9<T, double>(b);
    g.Q[i] = st9<T, double>(b + 9);
    g.t[i] = V3<T>{T(b[18]), T(b[19]), T(b[20])};
    g.s[i] = V3<T>{T(b[21]), T(b[22]), T(b[23])};
    g.L[i] = st9<T, double>(b + 24);
    g.z[i] = V3<T>{T(b[33]), T(b[34]), T(b[35])};
  } else {
    double v[9];
    ld9<double>(g.P[i], v);
    for (int k = 0; k < 9; ++k) b[k] = v[k];
    ld9<double>(g.Q[i], v);
    for (int k = 0; k < 9; ++k) b[9 + k] = v[k];
    const V3<T> t = g.t[i], s = g.s[i], z = g.z[i];
    b[18] = double(t.x); b[19] = double(t.y); b[20] = double(t.z);
    b[21] = double(s.x); b[22] = double(s.y); b[23] = double(s.z);
    ld9<double>(g.L[i], v);
    for (int k = 0; k < 9; ++k) b[24 + k] = v[k];
    b[33] = double(z.x); b[34] = double(z.y); b[35] = double(z.z);
  }
}

template <typename T>
__global__ void k_poses_c(DevChordal<T> g, double* __restrict__ R, double* __restrict__ t) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= g.n) return;
  if (R) {
    double v[9];
    ld9<double>(g.P[i], v);
    for (int k = 0; k < 9; ++k) R[9 * int64_t(i) + k] = v[k];
  }
  if (t) {
    const V3<T> x = g.t[i];
    t[3 * int64_t(i)] = double(x.x);
    t[3 * int64_t(i) + 1] = double(x.y);
    t[3 * int64_t(i) + 2] = double(x.z);
  }
}

dim3 grid_of(int64_t count, int block) { return dim3(unsigned((count + block - 1) / block)); }

}  // namespace

template <typename T>
hipError_t launch_phase_sweeps_c(const DevChordal<T>& g, int k, const SweepParams& sp, int block,
                                 hipStream_t st) {
  if (g.n <= 0 || k <= 0) return hipSuccess;
  if (block <= 0 || block > 1024 || block % 64) return hipErrorInvalidValue;
  const int nb = (g.n + block - 1) / block;
  hipLaunchKernelGGL((k_phase_c<0, T>), dim3(nb), dim3(block), 0, st, g, sp, 0);
  for (int it = 0; it < k; ++it) {
    const int save = it == k - 1;
    hipLaunchKernelGGL((k_phase_c<1, T>), dim3(nb), dim3(block), 0, st, g, sp, save);
    hipLaunchKernelGGL((k_phase_c<2, T>), dim3(nb), dim3(block), 0, st, g, sp, save);
    if (save)
      hipLaunchKernelGGL((k_phase_c<3, T>), dim3(nb), dim3(block), 0, st, g, sp, 1);
    else
      hipLaunchKernelGGL((k_phase_c<4, T>), dim3(nb), dim3(block), 0, st, g, sp, 0);
    const hipError_t err = hipGetLastError();
    if (err != hipSuccess) return err;
  }
  return hipSuccess;
}

template <typename T>
hipError_t launch_graph_sweeps_c(const DevChordal<T>& g, const int32_t* voff, const int32_t* order,
                                 int G, int k, const SweepParams& sp, int block, int max_n, int lds,
                                 hipStream_t st) {
  if (G <= 0 || k <= 0) return hipSuccess;
  if (block <= 0 || block > 1024 || block % 64) return hipErrorInvalidValue;
  // enough for all six arrays of the largest graph, within the 160 KiB of a CU
  constexpr size_t kLds = 160 * 1024;
  const size_t all = 3 * (sizeof(V3<T>) + sizeof(R3<T>));
  size_t bytes = lds ? std::min(kLds, all * size_t(max_n) + 6 * 16) : 0;  // + alignment slack
  if (bytes && hipFuncSetAttribute(reinterpret_cast<const void*>(&k_graph_sweeps_c<T>),
                                   hipFuncAttributeMaxDynamicSharedMemorySize,
                                   int(bytes)) != hipSuccess) {
    (void)hipGetLastError();  // clear a refused request; run without LDS residency
    bytes = 0;
  }
  hipLaunchKernelGGL((k_graph_sweeps_c<T>), dim3(G), dim3(block), bytes, st, g, voff, order, k,
                     sp, int(bytes));
  return hipGetLastError();
}

hipError_t launch_project_rot(const double* R, int64_t count, double* out, uint8_t* bad,
                              hipStream_t st) {
  if (count <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_project_rot, grid_of(count, 256), dim3(256), 0, st, R, count, out, bad);
  return hipGetLastError();
}

template <typename T>
hipError_t launch_fill_edges_c(const int32_t* perm, const int32_t* nbr_src, const double* R9,
                               const double* tm, const double* kappa, const double* tau, int64_t m,
                               int32_t* nbr, P4<T>* tt, R3<T>* Rw, hipStream_t st) {
  if (m <= 0) return hipSuccess;
  hipLaunchKernelGGL((k_fill_edges_c<T>), grid_of(m, 256), dim3(256), 0, st, perm, nbr_src, R9, tm,
                     kappa, tau, m, nbr, tt, Rw);
  return hipGetLastError();
}

template <typename T>
hipError_t launch_vertex_consts_c(int32_t n, const int32_t* o_ptr, const int32_t* o_perm,
                                  const double* kappa, T* cQ, hipStream_t st) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL((k_vertex_consts_c<T>), grid_of(n, 256), dim3(256), 0, st, n, o_ptr, o_perm,
                     kappa, cQ);
  return hipGetLastError();
}

template <typename T>
hipError_t launch_init_state_c(const DevChordal<T>& g, const double* P0, const double* t0,
                               hipStream_t st) {
  if (g.n <= 0) return hipSuccess;
  hipLaunchKernelGGL((k_init_state_c<T>), grid_of(g.n, 256), dim3(256), 0, st, g, P0, t0);
  return hipGetLastError();
}

template <typename T>
hipError_t launch_state_io_c(const DevChordal<T>& g, double* buf, int to_device, hipStream_t st) {
  if (g.n <= 0) return hipSuccess;
  hipLaunchKernelGGL((k_state_io_c<T>), grid_of(g.n, 256), dim3(256), 0, st, g, buf, to_device);
  return hipGetLastError();
}

template <typename T>
hipError_t launch_poses_c(const DevChordal<T>& g, double* R, double* t, hipStream_t st) {
  if (g.n <= 0) return hipSuccess;
  hipLaunchKernelGGL((k_poses_c<T>), grid_of(g.n, 256), dim3(256), 0, st, g, R, t);
  return hipGetLastError();
}

#define PGO_CHORDAL_INST(T)                                                                      \
  template hipError_t launch_phase_sweeps_c<T>(const DevChordal<T>&, int, const SweepParams&,   \
                                               int, hipStream_t);                                \
  template hipError_t launch_graph_sweeps_c<T>(const DevChordal<T>&, const int32_t*,            \
                                               const int32_t*, int, int, const SweepParams&,     \
                                               int, int, int, hipStream_t);                      \
  template hipError_t launch_fill_edges_c<T>(const int32_t*, const int32_t*, const double*,     \
                                             const double*, const double*, const double*,       \
                                             int64_t, int32_t*, P4<T>*, R3<T>*, hipStream_t);    \
  template hipError_t launch_vertex_consts_c<T>(int32_t, const int32_t*, const int32_t*,        \
                                                const double*, T*, hipStream_t);                 \
  template hipError_t launch_init_state_c<T>(const DevChordal<T>&, const double*, const double*, \
                                             hipStream_t);                                       \
  template hipError_t launch_state_io_c<T>(const DevChordal<T>&, double*, int, hipStream_t);    \
  template hipError_t launch_poses_c<T>(const DevChordal<T>&, double*, double*, hipStream_t);

PGO_CHORDAL_INST(float)
PGO_CHORDAL_INST(double)

}  // namespace pgo
