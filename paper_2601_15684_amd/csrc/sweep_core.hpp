// The PRADMM sweep on gfx950: four vertex-parallel phases per iteration
// (Alg. 1 steps 2-6), each a closed-form per-vertex update over the vertex's
// incident edges (App. B, scalar Sigma):
//
//   P  v_i = 2 sum_out [0, s_i - t_j] (x) q_i (x) [0, tau t~_e]
//          + 2 sum_in  q_l (x) (kappa q~_e) + beta q_i + lambda_i + H1 p_i
//      p_i = v_i / |v_i|                       (= -b1/|b1|, App. B.1; p kept if v = 0)
//   Q  q_i = (2 sum_out {[0, t_j - s_i] (x) p_i (x) [0, -tau t~_e]
//                        + p_j (x) (kappa q~_e)^*} + beta p_i - lambda_i + H2 q_i)
//            / (cQ_i + beta + H2)              (= A2^{-1} b2, App. B.2)
//      lambda_i -= gamma beta (p_i - q_i)      (eq. 3e)
//   T  t_i = (2 sum_in {tau s_l + Im(q_l (x) [0, tau t~_e] (x) p_l^*)}
//            + beta s_i + z_i + H3 t_i) / (cT_i + beta + H3)     (App. B.3)
//   S  s_i = (2 sum_out {tau t_j - Im(q_i (x) [0, tau t~_e] (x) p_i^*)}
//            + beta t_i - z_i + H4 s_i) / (cS_i + beta + H4)     (App. B.4)
//      z_i -= gamma beta (t_i - s_i)           (eq. 3f)
//
// Each fused product equals the paper's G-matrix expression by Lemma MW:
// G1^T r = r^* q_i t~ (G1 = M(q_i) M(t~) D), G2^T 1 = q_l q~ (G2 = W(q~) W(q_l) D),
// G3^T r = r p_i t~^*, G4^T 1 = p_j q~^*, G3^T G3 = |t~|^2 I, G4^T G4 = I.
//
// Inside a phase a vertex reads only values written by earlier phases, and
// writes only its own slots, so all updates are in place and race-free.
// Only three barriers per sweep are needed: P reads no neighbour's s (only
// neighbours' t and q, final before S starts, and its own new s), so the S
// of sweep k and the P of sweep k+1 run as one phase.  A k-sweep launch is
// P, then k times (Q, T, S+P), the last S+P being a plain S.
//
// Each edge record is read once per phase that needs it, and the three
// phases read 76 bytes per edge (FP32) between them:
//   * P's out-edge sum and Q's tau part are one linear map of two
//     quaternions.  For pure quaternions [0, a], [0, b] the product
//     [0, a] (x) q (x) [0, b] is linear in the outer product a b^T, so with
//     N = sum_out (s_i - t_j) u_j^T (u_e = tau t~_e, a 3x3 matrix)
//         sum_out [0, s_i - t_j] (x) q (x) [0, u_j] = K(N) q,
//         K(N) [w, v] = [-w tr N + v.c,  -N^T v + w c + tr(N) v - N v],
//     c the axial vector of N (c_x = N_yz - N_zy, ...), and Q's
//     sum_out [0, t_j - s_i] (x) p_i (x) [0, -u_j] is K(N) p_i with the same
//     N (Q reads t^k and s^k, the values S of the previous sweep finished).
//     The S pass gathers N, P applies it to q_i, and the new p_i gives
//     X_i = K(N) p_i, which the next Q starts its sum from: Q reads only
//     (neighbour, kappa q~) of each out-edge.  N is formed as
//     sum (t_i - t_j) u_j^T + (s_i - t_i) (sum u)^T, differences of nearby
//     positions, which keeps FP32's relative accuracy.
//   * P's in-edge sum Y_i = sum_in q_l (x) kappa q~ needs q at the values Q
//     just finished, so T gathers it in its own pass over the in-edges and
//     S+P reads no in-edge.
// A vertex's owner-only values -- lambda_i, z_i, and a slot xy_i that
// carries Y_i from T to S+P and then X_i from S+P to the next Q (with the
// magnitude of Y's terms for the FP32 check, xm_i) -- are passed to the
// vertex updates by reference: the per-graph kernel keeps them in
// registers for the whole launch, the per-phase launches in global memory.
// A P that opens a launch gathers N and Y itself, with the same arithmetic
// in the same edge order, so the per-phase launches and the per-graph
// kernel give identical bits, and so do k sweeps in one call and in several.
//
// Multiply-adds are not contracted in files that include this header: the
// P update runs in two code paths (alone at the start of a launch, fused
// with S inside it) that must round identically, and the compiler's choice
// of fused multiply-adds depends on the code around an expression.
#pragma once
#pragma clang fp contract(off)

#include "internal.hpp"

namespace pgo {

template <typename A, typename V>
__device__ __forceinline__ V3<A> v3a(const V& a) {  // first three components of P4 or V3
  return {A(a.x), A(a.y), A(a.z)};
}

template <typename A>
__device__ __forceinline__ void acc4(Q4<A>& s, const Q4<A>& t) {
  s.w += t.w; s.x += t.x; s.y += t.y; s.z += t.z;
}

// squared distance of two stored vectors, in FP64
template <typename T>
__device__ __forceinline__ double sq4(const Q4<T>& a, const Q4<T>& b) {
  const double w = double(a.w) - double(b.w), x = double(a.x) - double(b.x),
               y = double(a.y) - double(b.y), z = double(a.z) - double(b.z);
  return w * w + (x * x + y * y + z * z);
}

template <typename T>
__device__ __forceinline__ double sq3(const V3<T>& a, const V3<T>& b) {
  const double x = double(a.x) - double(b.x), y = double(a.y) - double(b.y),
               z = double(a.z) - double(b.z);
  return x * x + y * y + z * z;
}

template <typename A>
__device__ __forceinline__ A l1(const Q4<A>& t) {
  return fabs(t.w) + fabs(t.x) + fabs(t.y) + fabs(t.z);
}

template <typename A>
__device__ __forceinline__ A l1(const V3<A>& t) {
  return fabs(t.x) + fabs(t.y) + fabs(t.z);
}

// ---------------------------------------------------------------------------
// Where the gathered state (p, q, t, s) of the vertices being updated lives
// during a sweep: each array either in global memory (base 0) or, in a
// per-graph kernel, in LDS for the graph's vertices v0.. (base v0); element
// j of array k is ptr_k[j - base[k]].  Arrays in the order they are given
// LDS (HBM bytes each saves per sweep and per LDS byte: p is gathered by
// two phases, q, t, s by one; all are read by their owner in several).
// ---------------------------------------------------------------------------
constexpr int kArrays = 4;

template <typename T>
struct SwState {
  Q4<T>* p_;
  Q4<T>* q_;
  V3<T>* t_;
  V3<T>* s_;
  int b[kArrays];
  __device__ __forceinline__ Q4<T>& p(int j) const { return p_[j - b[0]]; }
  __device__ __forceinline__ Q4<T>& q(int j) const { return q_[j - b[1]]; }
  __device__ __forceinline__ V3<T>& t(int j) const { return t_[j - b[2]]; }
  __device__ __forceinline__ V3<T>& s(int j) const { return s_[j - b[3]]; }
};

template <typename T>
__device__ __forceinline__ SwState<T> sw_global(const DevGraph<T>& g) {
  return {g.p, g.q, g.t, g.s, {0, 0, 0, 0}};
}

// bytes per vertex of array k, and the LDS bytes of the first k arrays for
// n vertices (each array on a 16-byte boundary)
template <typename T>
__host__ __device__ __forceinline__ size_t sw_elem_bytes(int k) {
  return k < 2 ? 4 * sizeof(T) : 3 * sizeof(T);
}

template <typename T>
__host__ __device__ __forceinline__ size_t sw_lds_bytes(int k, size_t n) {
  size_t b = 0;
  for (int a = 0; a < k; ++a) b += (sw_elem_bytes<T>(a) * n + 15) & ~size_t(15);
  return b;
}

// ---------------------------------------------------------------------------
// The out-edge matrix N = sum (t_i - t_j) u_j^T, sum u_j and a magnitude
// bound (sum |t_i - t_j|_1 |u_j|_1) of the P terms, gathered in edge order.
// ---------------------------------------------------------------------------
template <typename A>
struct NSum {
  A n[9];
  V3<A> u;
  A mag;
};

template <typename A>
__device__ __forceinline__ NSum<A> nsum_zero() {
  NSum<A> r;
#pragma unroll
  for (int k = 0; k < 9; ++k) r.n[k] = A(0);
  r.u = {A(0), A(0), A(0)};
  r.mag = A(0);
  return r;
}

template <typename A, bool kMag, typename T>
__device__ __forceinline__ void nsum_add(NSum<A>& ns, const V3<A>& ti, const V3<T>& tj_,
                                         const P4<T>& u_) {
  const V3<A> tj = v3a<A>(tj_), u = v3a<A>(u_);
  const V3<A> d = {ti.x - tj.x, ti.y - tj.y, ti.z - tj.z};
  ns.n[0] += d.x * u.x; ns.n[1] += d.x * u.y; ns.n[2] += d.x * u.z;
  ns.n[3] += d.y * u.x; ns.n[4] += d.y * u.y; ns.n[5] += d.y * u.z;
  ns.n[6] += d.z * u.x; ns.n[7] += d.z * u.y; ns.n[8] += d.z * u.z;
  ns.u.x += u.x;
  ns.u.y += u.y;
  ns.u.z += u.z;
  if (kMag) ns.mag += l1(d) * l1(u);
}

// N of the P/Q out-edge sums: sum (s_i - t_j) u_j^T = sum (t_i - t_j) u_j^T
// + (s_i - t_i) (sum u)^T
template <typename A>
__device__ __forceinline__ void nsum_finish(NSum<A>& ns, const V3<A>& ti, const V3<A>& si) {
  const V3<A> r = {si.x - ti.x, si.y - ti.y, si.z - ti.z};
  ns.n[0] += r.x * ns.u.x; ns.n[1] += r.x * ns.u.y; ns.n[2] += r.x * ns.u.z;
  ns.n[3] += r.y * ns.u.x; ns.n[4] += r.y * ns.u.y; ns.n[5] += r.y * ns.u.z;
  ns.n[6] += r.z * ns.u.x; ns.n[7] += r.z * ns.u.y; ns.n[8] += r.z * ns.u.z;
  ns.mag += l1(r) * l1(ns.u);
}

// K(N) q = sum_j [0, a_j] (x) q (x) [0, b_j] for N = sum a_j b_j^T
template <typename A>
__device__ __forceinline__ Q4<A> kmul(const A (&N)[9], const Q4<A>& q) {
  const A tr = N[0] + N[4] + N[8];
  const V3<A> c = {N[5] - N[7], N[6] - N[2], N[1] - N[3]};
  const A vx = q.x, vy = q.y, vz = q.z;
  const V3<A> nv = {N[0] * vx + N[1] * vy + N[2] * vz, N[3] * vx + N[4] * vy + N[5] * vz,
                    N[6] * vx + N[7] * vy + N[8] * vz};
  const V3<A> ntv = {N[0] * vx + N[3] * vy + N[6] * vz, N[1] * vx + N[4] * vy + N[7] * vz,
                     N[2] * vx + N[5] * vy + N[8] * vz};
  return {(vx * c.x + vy * c.y + vz * c.z) - q.w * tr,
          ((q.w * c.x - ntv.x) + tr * vx) - nv.x,
          ((q.w * c.y - ntv.y) + tr * vy) - nv.y,
          ((q.w * c.z - ntv.z) + tr * vz) - nv.z};
}

// N (unfinished) over the out-edges of vertex i
template <typename A, bool kMag, int U = PGO_EDGE_UNROLL, typename T>
__device__ __forceinline__ NSum<A> gather_n(const DevGraph<T>& g, const SwState<T>& st, int i,
                                            const V3<A>& ti) {
  NSum<A> ns = nsum_zero<A>();
  struct OutE {
    V3<T> tj;
    P4<T> u;
  };
  edge_loop<U>(
      g.o_ptr[i], g.o_ptr[i + 1], [&](int e) { return OutE{st.t(g.o_nbr[e]), g.o_tt[e]}; },
      [&](const OutE& d) { nsum_add<A, kMag>(ns, ti, d.tj, d.u); });
  return ns;
}

// Y = sum_in q_l (x) kappa q~ over the in-edges of vertex i, and the L1 sum
// of its terms
template <typename A, bool kMag, int U = PGO_EDGE_UNROLL, typename T>
__device__ __forceinline__ Q4<A> gather_y(const DevGraph<T>& g, const SwState<T>& st, int i,
                                          A& mag) {
  Q4<A> y = {A(0), A(0), A(0), A(0)};
  struct InE {
    Q4<T> ql, w;
  };
  edge_loop<U>(
      g.i_ptr[i], g.i_ptr[i + 1], [&](int e) { return InE{st.q(g.i_nbr[e]), g.i_w[e]}; },
      [&](const InE& d) {
        const Q4<A> term = qmul(cvt<A>(d.ql), cvt<A>(d.w));
        acc4(y, term);
        if (kMag) mag += l1(term);
      });
  return y;
}

// The P update of vertex i in FP64 from the stored values (the FP32 path's
// island when its sum cancels); writes p_i and returns X_i.  Register-lean:
// v is accumulated term by term over the out- and in-edges, and X_i by a
// second pass over the out-edges once p_i is known.
template <typename T>
__device__ __forceinline__ Q4<T> p_island(const DevGraph<T>& g, const SwState<T>& st, int i,
                                          const SweepParams& sp, const Q4<T>& pi, const Q4<T>& li) {
  const Q4<double> qd = cvt<double>(st.q(i));
  const V3<double> sd = v3a<double>(st.s(i));
  const double bd = sp.beta, hd = sp.h1;
  Q4<double> v = {0.0, 0.0, 0.0, 0.0};
  const int o0 = g.o_ptr[i], o1 = g.o_ptr[i + 1];
#pragma unroll 1
  for (int e = o0; e < o1; ++e) {  // [0, s_i - t_j] q_i [0, u_e]
    const V3<double> tj = v3a<double>(st.t(g.o_nbr[e])), u = v3a<double>(g.o_tt[e]);
    acc4(v, qmul_vp(qmul_pv(V3<double>{sd.x - tj.x, sd.y - tj.y, sd.z - tj.z}, qd), u));
  }
#pragma unroll 1
  for (int e = g.i_ptr[i]; e < g.i_ptr[i + 1]; ++e)  // q_l kappa q~
    acc4(v, qmul(cvt<double>(st.q(g.i_nbr[e])), cvt<double>(g.i_w[e])));
  const Q4<double> ld = cvt<double>(li), pd = cvt<double>(pi);
  v = {2.0 * v.w + bd * qd.w + ld.w + hd * pd.w, 2.0 * v.x + bd * qd.x + ld.x + hd * pd.x,
       2.0 * v.y + bd * qd.y + ld.y + hd * pd.y, 2.0 * v.z + bd * qd.z + ld.z + hd * pd.z};
  const double dn = sqrt(v.w * v.w + v.x * v.x + v.y * v.y + v.z * v.z);
  Q4<T> pn = pi;
  if (dn > 0.0) pn = Q4<T>{T(v.w / dn), T(v.x / dn), T(v.y / dn), T(v.z / dn)};
  st.p(i) = pn;
  const Q4<double> pnd = cvt<double>(pn);
  Q4<double> x = {0.0, 0.0, 0.0, 0.0};
#pragma unroll 1
  for (int e = o0; e < o1; ++e) {  // [0, s_i - t_j] p_i [0, u_e]
    const V3<double> tj = v3a<double>(st.t(g.o_nbr[e])), u = v3a<double>(g.o_tt[e]);
    acc4(x, qmul_vp(qmul_pv(V3<double>{sd.x - tj.x, sd.y - tj.y, sd.z - tj.z}, pnd), u));
  }
  return Q4<T>{T(x.w), T(x.x), T(x.y), T(x.z)};
}

// The P update of vertex i from its own values and the two edge sums (N
// unfinished, Y with its magnitude); writes p_i and X_i = K(N) p_i (for the
// next Q) to x and returns true.  In FP32, when the sum cancels it writes
// nothing and returns false: the caller then runs p_island for the vertex,
// at once or after its other vertices of the phase (no vertex of a P phase
// reads another's p, and the island reads only stored values and lambda).
// The stored q_i, t_i, s_i equal qi, ti, si.
template <typename T>
__device__ __forceinline__ bool p_finish(const DevGraph<T>& g, const SwState<T>& st, int i,
                                         const SweepParams& sp, const Q4<T>& qi, const V3<T>& ti,
                                         const V3<T>& si, const Q4<T>& pi, const Q4<T>& li,
                                         NSum<T> ns, const Q4<T>& y, T ymag, Q4<T>& x) {
  constexpr bool kF32 = sizeof(T) == 4;
  nsum_finish(ns, ti, si);
  const Q4<T> out = kmul(ns.n, qi);
  const T b = T(sp.beta), h = T(sp.h1);
  const Q4<T> v = {T(2) * (out.w + y.w) + b * qi.w + li.w + h * pi.w,
                   T(2) * (out.x + y.x) + b * qi.x + li.x + h * pi.x,
                   T(2) * (out.y + y.y) + b * qi.y + li.y + h * pi.y,
                   T(2) * (out.z + y.z) + b * qi.z + li.z + h * pi.z};
  const T nrm = sqrt(v.w * v.w + v.x * v.x + v.y * v.y + v.z * v.z);
  if (kF32) {
    // FP64 island: when the sum cancels, both edge sums and the update are
    // redone in double from the stored values.
    const T tot = T(2) * (l1(qi) * ns.mag + ymag) + b * l1(qi) + l1(li) + h * l1(pi);
    if (!(nrm >= T(1e-3) * tot)) return false;
  }
  Q4<T> pn = pi;
  if (nrm > T(0)) pn = Q4<T>{v.w / nrm, v.x / nrm, v.y / nrm, v.z / nrm};
  st.p(i) = pn;
  x = kmul(ns.n, pn);
  return true;
}

// The P update that opens a launch: gathers both edge sums itself; writes
// X_i to x (false: the FP64 island is due, see p_finish).
template <int U = PGO_EDGE_UNROLL, typename T>
__device__ __forceinline__ bool vertex_P(const DevGraph<T>& g, const SwState<T>& st, int i,
                                         const SweepParams& sp, const Q4<T>& li, Q4<T>& x) {
  constexpr bool kF32 = sizeof(T) == 4;
  const Q4<T> qi = st.q(i), pi = st.p(i);
  const V3<T> ti = st.t(i), si = st.s(i);
  const NSum<T> ns = gather_n<T, kF32, U>(g, st, i, ti);
  T ymag = T(0);
  const Q4<T> y = gather_y<T, kF32, U>(g, st, i, ymag);
  return p_finish(g, st, i, sp, qi, ti, si, pi, li, ns, y, ymag, x);
}

// Q update of vertex i; x = X_i (the tau part of the out-edge sum), cq =
// cQ_i (a per-vertex constant the caller may hold in a register), lam is
// updated in place.
template <int U = PGO_EDGE_UNROLL, typename T>
__device__ __forceinline__ void vertex_Q(const DevGraph<T>& g, const SwState<T>& st, int i,
                                         const SweepParams& sp, bool save, Q4<T>& lam,
                                         const Q4<T>& x, T cq, double* dsq = nullptr) {
  const Q4<T> pi = st.p(i), qi = st.q(i), li = lam;
  Q4<T> acc = x;
  struct OutE {
    Q4<T> pj, w;
  };
  edge_loop<U>(
      g.o_ptr[i], g.o_ptr[i + 1], [&](int e) { return OutE{st.p(g.o_nbr[e]), g.o_w[e]}; },
      [&](const OutE& d) { acc4(acc, qmul(d.pj, qconj(d.w))); });
  const T b = T(sp.beta), h = T(sp.h2);
  const T a = cq + b + h;
  const Q4<T> qn = {(T(2) * acc.w + b * pi.w - li.w + h * qi.w) / a,
                    (T(2) * acc.x + b * pi.x - li.x + h * qi.x) / a,
                    (T(2) * acc.y + b * pi.y - li.y + h * qi.y) / a,
                    (T(2) * acc.z + b * pi.z - li.z + h * qi.z) / a};
  const T gb = T(sp.gamma * sp.beta);
  if (save) {
    g.q_prev[i] = qi;
    g.lam_prev[i] = li;
  }
  const Q4<T> ln = {li.w - gb * (pi.w - qn.w), li.x - gb * (pi.x - qn.x),
                    li.y - gb * (pi.y - qn.y), li.z - gb * (pi.z - qn.z)};
  st.q(i) = qn;
  lam = ln;
  if (dsq) {  // |dq|^2 and |dlambda|^2 of the stored values, FP64
    dsq[0] += sq4(qn, qi);
    dsq[1] += sq4(ln, li);
  }
}

// T update of vertex i; the same pass over the in-edges gathers the next
// P's in-edge sum Y_i (q is final after Q) and its terms' magnitude.
template <int U = PGO_EDGE_UNROLL, typename T>
__device__ __forceinline__ void vertex_T(const DevGraph<T>& g, const SwState<T>& st, int i,
                                         const SweepParams& sp, bool save, const V3<T>& zi,
                                         Q4<T>& y_out, T& ymag_out, double* dsq = nullptr) {
  constexpr bool kF32 = sizeof(T) == 4;
  V3<T> acc = {T(0), T(0), T(0)};
  Q4<T> y = {T(0), T(0), T(0), T(0)};
  T ymag = T(0);
  T tau_in = T(0);  // sum_in tau: cT_i / 2, formed here instead of loaded
  struct InE {
    P4<T> u;
    Q4<T> w;
    V3<T> sl;
    Q4<T> ql, pl;
  };
  edge_loop<U>(
      g.i_ptr[i], g.i_ptr[i + 1],
      [&](int e) {
        const int l = g.i_nbr[e];
        return InE{g.i_tt[e], g.i_w[e], st.s(l), st.q(l), st.p(l)};
      },
      [&](const InE& d) {
        const V3<T> c = im_mul_conj(qmul_vp(d.ql, v3(d.u)), d.pl);  // Im(q_l [0,tau t~] p_l^*)
        acc.x += d.u.u * d.sl.x + c.x;
        acc.y += d.u.u * d.sl.y + c.y;
        acc.z += d.u.u * d.sl.z + c.z;
        tau_in += d.u.u;
        const Q4<T> term = qmul(d.ql, d.w);
        acc4(y, term);
        if (kF32) ymag += l1(term);
      });
  const V3<T> ti = st.t(i), si = st.s(i);
  const T b = T(sp.beta), h = T(sp.h3);
  const T a = T(2) * tau_in + b + h;
  if (save) g.t_prev[i] = ti;
  const V3<T> tn = {(T(2) * acc.x + b * si.x + zi.x + h * ti.x) / a,
                    (T(2) * acc.y + b * si.y + zi.y + h * ti.y) / a,
                    (T(2) * acc.z + b * si.z + zi.z + h * ti.z) / a};
  st.t(i) = tn;
  y_out = y;
  ymag_out = ymag;
  if (dsq) dsq[2] += sq3(tn, ti);  // |dt|^2
}

// S update of vertex i (z updated in place).  The edge term
// Im(q_i [0, u_e] p_i^*) is linear in u_e, so the pass over the out-edges
// sums tau t_j and u_e only and rotates the sum once.  With kFuse, the same
// pass also gathers N and the P of the next sweep follows: xy holds Y_i on
// entry and X_i on return (false: the P's FP64 island is due and xy is
// unchanged, see p_finish).
template <bool kFuse, int U = PGO_EDGE_UNROLL, typename T>
__device__ __forceinline__ bool vertex_S(const DevGraph<T>& g, const SwState<T>& st, int i,
                                         const SweepParams& sp, bool save, V3<T>& z,
                                         const Q4<T>& lam, Q4<T>& xy, T ymag,
                                         double* dsq = nullptr) {
  constexpr bool kF32 = sizeof(T) == 4;
  const V3<T> ti = st.t(i);
  V3<T> acc = {T(0), T(0), T(0)};  // sum tau t_j
  T tau_out = T(0);                 // sum_out tau: cS_i / 2, formed here instead of loaded
  NSum<T> ns = nsum_zero<T>();      // ns.u: sum u_e (both forms)
  struct OutE {
    P4<T> u;
    V3<T> tj;
  };
  edge_loop<U>(
      g.o_ptr[i], g.o_ptr[i + 1], [&](int e) { return OutE{g.o_tt[e], st.t(g.o_nbr[e])}; },
      [&](const OutE& d) {
        acc.x += d.u.u * d.tj.x;
        acc.y += d.u.u * d.tj.y;
        acc.z += d.u.u * d.tj.z;
        tau_out += d.u.u;
        if (kFuse) {
          nsum_add<T, kF32>(ns, ti, d.tj, d.u);  // the next P's N (and sum u)
        } else {
          ns.u.x += d.u.x;
          ns.u.y += d.u.y;
          ns.u.z += d.u.z;
        }
      });
  const Q4<T> pi = st.p(i), qi = st.q(i);
  const V3<T> si = st.s(i);
  const V3<T> c = im_mul_conj(qmul_vp(qi, ns.u), pi);  // Im(q_i [0, sum u] p_i^*)
  const V3<T> zi = z;
  const T b = T(sp.beta), h = T(sp.h4);
  const T a = T(2) * tau_out + b + h;
  const V3<T> sn = {(T(2) * (acc.x - c.x) + b * ti.x - zi.x + h * si.x) / a,
                    (T(2) * (acc.y - c.y) + b * ti.y - zi.y + h * si.y) / a,
                    (T(2) * (acc.z - c.z) + b * ti.z - zi.z + h * si.z) / a};
  const T gb = T(sp.gamma * sp.beta);
  if (save) {
    g.s_prev[i] = si;
    g.z_prev[i] = zi;
  }
  st.s(i) = sn;
  const V3<T> zn = {zi.x - gb * (ti.x - sn.x), zi.y - gb * (ti.y - sn.y), zi.z - gb * (ti.z - sn.z)};
  z = zn;
  if (dsq) dsq[3] += sq3(zn, zi);  // |dz|^2
  if (kFuse) return p_finish(g, st, i, sp, qi, ti, sn, pi, lam, ns, xy, ymag, xy);
  return true;
}

}  // namespace pgo

namespace pgo {

// One phase of vertex i with its owner-only values in global memory
// (0 P, 1 Q, 2 T, 3 S, 4 S of this sweep + P of the next).
template <int PH, typename T>
__device__ __forceinline__ void phase_mem(const DevGraph<T>& g, const SwState<T>& st, int i,
                                          const SweepParams& sp, bool save,
                                          double* dsq = nullptr) {
  if (PH == 0) {
    const Q4<T> lam = g.lam[i];
    Q4<T> x;
    if (!vertex_P(g, st, i, sp, lam, x)) x = p_island(g, st, i, sp, st.p(i), lam);
    g.xy[i] = x;
  } else if (PH == 1) {
    Q4<T> lam = g.lam[i];
    vertex_Q(g, st, i, sp, save, lam, g.xy[i], g.cQ[i], dsq);
    g.lam[i] = lam;
  } else if (PH == 2) {
    Q4<T> y;
    T ym;
    vertex_T(g, st, i, sp, save, g.z[i], y, ym, dsq);
    g.xy[i] = y;
    if (sizeof(T) == 4) g.xm[i] = ym;
  } else {
    V3<T> z = g.z[i];
    if (PH == 4) {
      Q4<T> xy = g.xy[i];
      const T ym = sizeof(T) == 4 ? g.xm[i] : T(0);
      const Q4<T> lam = g.lam[i];
      if (!vertex_S<true>(g, st, i, sp, false, z, lam, xy, ym))
        xy = p_island(g, st, i, sp, st.p(i), lam);
      g.xy[i] = xy;
    } else {
      Q4<T> unused = {};
      vertex_S<false>(g, st, i, sp, save, z, Q4<T>{}, unused, T(0), dsq);
    }
    g.z[i] = z;
  }
}

}  // namespace pgo
