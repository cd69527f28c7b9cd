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
// Per-vertex sums run over the CSR/CSC segment in edge order, one thread per
// vertex, with no atomics: results are deterministic and identical between
// the per-phase launches and the per-graph persistent kernel.
//
// Multiply-adds are not contracted in this file: the P update runs in two
// code paths (alone at the start of a launch, fused with S inside it) that
// must round identically, so k sweeps in one launch equal k sweeps over
// several, and the compiler's choice of fused multiply-adds depends on the
// code around an expression.
#pragma clang fp contract(off)
#include <algorithm>

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

// Out-edge part of the P sum.  Each term [0, s_i - t_j] (x) q_i (x) [0, u_e]
// (u_e = tau t~_e) is linear in s_i, so the sum over the out-edges is
//   [0, s_i - t_i] (x) q_i (x) [0, sum u_e] + sum [0, t_i - t_j] (x) q_i (x) [0, u_e],
// and the second sum needs no s_i: the S update of the same vertex gathers
// it in its own pass over the out-edges, and P only finishes it once the new
// s_i is known.  Both brackets are differences of nearby positions, which
// keeps FP32's relative accuracy where coordinates are large.  mag collects
// the L1 size of every term (used only by the FP32 cancellation check).
template <typename A>
struct POut {
  Q4<A> x;
  V3<A> u;
  A mag;
};

template <typename A>
__device__ __forceinline__ POut<A> p_out_zero() {
  return {{A(0), A(0), A(0), A(0)}, {A(0), A(0), A(0)}, A(0)};
}

template <typename A, bool kMag, typename T>
__device__ __forceinline__ void p_out_add(POut<A>& po, const Q4<A>& qi, const V3<A>& ti,
                                          const V3<T>& tj_, const P4<T>& u_) {
  const V3<A> tj = v3a<A>(tj_), u = v3a<A>(u_);
  const V3<A> d = {ti.x - tj.x, ti.y - tj.y, ti.z - tj.z};
  const Q4<A> term = qmul_vp(qmul_pv(d, qi), u);
  acc4(po.x, term);
  po.u.x += u.x;
  po.u.y += u.y;
  po.u.z += u.z;
  if (kMag) po.mag += l1(term);
}

template <typename A, bool kMag>
__device__ __forceinline__ Q4<A> p_out_finish(const POut<A>& po, const Q4<A>& qi,
                                              const V3<A>& ti, const V3<A>& si, A& mag) {
  const V3<A> r = {si.x - ti.x, si.y - ti.y, si.z - ti.z};
  const Q4<A> head = qmul_vp(qmul_pv(r, qi), po.u);
  if (kMag) mag += po.mag + l1(head);
  return {head.w + po.x.w, head.x + po.x.x, head.y + po.x.y, head.z + po.x.z};
}

// Sum of the edge terms of the P phase, in accumulation type A; the
// out-edge part is taken from pre when the caller gathered it already.
template <typename A, typename T, bool kMag>
__device__ __forceinline__ Q4<A> p_edge_sum(const DevGraph<T>& g, const State<T>& st, int i,
                                            const Q4<T>& q_i, const V3<T>& t_i, const V3<T>& s_i,
                                            A& mag, const POut<A>* pre = nullptr) {
  const Q4<A> qi = cvt<A>(q_i);
  const V3<A> ti = v3a<A>(t_i);
  POut<A> po;
  if (pre) {
    po = *pre;
  } else {
    po = p_out_zero<A>();
    struct OutE {
      V3<T> tj;
      P4<T> u;
    };
    edge_loop(
        g.o_ptr[i], g.o_ptr[i + 1], [&](int e) { return OutE{st.t(g.o_nbr[e]), g.o_tt[e]}; },
        [&](const OutE& d) { p_out_add<A, kMag>(po, qi, ti, d.tj, d.u); });
  }
  Q4<A> acc = p_out_finish<A, kMag>(po, qi, ti, v3a<A>(s_i), mag);
  struct InE {
    Q4<T> ql, w;
  };
  edge_loop(
      g.i_ptr[i], g.i_ptr[i + 1], [&](int e) { return InE{st.q(g.i_nbr[e]), g.i_w[e]}; },
      [&](const InE& d) {
        const Q4<A> term = qmul(cvt<A>(d.ql), cvt<A>(d.w));
        acc4(acc, term);
        if (kMag) mag += l1(term);
      });
  return acc;
}

template <typename A, typename T>
__device__ __forceinline__ Q4<A> p_vector(const Q4<A>& acc, const Q4<T>& q_i, const Q4<T>& p_i,
                                          const Q4<T>& lam, const SweepParams& sp) {
  const Q4<A> qi = cvt<A>(q_i), li = cvt<A>(lam), pi = cvt<A>(p_i);
  const A b = A(sp.beta), h = A(sp.h1);
  return {A(2) * acc.w + b * qi.w + li.w + h * pi.w, A(2) * acc.x + b * qi.x + li.x + h * pi.x,
          A(2) * acc.y + b * qi.y + li.y + h * pi.y, A(2) * acc.z + b * qi.z + li.z + h * pi.z};
}

// P update of vertex i from its own values q_i, t_i, s_i, p_i, lambda_i
// (passed in, so a caller that has them in registers does not reload them)
// and, from the fused S+P phase, the out-edge sum S gathered.
template <typename T>
__device__ __forceinline__ void vertex_P_own(const DevGraph<T>& g, const State<T>& st, int i,
                                             const SweepParams& sp, const Q4<T>& qi,
                                             const V3<T>& ti, const V3<T>& si, const Q4<T>& pi,
                                             const Q4<T>& li, const POut<T>* pre = nullptr) {
  constexpr bool kF32 = sizeof(T) == 4;
  T mag = T(0);
  const Q4<T> acc = p_edge_sum<T, T, kF32>(g, st, i, qi, ti, si, mag, pre);
  const Q4<T> v = p_vector<T, T>(acc, qi, pi, li, sp);
  const T nrm = sqrt(v.w * v.w + v.x * v.x + v.y * v.y + v.z * v.z);
  if (kF32) {
    // FP64 island: when the sum cancels, redo it in double.
    const T tot = T(2) * mag + T(sp.beta) * l1(qi) + l1(li) + T(sp.h1) * l1(pi);
    if (!(nrm >= T(1e-3) * tot)) {
      double dm = 0.0;
      const Q4<double> dacc = p_edge_sum<double, T, false>(g, st, i, qi, ti, si, dm);
      const Q4<double> dv = p_vector<double, T>(dacc, qi, pi, li, sp);
      const double dn = sqrt(dv.w * dv.w + dv.x * dv.x + dv.y * dv.y + dv.z * dv.z);
      if (dn > 0.0)
        st.p(i) = Q4<T>{T(dv.w / dn), T(dv.x / dn), T(dv.y / dn), T(dv.z / dn)};
      return;
    }
  }
  if (nrm > T(0)) st.p(i) = Q4<T>{v.w / nrm, v.x / nrm, v.y / nrm, v.z / nrm};
}

template <typename T>
__device__ __forceinline__ void vertex_P(const DevGraph<T>& g, const State<T>& st, int i,
                                         const SweepParams& sp) {
  vertex_P_own(g, st, i, sp, st.q(i), st.t(i), st.s(i), st.p(i), st.lam(i));
}

template <typename T>
__device__ __forceinline__ void vertex_Q(const DevGraph<T>& g, const State<T>& st, int i,
                                         const SweepParams& sp, bool save,
                                         double* dsq = nullptr) {
  const Q4<T> pi = st.p(i), qi = st.q(i), li = st.lam(i);
  const V3<T> si = st.s(i);
  Q4<T> acc = {T(0), T(0), T(0), T(0)};
  struct OutE {
    V3<T> tj;
    P4<T> u;
    Q4<T> pj, w;
  };
  edge_loop(
      g.o_ptr[i], g.o_ptr[i + 1],
      [&](int e) {
        const int j = g.o_nbr[e];
        return OutE{st.t(j), g.o_tt[e], st.p(j), g.o_w[e]};
      },
      [&](const OutE& d) {
        const V3<T> tj = d.tj;
        const V3<T> r = {tj.x - si.x, tj.y - si.y, tj.z - si.z};
        const V3<T> mu = {-d.u.x, -d.u.y, -d.u.z};  // [0, tau t~]^*
        acc4(acc, qmul_vp(qmul_pv(r, pi), mu));
        acc4(acc, qmul(d.pj, qconj(d.w)));
      });
  const T b = T(sp.beta), h = T(sp.h2);
  const T a = g.cQ[i] + b + h;
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
  st.lam(i) = ln;
  if (dsq) {  // |dq|^2 and |dlambda|^2 of the stored values, FP64
    dsq[0] += sq4(qn, qi);
    dsq[1] += sq4(ln, li);
  }
}

template <typename T>
__device__ __forceinline__ void vertex_T(const DevGraph<T>& g, const State<T>& st, int i,
                                         const SweepParams& sp, bool save,
                                         double* dsq = nullptr) {
  V3<T> acc = {T(0), T(0), T(0)};
  struct InE {
    P4<T> u;
    V3<T> sl;
    Q4<T> ql, pl;
  };
  edge_loop(
      g.i_ptr[i], g.i_ptr[i + 1],
      [&](int e) {
        const int l = g.i_nbr[e];
        return InE{g.i_tt[e], st.s(l), st.q(l), st.p(l)};
      },
      [&](const InE& d) {
        const V3<T> c = im_mul_conj(qmul_vp(d.ql, v3(d.u)), d.pl);  // Im(q_l [0,tau t~] p_l^*)
        acc.x += d.u.u * d.sl.x + c.x;
        acc.y += d.u.u * d.sl.y + c.y;
        acc.z += d.u.u * d.sl.z + c.z;
      });
  const V3<T> ti = st.t(i), si = st.s(i), zi = st.z(i);
  const T b = T(sp.beta), h = T(sp.h3);
  const T a = g.cT[i] + b + h;
  if (save) g.t_prev[i] = ti;
  const V3<T> tn = {(T(2) * acc.x + b * si.x + zi.x + h * ti.x) / a,
                    (T(2) * acc.y + b * si.y + zi.y + h * ti.y) / a,
                    (T(2) * acc.z + b * si.z + zi.z + h * ti.z) / a};
  st.t(i) = tn;
  if (dsq) dsq[2] += sq3(tn, ti);  // |dt|^2
}

// S update of vertex i; with po, the same pass over the out-edges also
// gathers the next P's out-edge sum, and the vertex's own values are handed
// over in pi, qi, ti, si_new.
template <typename T>
__device__ __forceinline__ void vertex_S(const DevGraph<T>& g, const State<T>& st, int i,
                                         const SweepParams& sp, bool save,
                                         POut<T>* po = nullptr, Q4<T>* p_out = nullptr,
                                         Q4<T>* q_out = nullptr, V3<T>* t_out = nullptr,
                                         V3<T>* s_out = nullptr, double* dsq = nullptr) {
  constexpr bool kF32 = sizeof(T) == 4;
  const Q4<T> pi = st.p(i), qi = st.q(i);
  const V3<T> ti = st.t(i), si = st.s(i);
  const V3<T> tiv = ti;
  V3<T> acc = {T(0), T(0), T(0)};
  struct OutE {
    P4<T> u;
    V3<T> tj;
  };
  edge_loop(
      g.o_ptr[i], g.o_ptr[i + 1], [&](int e) { return OutE{g.o_tt[e], st.t(g.o_nbr[e])}; },
      [&](const OutE& d) {
        const V3<T> c = im_mul_conj(qmul_vp(qi, v3(d.u)), pi);  // Im(q_i [0,tau t~] p_i^*)
        acc.x += d.u.u * d.tj.x - c.x;
        acc.y += d.u.u * d.tj.y - c.y;
        acc.z += d.u.u * d.tj.z - c.z;
        if (po) p_out_add<T, kF32>(*po, qi, tiv, d.tj, d.u);  // the next P's out-edge sum
      });
  const V3<T> zi = st.z(i);
  const T b = T(sp.beta), h = T(sp.h4);
  const T a = g.cS[i] + b + h;
  const V3<T> sn = {(T(2) * acc.x + b * ti.x - zi.x + h * si.x) / a,
                    (T(2) * acc.y + b * ti.y - zi.y + h * si.y) / a,
                    (T(2) * acc.z + b * ti.z - zi.z + h * si.z) / a};
  const T gb = T(sp.gamma * sp.beta);
  if (save) {
    g.s_prev[i] = si;
    g.z_prev[i] = zi;
  }
  st.s(i) = sn;
  const V3<T> zn = {zi.x - gb * (ti.x - sn.x), zi.y - gb * (ti.y - sn.y), zi.z - gb * (ti.z - sn.z)};
  st.z(i) = zn;
  if (dsq) dsq[3] += sq3(zn, zi);  // |dz|^2
  if (p_out) {
    *p_out = pi;
    *q_out = qi;
    *t_out = ti;
    *s_out = sn;
  }
}

// S of one sweep fused with P of the next: P reads no neighbour's s, only
// its own new s and neighbour values finished before S began, so no barrier
// is needed between them; P reuses S's own values and the out-edge sum S
// gathered in its pass, so the out-edges are read once for both.
template <typename T>
__device__ __forceinline__ void vertex_SP(const DevGraph<T>& g, const State<T>& st, int i,
                                          const SweepParams& sp) {
  Q4<T> pi, qi;
  V3<T> ti, si;
  POut<T> po = p_out_zero<T>();
  vertex_S(g, st, i, sp, false, &po, &pi, &qi, &ti, &si);
  vertex_P_own(g, st, i, sp, qi, ti, si, pi, st.lam(i), &po);
}

// phase bodies: 0 P, 1 Q, 2 T, 3 S, 4 S of this sweep + P of the next
template <int PH, typename T>
__device__ __forceinline__ void phase(const DevGraph<T>& g, const State<T>& st, int i,
                                      const SweepParams& sp, bool save) {
  if (PH == 0) vertex_P(g, st, i, sp);
  if (PH == 1) vertex_Q(g, st, i, sp, save);
  if (PH == 2) vertex_T(g, st, i, sp, save);
  if (PH == 3) vertex_S(g, st, i, sp, save);
  if (PH == 4) vertex_SP(g, st, i, sp);
}

// ---------------------------------------------------------------------------
// one launch per phase
// ---------------------------------------------------------------------------
constexpr int kXcds = 8;

// Workgroups are dispatched to the 8 XCDs round-robin; renumber them so each
// XCD works on one contiguous range of vertices (neighbour gathers then hit
// that XCD's own L2).  A bijection on [0, gridDim.x).
__device__ __forceinline__ int xcd_block() {
  const int b = blockIdx.x, nb = gridDim.x;
  const int xcd = b % kXcds, local = b / kXcds;
  const int per = nb / kXcds, rem = nb % kXcds;
  return xcd < rem ? xcd * (per + 1) + local : rem * (per + 1) + (xcd - rem) * per + local;
}

template <int PH, typename T>
__global__ void k_phase(DevGraph<T> g, SweepParams sp, int save) {
  const int i = xcd_block() * blockDim.x + threadIdx.x;
  if (i >= g.n) return;
  if (sp.active && !sp.active[g.gid[i]]) return;
  if (sp.beta_g) sp.beta = sp.beta_g[g.gid[i]];
  phase<PH, T>(g, global_state(g), i, sp, save != 0);
}

template <typename T>
hipError_t launch_phase_sweeps(const DevGraph<T>& g, int k, const SweepParams& sp, int block,
                               hipStream_t st) {
  if (g.n <= 0 || k <= 0) return hipSuccess;
  if (block <= 0 || block > 1024 || block % 64) return hipErrorInvalidValue;
  const int nb = (g.n + block - 1) / block;
  hipLaunchKernelGGL((k_phase<0, T>), dim3(nb), dim3(block), 0, st, g, sp, 0);
  for (int it = 0; it < k; ++it) {
    const int save = it == k - 1;
    hipLaunchKernelGGL((k_phase<1, T>), dim3(nb), dim3(block), 0, st, g, sp, save);
    hipLaunchKernelGGL((k_phase<2, T>), dim3(nb), dim3(block), 0, st, g, sp, save);
    if (save)
      hipLaunchKernelGGL((k_phase<3, T>), dim3(nb), dim3(block), 0, st, g, sp, 1);
    else
      hipLaunchKernelGGL((k_phase<4, T>), dim3(nb), dim3(block), 0, st, g, sp, 0);
    const hipError_t err = hipGetLastError();
    if (err != hipSuccess) return err;
  }
  return hipSuccess;
}

// ---------------------------------------------------------------------------
// one persistent workgroup per graph: all k sweeps in one launch; the phase
// barrier is the workgroup barrier, so no grid-wide synchronisation exists.
// order[] lists graphs largest first (the hardware hands out workgroups in
// index order, which makes this a longest-first greedy schedule).
//
// A graph is updated by one workgroup only, so the part of its state that
// fits the launch's LDS stays there for all k sweeps (loaded once, written
// back once) and every read of it, the neighbour gathers included, is served
// on chip.  The arrays go to LDS in the order of what a slot saves per
// sweep: p, q and t are read by their owner and gathered by neighbours in
// two phases each, s in one, lambda and z only by their owner.  A graph of
// n vertices keeps the first kSlots of p, q, t, s, lambda, z there, kSlots
// the most that fit the launch's LDS (state_lds_bytes).
// ---------------------------------------------------------------------------
template <int kSlots, typename T>
__device__ __forceinline__ void graph_sweeps(const DevGraph<T>& g, int v0, int v1, int k,
                                             const SweepParams& sp, unsigned char* lds) {
  const State<T> st = state_load<kSlots>(g, v0, v1, lds);
  for (int i = v0 + threadIdx.x; i < v1; i += blockDim.x) phase<0, T>(g, st, i, sp, false);
  __syncthreads();
  for (int it = 0; it < k; ++it) {
    const bool save = it == k - 1;
    for (int i = v0 + threadIdx.x; i < v1; i += blockDim.x) phase<1, T>(g, st, i, sp, save);
    __syncthreads();
    for (int i = v0 + threadIdx.x; i < v1; i += blockDim.x) phase<2, T>(g, st, i, sp, save);
    __syncthreads();
    if (save) {
      for (int i = v0 + threadIdx.x; i < v1; i += blockDim.x) phase<3, T>(g, st, i, sp, true);
    } else {
      for (int i = v0 + threadIdx.x; i < v1; i += blockDim.x) phase<4, T>(g, st, i, sp, false);
    }
    __syncthreads();
  }
  state_store<kSlots>(g, st, v0, v1);
}

template <typename T>
__global__ void __launch_bounds__(1024) k_graph_sweeps(DevGraph<T> g,
                                                       const int32_t* __restrict__ voff,
                                                       const int32_t* __restrict__ order, int k,
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
    case 6: graph_sweeps<6, T>(g, v0, v1, k, sp, lds_raw); break;
    case 5: graph_sweeps<5, T>(g, v0, v1, k, sp, lds_raw); break;
    case 4: graph_sweeps<4, T>(g, v0, v1, k, sp, lds_raw); break;
    case 3: graph_sweeps<3, T>(g, v0, v1, k, sp, lds_raw); break;
    case 2: graph_sweeps<2, T>(g, v0, v1, k, sp, lds_raw); break;
    case 1: graph_sweeps<1, T>(g, v0, v1, k, sp, lds_raw); break;
    default: graph_sweeps<0, T>(g, v0, v1, k, sp, lds_raw); break;
  }
}

// The per-graph kernel with the stopping rule evaluated inside it (see
// launch_graph_sweeps_stop).  The four squared changes of a check sweep are
// summed in FP64 per thread, then over the workgroup: wave shuffles, one
// slot per wave, thread 0 adding the slots in order (deterministic).
constexpr int kStopSlots = 80;  // 16 waves x 4 sums, and the decision

__device__ __forceinline__ void block_sum4(double v[4], double* red) {
#pragma unroll
  for (int k = 0; k < 4; ++k)
    for (int off = 32; off > 0; off >>= 1) v[k] += __shfl_xor(v[k], off, 64);
  const int wave = int(threadIdx.x) / 64, nw = (int(blockDim.x) + 63) / 64;
  if (threadIdx.x % 64 == 0)
    for (int k = 0; k < 4; ++k) red[4 * wave + k] = v[k];
  __syncthreads();
  if (threadIdx.x == 0)
    for (int k = 0; k < 4; ++k) {
      double s = 0.0;
      for (int w = 0; w < nw; ++w) s += red[4 * w + k];
      v[k] = s;
    }
}

template <int kSlots, typename T>
__device__ __forceinline__ void graph_sweeps_stop(const DevGraph<T>& g, int gr, int v0, int v1,
                                                  int k, const SweepParams& sp,
                                                  unsigned char* lds, double* red) {
  const State<T> st = state_load<kSlots>(g, v0, v1, lds);
  const int C = sp.check_every;
  for (int i = v0 + threadIdx.x; i < v1; i += blockDim.x) phase<0, T>(g, st, i, sp, false);
  __syncthreads();
  int done = k;
  for (int it = 0; it < k; ++it) {
    const bool check = (it + 1) % C == 0;
    // |dq|^2, |dlambda|^2, |dt|^2, |dz|^2 of this sweep (kept in registers:
    // every sweep adds to them, a check sweep uses them)
    double d[4] = {0.0, 0.0, 0.0, 0.0};
    for (int i = v0 + threadIdx.x; i < v1; i += blockDim.x) vertex_Q(g, st, i, sp, check, d);
    __syncthreads();
    for (int i = v0 + threadIdx.x; i < v1; i += blockDim.x) vertex_T(g, st, i, sp, check, d);
    __syncthreads();
    if (!check) {
      for (int i = v0 + threadIdx.x; i < v1; i += blockDim.x) phase<4, T>(g, st, i, sp, false);
      __syncthreads();
      continue;
    }
    // a check sweep ends with a plain S, as the last sweep of any launch
    for (int i = v0 + threadIdx.x; i < v1; i += blockDim.x)
      vertex_S<T>(g, st, i, sp, true, nullptr, nullptr, nullptr, nullptr, nullptr, d);
    block_sum4(d, red);
    if (threadIdx.x == 0) {
      const double e = (d[1] + d[3]) / sp.beta + sp.beta * (d[0] + d[2]);
      red[kStopSlots - 1] = (e < sp.tol || it + 1 == k) ? 1.0 : 0.0;
    }
    __syncthreads();
    const bool stop = red[kStopSlots - 1] != 0.0;
    __syncthreads();  // the decision is read before the slots are reused
    if (stop) {
      done = it + 1;
      break;
    }
    for (int i = v0 + threadIdx.x; i < v1; i += blockDim.x) phase<0, T>(g, st, i, sp, false);
    __syncthreads();
  }
  state_store<kSlots>(g, st, v0, v1);
  if (threadIdx.x == 0) sp.done[gr] = done;
}

template <typename T>
__global__ void __launch_bounds__(1024) k_graph_sweeps_stop(DevGraph<T> g,
                                                            const int32_t* __restrict__ voff,
                                                            const int32_t* __restrict__ order,
                                                            int k, SweepParams sp, int lds_bytes) {
  extern __shared__ unsigned char lds_raw[];
  const int gr = order[blockIdx.x];
  const int v0 = voff[gr], v1 = voff[gr + 1];
  if (sp.active && !sp.active[gr]) {
    if (threadIdx.x == 0) sp.done[gr] = 0;
    return;
  }
  if (sp.beta_g) sp.beta = sp.beta_g[gr];
  double* red = reinterpret_cast<double*>(lds_raw);
  unsigned char* lds = lds_raw + sizeof(double) * kStopSlots;
  const size_t budget = size_t(lds_bytes) - sizeof(double) * kStopSlots;
  const size_t n = size_t(v1 - v0);
  int slots = 0;
  while (slots < 6 && state_lds_bytes<T>(slots + 1, n) <= budget) ++slots;
  switch (slots) {
    case 6: graph_sweeps_stop<6, T>(g, gr, v0, v1, k, sp, lds, red); break;
    case 5: graph_sweeps_stop<5, T>(g, gr, v0, v1, k, sp, lds, red); break;
    case 4: graph_sweeps_stop<4, T>(g, gr, v0, v1, k, sp, lds, red); break;
    case 3: graph_sweeps_stop<3, T>(g, gr, v0, v1, k, sp, lds, red); break;
    case 2: graph_sweeps_stop<2, T>(g, gr, v0, v1, k, sp, lds, red); break;
    case 1: graph_sweeps_stop<1, T>(g, gr, v0, v1, k, sp, lds, red); break;
    default: graph_sweeps_stop<0, T>(g, gr, v0, v1, k, sp, lds, red); break;
  }
}

constexpr size_t kLdsBytes = 160 * 1024;

template <typename T>
hipError_t launch_graph_sweeps_stop(const DevGraph<T>& g, const int32_t* voff,
                                    const int32_t* order, int G, int k, const SweepParams& sp,
                                    int block, int max_n, int lds, hipStream_t st) {
  if (G <= 0 || k <= 0) return hipSuccess;
  if (block <= 0 || block > 1024 || block % 64) return hipErrorInvalidValue;
  if (sp.check_every < 1 || k % sp.check_every || !sp.done) return hipErrorInvalidValue;
  const size_t red = sizeof(double) * kStopSlots;
  const size_t bytes =
      lds ? std::min(kLdsBytes, red + state_lds_bytes<T>(6, size_t(max_n))) : red;
  if (hipFuncSetAttribute(reinterpret_cast<const void*>(&k_graph_sweeps_stop<T>),
                          hipFuncAttributeMaxDynamicSharedMemorySize, int(bytes)) != hipSuccess)
    return hipGetLastError();
  hipLaunchKernelGGL((k_graph_sweeps_stop<T>), dim3(G), dim3(block), bytes, st, g, voff, order, k,
                     sp, int(bytes));
  return hipGetLastError();
}

template <typename T>
hipError_t launch_graph_sweeps(const DevGraph<T>& g, const int32_t* voff, const int32_t* order,
                               int G, int k, const SweepParams& sp, int block, int max_n,
                               int lds, hipStream_t st) {
  if (G <= 0 || k <= 0) return hipSuccess;
  if (block <= 0 || block > 1024 || block % 64) return hipErrorInvalidValue;
  // enough for all six arrays of the largest graph, within the 160 KiB of a CU
  size_t bytes = lds ? std::min(kLdsBytes, state_lds_bytes<T>(6, size_t(max_n))) : 0;
  if (bytes && hipFuncSetAttribute(reinterpret_cast<const void*>(&k_graph_sweeps<T>),
                                   hipFuncAttributeMaxDynamicSharedMemorySize,
                                   int(bytes)) != hipSuccess) {
    (void)hipGetLastError();  // clear a refused request; run without LDS residency
    bytes = 0;
  }
  hipLaunchKernelGGL((k_graph_sweeps<T>), dim3(G), dim3(block), bytes, st, g, voff, order, k, sp,
                     int(bytes));
  return hipGetLastError();
}

template hipError_t launch_phase_sweeps<float>(const DevGraph<float>&, int, const SweepParams&,
                                               int, hipStream_t);
template hipError_t launch_phase_sweeps<double>(const DevGraph<double>&, int,
                                                const SweepParams&, int, hipStream_t);
template hipError_t launch_graph_sweeps<float>(const DevGraph<float>&, const int32_t*,
                                               const int32_t*, int, int, const SweepParams&, int,
                                               int, int, hipStream_t);
template hipError_t launch_graph_sweeps<double>(const DevGraph<double>&, const int32_t*,
                                                const int32_t*, int, int, const SweepParams&, int,
                                                int, int, hipStream_t);
template hipError_t launch_graph_sweeps_stop<float>(const DevGraph<float>&, const int32_t*,
                                                    const int32_t*, int, int, const SweepParams&,
                                                    int, int, int, hipStream_t);
template hipError_t launch_graph_sweeps_stop<double>(const DevGraph<double>&, const int32_t*,
                                                     const int32_t*, int, int, const SweepParams&,
                                                     int, int, int, hipStream_t);

}  // namespace pgo
