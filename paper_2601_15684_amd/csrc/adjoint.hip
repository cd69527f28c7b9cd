// Hand-written reverse mode of K unrolled PRADMM sweeps.
//
// A sweep x^k -> x^{k+1} is the composition P, Q (+lambda), T, S (+z) of
// the per-vertex closed forms in sweep.hip.  Its adjoint runs the phases
// backwards, S, T, Q, P, one vertex per thread.  A vertex writes only its
// own adjoint slots; a contribution that belongs to a neighbour (the
// derivative with respect to a gathered value) is written as a message on
// the edge that carried it, and the next reverse phase gathers the
// messages of each vertex over the transposed incidence (in2out / out2in),
// in edge order.  No atomics: results are deterministic.
//
// Stored edge quantities a = tau t~, tau, w = kappa q~ and the vertex
// constants cQ, cT, cS receive FP64 gradient accumulators, turned at the
// end into gradients with respect to kappa, tau, t~ and the rotation
// perturbation omega (q~ = q~0 (x) E(omega), E(w) = [cos(|w|/2),
// sin(|w|/2) w/|w|], i.e. R~ = R~0 Exp(omega)).
//
// Conventions used below (Lemma MW): for A = x (x) q (x) y,
//   dq = x^* (x) dA (x) y^*,  dx = dA (x) (q (x) y)^*,  dy = (x (x) q)^* (x) dA.
#include "internal.hpp"

namespace pgo {

namespace {

template <typename T>
__device__ __forceinline__ void add3(P4<T>& a, const V3<T>& b) {
  a.x += b.x; a.y += b.y; a.z += b.z;
}
template <typename T>
__device__ __forceinline__ void add4(Q4<T>& a, const Q4<T>& b) {
  a.w += b.w; a.x += b.x; a.y += b.y; a.z += b.z;
}
template <typename T>
__device__ __forceinline__ V3<T> neg(const V3<T>& a) {
  return {-a.x, -a.y, -a.z};
}
template <typename T>
__device__ __forceinline__ V3<T> scale(const V3<T>& a, T s) {
  return {a.x * s, a.y * s, a.z * s};
}
template <typename T>
__device__ __forceinline__ T dot3v(const V3<T>& a, const V3<T>& b) {
  return a.x * b.x + a.y * b.y + a.z * b.z;
}
template <typename T>
__device__ __forceinline__ T dot4(const Q4<T>& a, const Q4<T>& b) {
  return a.w * b.w + a.x * b.x + a.y * b.y + a.z * b.z;
}

}  // namespace

namespace {

template <typename T>
__global__ void k_rev_S(DevGraph<T> g, StateRef<T> X, StateRef<T> Y, AdjRef<T> A, SweepParams sp,
                        int first) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= g.n) return;
  const int o0 = g.o_ptr[i], o1 = g.o_ptr[i + 1];
  const int n0 = g.i_ptr[i], n1 = g.i_ptr[i + 1];
  P4<T> tb = A.tb[i];
  Q4<T> qb = A.qb[i], pb = A.pb[i];
  if (!first) {  // messages of the P phase of the following sweep
    for (int n = n0; n < n1; ++n) add3(tb, v3(A.moP[A.in2out[n]]));
    for (int o = o0; o < o1; ++o) add4(qb, A.miP[A.out2in[o]]);
  }
  const T b = T(sp.beta), gb = T(sp.gamma * sp.beta);
  const V3<T> sbar0 = v3(A.sb[i]), zbar = v3(A.zb[i]);
  const V3<T> Sb = {sbar0.x + gb * zbar.x, sbar0.y + gb * zbar.y, sbar0.z + gb * zbar.z};
  const T D = g.cS[i] + b + T(sp.h4);
  const V3<T> N = scale(Sb, T(1) / D);
  A.csb[i] += -double(dot3v(Sb, v3(Y.s[i]))) / double(D);
  tb.x += -gb * zbar.x + b * N.x;
  tb.y += -gb * zbar.y + b * N.y;
  tb.z += -gb * zbar.z + b * N.z;
  const V3<T> Fb = scale(N, T(2));
  const Q4<T> Yp = Y.p[i], Yq = Y.q[i];
  for (int o = o0; o < o1; ++o) {
    const int j = g.o_nbr[o];
    const P4<T> u = g.o_tt[o];
    const V3<T> a = v3(u);
    A.ga_o[o].u += double(dot3v(Fb, v3(Y.t[j])));
    A.moS[o] = pad3(scale(Fb, u.u));
    // c = Im(q_i [0,a] p_i^*) enters with -: G = [0, -Fb]
    add4(qb, qmul_vp(qmul_pv(neg(Fb), Yp), neg(a)));
    add4(pb, qmul_vp(qmul_pv(Fb, Yq), a));
    const V3<T> ga = im(qmul(qmul_vp(qconj(Yq), neg(Fb)), Yp));
    A.ga_o[o].x += double(ga.x);
    A.ga_o[o].y += double(ga.y);
    A.ga_o[o].z += double(ga.z);
  }
  A.sb[i] = pad3(scale(N, T(sp.h4)));
  A.zb[i] = P4<T>{zbar.x - N.x, zbar.y - N.y, zbar.z - N.z, T(0)};
  A.tb[i] = tb;
  A.qb[i] = qb;
  A.pb[i] = pb;
}

template <typename T>
__global__ void k_rev_T(DevGraph<T> g, StateRef<T> X, StateRef<T> Y, AdjRef<T> A, SweepParams sp) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= g.n) return;
  const int n0 = g.i_ptr[i], n1 = g.i_ptr[i + 1];
  P4<T> tb = A.tb[i];
  for (int n = n0; n < n1; ++n) add3(tb, v3(A.moS[A.in2out[n]]));
  const T b = T(sp.beta);
  const V3<T> Tb = v3(tb);
  const T D = g.cT[i] + b + T(sp.h3);
  const V3<T> N = scale(Tb, T(1) / D);
  A.ctb[i] += -double(dot3v(Tb, v3(Y.t[i]))) / double(D);
  P4<T> sb = A.sb[i], zb = A.zb[i];
  add3(sb, scale(N, b));
  add3(zb, N);
  const V3<T> Eb = scale(N, T(2));
  for (int n = n0; n < n1; ++n) {
    const int l = g.i_nbr[n];
    const P4<T> u = g.i_tt[n];
    const V3<T> a = v3(u);
    A.ga_i[n].u += double(dot3v(Eb, v3(X.s[l])));
    A.miT3[n] = pad3(scale(Eb, u.u));
    const Q4<T> Yp = Y.p[l], Yq = Y.q[l];
    A.miT4q[n] = qmul_vp(qmul_pv(Eb, Yp), neg(a));
    A.miT4p[n] = qmul_vp(qmul_pv(neg(Eb), Yq), a);
    const V3<T> ga = im(qmul(qmul_vp(qconj(Yq), Eb), Yp));
    A.ga_i[n].x += double(ga.x);
    A.ga_i[n].y += double(ga.y);
    A.ga_i[n].z += double(ga.z);
  }
  A.tb[i] = pad3(scale(N, T(sp.h3)));
  A.sb[i] = sb;
  A.zb[i] = zb;
}

template <typename T>
__global__ void k_rev_Q(DevGraph<T> g, StateRef<T> X, StateRef<T> Y, AdjRef<T> A, SweepParams sp) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= g.n) return;
  const int o0 = g.o_ptr[i], o1 = g.o_ptr[i + 1];
  P4<T> sb = A.sb[i];
  Q4<T> qb = A.qb[i], pb = A.pb[i];
  for (int o = o0; o < o1; ++o) {
    const int n = A.out2in[o];
    add3(sb, v3(A.miT3[n]));
    add4(qb, A.miT4q[n]);
    add4(pb, A.miT4p[n]);
  }
  const T b = T(sp.beta), gb = T(sp.gamma * sp.beta);
  const Q4<T> lb = A.lb[i];
  const Q4<T> Qb = {qb.w + gb * lb.w, qb.x + gb * lb.x, qb.y + gb * lb.y, qb.z + gb * lb.z};
  const T D = g.cQ[i] + b + T(sp.h2);
  const T inv = T(1) / D;
  const Q4<T> N = {Qb.w * inv, Qb.x * inv, Qb.y * inv, Qb.z * inv};
  A.cqb[i] += -double(dot4(Qb, Y.q[i])) / double(D);
  pb.w += -gb * lb.w + b * N.w;
  pb.x += -gb * lb.x + b * N.x;
  pb.y += -gb * lb.y + b * N.y;
  pb.z += -gb * lb.z + b * N.z;
  const Q4<T> Cb = {T(2) * N.w, T(2) * N.x, T(2) * N.y, T(2) * N.z};
  const Q4<T> Yp = Y.p[i];
  const V3<T> si = v3(X.s[i]);
  for (int o = o0; o < o1; ++o) {
    const int j = g.o_nbr[o];
    const V3<T> a = v3(g.o_tt[o]);
    const Q4<T> w = g.o_w[o];
    const V3<T> tj = v3(X.t[j]);
    const V3<T> r = {tj.x - si.x, tj.y - si.y, tj.z - si.z};
    add4(pb, qmul_vp(qmul_pv(neg(r), Cb), a));
    const V3<T> rb = im_mul_conj(qmul_vp(Cb, a), Yp);
    A.moQ3[o] = pad3(rb);
    sb.x -= rb.x;
    sb.y -= rb.y;
    sb.z -= rb.z;
    const V3<T> ga = im(qmul(qmul_vp(qconj(Yp), r), Cb));
    A.ga_o[o].x += double(ga.x);
    A.ga_o[o].y += double(ga.y);
    A.ga_o[o].z += double(ga.z);
    A.moQ4[o] = qmul(Cb, w);
    const Q4<T> gw = qmul(qconj(Cb), Y.p[j]);
    A.gw_o[o].w += double(gw.w);
    A.gw_o[o].x += double(gw.x);
    A.gw_o[o].y += double(gw.y);
    A.gw_o[o].z += double(gw.z);
  }
  A.lb[i] = Q4<T>{lb.w - N.w, lb.x - N.x, lb.y - N.y, lb.z - N.z};
  A.qb[i] = Q4<T>{T(sp.h2) * N.w, T(sp.h2) * N.x, T(sp.h2) * N.y, T(sp.h2) * N.z};
  A.pb[i] = pb;
  A.sb[i] = sb;
}

template <typename T>
__global__ void k_rev_P(DevGraph<T> g, StateRef<T> X, StateRef<T> Y, AdjRef<T> A, SweepParams sp) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= g.n) return;
  const int o0 = g.o_ptr[i], o1 = g.o_ptr[i + 1];
  const int n0 = g.i_ptr[i], n1 = g.i_ptr[i + 1];
  Q4<T> pb = A.pb[i];
  P4<T> tb = A.tb[i];
  for (int n = n0; n < n1; ++n) {
    const int o = A.in2out[n];
    add4(pb, A.moQ4[o]);
    add3(tb, v3(A.moQ3[o]));
  }
  A.tb[i] = tb;
  // recompute v_i from x^k (same expression as the forward P phase)
  const Q4<T> qi = X.q[i], li = X.lam[i], pi = X.p[i];
  const V3<T> si = v3(X.s[i]);
  Q4<T> acc = {T(0), T(0), T(0), T(0)};
  for (int o = o0; o < o1; ++o) {
    const V3<T> tj = v3(X.t[g.o_nbr[o]]);
    const V3<T> mr = {si.x - tj.x, si.y - tj.y, si.z - tj.z};
    add4(acc, qmul_vp(qmul_pv(mr, qi), v3(g.o_tt[o])));
  }
  for (int n = n0; n < n1; ++n) add4(acc, qmul(X.q[g.i_nbr[n]], g.i_w[n]));
  const T b = T(sp.beta), h = T(sp.h1);
  const Q4<T> v = {T(2) * acc.w + b * qi.w + li.w + h * pi.w, T(2) * acc.x + b * qi.x + li.x + h * pi.x,
                   T(2) * acc.y + b * qi.y + li.y + h * pi.y, T(2) * acc.z + b * qi.z + li.z + h * pi.z};
  const T nv = sqrt(dot4(v, v));
  if (!(nv > T(0))) {  // p kept: p^{k+1} = p^k, the adjoint passes through
    A.pb[i] = pb;
    for (int o = o0; o < o1; ++o) A.moP[o] = P4<T>{T(0), T(0), T(0), T(0)};
    for (int n = n0; n < n1; ++n) A.miP[n] = Q4<T>{T(0), T(0), T(0), T(0)};
    return;
  }
  const Q4<T> pp = Y.p[i];
  const T c = dot4(pp, pb);
  const T inv = T(1) / nv;
  const Q4<T> vb = {(pb.w - pp.w * c) * inv, (pb.x - pp.x * c) * inv, (pb.y - pp.y * c) * inv,
                    (pb.z - pp.z * c) * inv};
  A.pb[i] = Q4<T>{h * vb.w, h * vb.x, h * vb.y, h * vb.z};
  Q4<T> qb = A.qb[i], lb = A.lb[i];
  qb.w += b * vb.w; qb.x += b * vb.x; qb.y += b * vb.y; qb.z += b * vb.z;
  add4(lb, vb);
  P4<T> sb = A.sb[i];
  const Q4<T> Ab = {T(2) * vb.w, T(2) * vb.x, T(2) * vb.y, T(2) * vb.z};
  for (int o = o0; o < o1; ++o) {
    const V3<T> a = v3(g.o_tt[o]);
    const V3<T> tj = v3(X.t[g.o_nbr[o]]);
    const V3<T> m = {si.x - tj.x, si.y - tj.y, si.z - tj.z};
    add4(qb, qmul_vp(qmul_pv(neg(m), Ab), neg(a)));
    const V3<T> mb = im_mul_conj(qmul_vp(Ab, neg(a)), qi);
    add3(sb, mb);
    A.moP[o] = pad3(neg(mb));
    const V3<T> ga = im(qmul(qmul_vp(qconj(qi), neg(m)), Ab));
    A.ga_o[o].x += double(ga.x);
    A.ga_o[o].y += double(ga.y);
    A.ga_o[o].z += double(ga.z);
  }
  for (int n = n0; n < n1; ++n) {
    const Q4<T> w = g.i_w[n];
    A.miP[n] = qmul(Ab, qconj(w));
    const Q4<T> gw = qmul(qconj(X.q[g.i_nbr[n]]), Ab);
    A.gw_i[n].w += double(gw.w);
    A.gw_i[n].x += double(gw.x);
    A.gw_i[n].y += double(gw.y);
    A.gw_i[n].z += double(gw.z);
  }
  A.qb[i] = qb;
  A.lb[i] = lb;
  A.sb[i] = sb;
}

// messages of the last P reverse phase (sweep 0) -> adjoint of x^0
template <typename T>
__global__ void k_rev_gather_P(DevGraph<T> g, AdjRef<T> A) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= g.n) return;
  P4<T> tb = A.tb[i];
  Q4<T> qb = A.qb[i];
  for (int n = g.i_ptr[i]; n < g.i_ptr[i + 1]; ++n) add3(tb, v3(A.moP[A.in2out[n]]));
  for (int o = g.o_ptr[i]; o < g.o_ptr[i + 1]; ++o) add4(qb, A.miP[A.out2in[o]]);
  A.tb[i] = tb;
  A.qb[i] = qb;
}

// dL/dx (n x 21 doubles) <-> adjoint arrays
template <typename T>
__global__ void k_adj_io(int n, AdjRef<T> A, double* buf, int to_device) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  double* b = buf + 21 * int64_t(i);
  if (to_device) {
    A.pb[i] = Q4<T>{T(b[0]), T(b[1]), T(b[2]), T(b[3])};
    A.qb[i] = Q4<T>{T(b[4]), T(b[5]), T(b[6]), T(b[7])};
    A.tb[i] = P4<T>{T(b[8]), T(b[9]), T(b[10]), T(0)};
    A.sb[i] = P4<T>{T(b[11]), T(b[12]), T(b[13]), T(0)};
    A.lb[i] = Q4<T>{T(b[14]), T(b[15]), T(b[16]), T(b[17])};
    A.zb[i] = P4<T>{T(b[18]), T(b[19]), T(b[20]), T(0)};
    A.cqb[i] = 0.0;
    A.ctb[i] = 0.0;
    A.csb[i] = 0.0;
  } else {
    const Q4<T> p = A.pb[i], q = A.qb[i], l = A.lb[i];
    const P4<T> t = A.tb[i], s = A.sb[i], z = A.zb[i];
    const double v[21] = {double(p.w), double(p.x), double(p.y), double(p.z), double(q.w),
                          double(q.x), double(q.y), double(q.z), double(t.x), double(t.y),
                          double(t.z), double(s.x), double(s.y), double(s.z), double(l.w),
                          double(l.x), double(l.y), double(l.z), double(z.x), double(z.y),
                          double(z.z)};
    for (int k = 0; k < 21; ++k) b[k] = v[k];
  }
}

template <typename T>
__global__ void k_adj_zero_edges(int64_t m, AdjRef<T> A) {
  const int64_t e = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (e >= m) return;
  A.ga_o[e] = P4<double>{0.0, 0.0, 0.0, 0.0};
  A.ga_i[e] = P4<double>{0.0, 0.0, 0.0, 0.0};
  A.gw_o[e] = Q4<double>{0.0, 0.0, 0.0, 0.0};
  A.gw_i[e] = Q4<double>{0.0, 0.0, 0.0, 0.0};
}

// derivative of E(w) = [cos(|w|/2), sin(|w|/2) w/|w|] transposed, applied to dE
__device__ V3<double> exp_vjp(const V3<double>& w, const Q4<double>& dE) {
  const double th2 = w.x * w.x + w.y * w.y + w.z * w.z;
  const double th = sqrt(th2);
  double s, ds_over_th;  // s = sin(th/2)/th, ds/dth / th
  if (th < 1e-4) {
    s = 0.5 - th2 / 48.0;
    ds_over_th = -1.0 / 24.0 + th2 / 960.0;
  } else {
    s = sin(0.5 * th) / th;
    ds_over_th = (0.5 * cos(0.5 * th) * th - sin(0.5 * th)) / (th2 * th);
  }
  const double wv = w.x * dE.x + w.y * dE.y + w.z * dE.z;
  const double c0 = -0.5 * s * dE.w;  // d cos(th/2)/dw = -(s/2) w
  return {c0 * w.x + s * dE.x + ds_over_th * wv * w.x, c0 * w.y + s * dE.y + ds_over_th * wv * w.y,
          c0 * w.z + s * dE.z + ds_over_th * wv * w.z};
}

__device__ Q4<double> exp_quat(const V3<double>& w) {
  const double th = sqrt(w.x * w.x + w.y * w.y + w.z * w.z);
  const double s = th < 1e-8 ? 0.5 - th * th / 48.0 : sin(0.5 * th) / th;
  return {cos(0.5 * th), s * w.x, s * w.y, s * w.z};
}

template <typename T>
__global__ void k_adj_params(int64_t m, AdjRef<T> A, const int32_t* __restrict__ pos_out,
                             const int32_t* __restrict__ pos_in, const int32_t* __restrict__ ei,
                             const int32_t* __restrict__ ej, const double* __restrict__ tm,
                             const double* __restrict__ kappa, const double* __restrict__ tau,
                             const Q4<double>* __restrict__ qe0, const double* __restrict__ omega,
                             double* g_kappa, double* g_tau, double* g_tm, double* g_omega) {
  const int64_t e = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (e >= m) return;
  const int o = pos_out[e], n = pos_in[e];
  const int i = ei[e], j = ej[e];
  const P4<double> go = A.ga_o[o], gi = A.ga_i[n];
  const V3<double> ab = {go.x + gi.x, go.y + gi.y, go.z + gi.z};
  const Q4<double> wo = A.gw_o[o], wi = A.gw_i[n];
  const Q4<double> wb = {wo.w + wi.w, wo.x + wi.x, wo.y + wi.y, wo.z + wi.z};
  const V3<double> tt = {tm[3 * e], tm[3 * e + 1], tm[3 * e + 2]};
  const double ta = tau[e], ka = kappa[e];
  const double cq = A.cqb[i], cs = A.csb[i], ct = A.ctb[j];
  const double tt2 = tt.x * tt.x + tt.y * tt.y + tt.z * tt.z;
  const V3<double> w = {omega[3 * e], omega[3 * e + 1], omega[3 * e + 2]};
  const Q4<double> E = exp_quat(w);
  const Q4<double> q = qmul(qe0[e], E);
  if (g_tau)
    g_tau[e] = go.u + gi.u + (ab.x * tt.x + ab.y * tt.y + ab.z * tt.z) + 2.0 * tt2 * cq + 2.0 * cs +
               2.0 * ct;
  if (g_tm) {
    g_tm[3 * e] = ta * ab.x + 4.0 * ta * tt.x * cq;
    g_tm[3 * e + 1] = ta * ab.y + 4.0 * ta * tt.y * cq;
    g_tm[3 * e + 2] = ta * ab.z + 4.0 * ta * tt.z * cq;
  }
  if (g_kappa) g_kappa[e] = (wb.w * q.w + wb.x * q.x + wb.y * q.y + wb.z * q.z) + 2.0 * cq;
  if (g_omega) {
    const Q4<double> qb = {ka * wb.w, ka * wb.x, ka * wb.y, ka * wb.z};
    const Q4<double> Eb = qmul(qconj(qe0[e]), qb);  // q = q0 E  ->  dE = q0^* dq
    const V3<double> gw = exp_vjp(w, Eb);
    g_omega[3 * e] = gw.x;
    g_omega[3 * e + 1] = gw.y;
    g_omega[3 * e + 2] = gw.z;
  }
}

// q~ = q~0 E(omega) (right perturbation of the measured rotation)
__global__ void k_perturb(int64_t m, const Q4<double>* __restrict__ qe0,
                          const double* __restrict__ omega, Q4<double>* __restrict__ qe) {
  const int64_t e = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (e >= m) return;
  const V3<double> w = {omega[3 * e], omega[3 * e + 1], omega[3 * e + 2]};
  qe[e] = qmul(qe0[e], exp_quat(w));
}

__global__ void k_maps(int64_t m, const int32_t* __restrict__ o_perm,
                       const int32_t* __restrict__ i_perm, int32_t* pos_out, int32_t* pos_in) {
  const int64_t k = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (k >= m) return;
  pos_out[o_perm[k]] = int32_t(k);
  pos_in[i_perm[k]] = int32_t(k);
}

__global__ void k_maps2(int64_t m, const int32_t* __restrict__ o_perm,
                        const int32_t* __restrict__ i_perm, const int32_t* __restrict__ pos_out,
                        const int32_t* __restrict__ pos_in, int32_t* in2out, int32_t* out2in) {
  const int64_t k = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (k >= m) return;
  in2out[k] = pos_out[i_perm[k]];
  out2in[k] = pos_in[o_perm[k]];
}

inline dim3 grid1(int64_t count, int block) { return dim3(unsigned((count + block - 1) / block)); }

}  // namespace

// ---------------------------------------------------------------------------
// launchers
// ---------------------------------------------------------------------------
template <typename T>
hipError_t launch_reverse_sweep(const DevGraph<T>& g, const StateRef<T>& X, const StateRef<T>& Y,
                                const AdjRef<T>& A, const SweepParams& sp, int first,
                                hipStream_t st) {
  if (g.n <= 0) return hipSuccess;
  const dim3 grid = grid1(g.n, 256), blk(256);
  hipLaunchKernelGGL((k_rev_S<T>), grid, blk, 0, st, g, X, Y, A, sp, first);
  hipLaunchKernelGGL((k_rev_T<T>), grid, blk, 0, st, g, X, Y, A, sp);
  hipLaunchKernelGGL((k_rev_Q<T>), grid, blk, 0, st, g, X, Y, A, sp);
  hipLaunchKernelGGL((k_rev_P<T>), grid, blk, 0, st, g, X, Y, A, sp);
  return hipGetLastError();
}

template <typename T>
hipError_t launch_reverse_finish(const DevGraph<T>& g, const AdjRef<T>& A, hipStream_t st) {
  if (g.n <= 0) return hipSuccess;
  hipLaunchKernelGGL((k_rev_gather_P<T>), grid1(g.n, 256), dim3(256), 0, st, g, A);
  return hipGetLastError();
}

template <typename T>
hipError_t launch_adj_io(int n, const AdjRef<T>& A, double* buf, int to_device, hipStream_t st) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL((k_adj_io<T>), grid1(n, 256), dim3(256), 0, st, n, A, buf, to_device);
  return hipGetLastError();
}

template <typename T>
hipError_t launch_adj_zero_edges(int64_t m, const AdjRef<T>& A, hipStream_t st) {
  if (m <= 0) return hipSuccess;
  hipLaunchKernelGGL((k_adj_zero_edges<T>), grid1(m, 256), dim3(256), 0, st, m, A);
  return hipGetLastError();
}

template <typename T>
hipError_t launch_adj_params(int64_t m, const AdjRef<T>& A, const int32_t* pos_out,
                             const int32_t* pos_in, const int32_t* ei, const int32_t* ej,
                             const double* tm, const double* kappa, const double* tau,
                             const Q4<double>* qe0, const double* omega, double* g_kappa,
                             double* g_tau, double* g_tm, double* g_omega, hipStream_t st) {
  if (m <= 0) return hipSuccess;
  hipLaunchKernelGGL((k_adj_params<T>), grid1(m, 256), dim3(256), 0, st, m, A, pos_out, pos_in, ei,
                     ej, tm, kappa, tau, qe0, omega, g_kappa, g_tau, g_tm, g_omega);
  return hipGetLastError();
}

hipError_t launch_perturb(int64_t m, const Q4<double>* qe0, const double* omega, Q4<double>* qe,
                          hipStream_t st) {
  if (m <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_perturb, grid1(m, 256), dim3(256), 0, st, m, qe0, omega, qe);
  return hipGetLastError();
}

hipError_t launch_edge_maps(int64_t m, const int32_t* o_perm, const int32_t* i_perm,
                            int32_t* pos_out, int32_t* pos_in, int32_t* in2out, int32_t* out2in,
                            hipStream_t st) {
  if (m <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_maps, grid1(m, 256), dim3(256), 0, st, m, o_perm, i_perm, pos_out, pos_in);
  hipLaunchKernelGGL(k_maps2, grid1(m, 256), dim3(256), 0, st, m, o_perm, i_perm, pos_out, pos_in,
                     in2out, out2in);
  return hipGetLastError();
}

#define PGO_ADJ_INST(T)                                                                          \
  template hipError_t launch_reverse_sweep<T>(const DevGraph<T>&, const StateRef<T>&,             \
                                              const StateRef<T>&, const AdjRef<T>&,               \
                                              const SweepParams&, int, hipStream_t);              \
  template hipError_t launch_reverse_finish<T>(const DevGraph<T>&, const AdjRef<T>&, hipStream_t); \
  template hipError_t launch_adj_io<T>(int, const AdjRef<T>&, double*, int, hipStream_t);         \
  template hipError_t launch_adj_zero_edges<T>(int64_t, const AdjRef<T>&, hipStream_t);          \
  template hipError_t launch_adj_params<T>(int64_t, const AdjRef<T>&, const int32_t*,            \
                                           const int32_t*, const int32_t*, const int32_t*,       \
                                           const double*, const double*, const double*,          \
                                           const Q4<double>*, const double*, double*, double*,   \
                                           double*, double*, hipStream_t);
PGO_ADJ_INST(float)
PGO_ADJ_INST(double)
#undef PGO_ADJ_INST

}  // namespace pgo
