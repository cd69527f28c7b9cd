// Internal interfaces between the host side of the library (handle.hpp and
// the .cpp files) and the kernel translation units.  Nothing here is part of
// the C ABI.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "qmath.hpp"

namespace pgo {

// Device view of one handle's graph and state for precision T.
//
// Edges are stored twice, structure-of-arrays, in the order "by tail" (out,
// CSR) and "by head" (in, CSC); inside one vertex the edges keep the
// caller's edge order.  Each edge record is
//   nbr  the other end (head for out-order, tail for in-order)
//   tt   (tau t~_e, tau_e)
//   w    kappa_e q~_e
// so the per-edge terms are linear in the stored quantities.
// Vertex constants (depend only on the edges):
//   cQ_i = 2 sum_out (tau_e |t~_e|^2 + kappa_e)   (A2 = (cQ + beta + H2) I)
//   cT_i = 2 sum_in  tau_e                        (A3 = (cT + beta + H3) I)
//   cS_i = 2 sum_out tau_e                        (A4 = (cS + beta + H4) I)
template <typename T>
struct DevGraph {
  int32_t n;
  const int32_t* gid;  // graph of each vertex (per-graph penalties)
  const int32_t* o_ptr;
  const int32_t* o_nbr;
  const P4<T>* o_tt;
  const Q4<T>* o_w;
  const int32_t* i_ptr;
  const int32_t* i_nbr;
  const P4<T>* i_tt;
  const Q4<T>* i_w;
  const T* cQ;
  const T* cT;
  const T* cS;
  Q4<T>* p;
  Q4<T>* q;
  Q4<T>* lam;
  V3<T>* t;
  V3<T>* s;
  V3<T>* z;
  // per-vertex slot between phases of the sweep (scratch): P's in-edge sum
  // from T to S+P, then the tau part of Q's out-edge sum from S+P to Q, and
  // the magnitude of the in-edge terms (FP32 cancellation check)
  Q4<T>* xy;
  T* xm;
  // values before the last sweep of an iterate call (residual history)
  Q4<T>* q_prev;
  Q4<T>* lam_prev;
  V3<T>* t_prev;
  V3<T>* s_prev;
  V3<T>* z_prev;
};

// Where the state of the vertices being updated lives during a sweep: each
// array either in global memory (base 0) or, in a per-graph kernel, in LDS
// for the graph's vertices v0.. (base v0); element j of an array is
// x[j - xb].
template <typename T>
struct State {
  Q4<T>* p_;
  Q4<T>* q_;
  V3<T>* t_;
  V3<T>* s_;
  Q4<T>* lam_;
  V3<T>* z_;
  int pb, qb, tb, sb, lb, zb;
  __device__ __forceinline__ Q4<T>& p(int j) const { return p_[j - pb]; }
  __device__ __forceinline__ Q4<T>& q(int j) const { return q_[j - qb]; }
  __device__ __forceinline__ V3<T>& t(int j) const { return t_[j - tb]; }
  __device__ __forceinline__ V3<T>& s(int j) const { return s_[j - sb]; }
  __device__ __forceinline__ Q4<T>& lam(int j) const { return lam_[j - lb]; }
  __device__ __forceinline__ V3<T>& z(int j) const { return z_[j - zb]; }
};

template <typename T>
__device__ __forceinline__ State<T> global_state(const DevGraph<T>& g) {
  return {g.p, g.q, g.t, g.s, g.lam, g.z, 0, 0, 0, 0, 0, 0};
}

// LDS bytes of the first k of p, q, t, s, lambda, z for n vertices, each
// array starting on a 16-byte boundary.
template <typename T>
__host__ __device__ __forceinline__ size_t state_lds_bytes(int k, size_t n) {
  const size_t q = (sizeof(Q4<T>) * n + 15) & ~size_t(15), v = (sizeof(V3<T>) * n + 15) & ~size_t(15);
  const size_t c[7] = {0, q, 2 * q, 2 * q + v, 2 * q + 2 * v, 3 * q + 2 * v, 3 * q + 3 * v};
  return c[k];
}

// Places the first k of p, q, t, s, lambda, z of the graph's vertices
// [v0, v1) in LDS (laid out as state_lds_bytes counts them), loads them,
// and returns the view; the caller runs its sweeps and hands the view to
// state_store.  Every vertex's slots are written only by the thread that
// owns the vertex, which also loads and stores them.
template <int kSlots, typename T>
__device__ __forceinline__ State<T> state_load(const DevGraph<T>& g, int v0, int v1,
                                               unsigned char* lds) {
  const size_t n = size_t(v1 - v0);
  State<T> st = global_state(g);
  const size_t qb = state_lds_bytes<T>(1, n), vb = state_lds_bytes<T>(3, n) - 2 * qb;
  unsigned char* at = lds;
  if (kSlots >= 1) st.p_ = reinterpret_cast<Q4<T>*>(at), st.pb = v0, at += qb;
  if (kSlots >= 2) st.q_ = reinterpret_cast<Q4<T>*>(at), st.qb = v0, at += qb;
  if (kSlots >= 3) st.t_ = reinterpret_cast<V3<T>*>(at), st.tb = v0, at += vb;
  if (kSlots >= 4) st.s_ = reinterpret_cast<V3<T>*>(at), st.sb = v0, at += vb;
  if (kSlots >= 5) st.lam_ = reinterpret_cast<Q4<T>*>(at), st.lb = v0, at += qb;
  if (kSlots >= 6) st.z_ = reinterpret_cast<V3<T>*>(at), st.zb = v0;
  if (kSlots >= 1) {
    for (int i = v0 + int(threadIdx.x); i < v1; i += int(blockDim.x)) {
      st.p(i) = g.p[i];
      if (kSlots >= 2) st.q(i) = g.q[i];
      if (kSlots >= 3) st.t(i) = g.t[i];
      if (kSlots >= 4) st.s(i) = g.s[i];
      if (kSlots >= 5) st.lam(i) = g.lam[i];
      if (kSlots >= 6) st.z(i) = g.z[i];
    }
    __syncthreads();
  }
  return st;
}

template <int kSlots, typename T>
__device__ __forceinline__ void state_store(const DevGraph<T>& g, const State<T>& st, int v0,
                                            int v1) {
  if (kSlots >= 1) {
    for (int i = v0 + int(threadIdx.x); i < v1; i += int(blockDim.x)) {
      g.p[i] = st.p(i);
      if (kSlots >= 2) g.q[i] = st.q(i);
      if (kSlots >= 3) g.t[i] = st.t(i);
      if (kSlots >= 4) g.s[i] = st.s(i);
      if (kSlots >= 5) g.lam[i] = st.lam(i);
      if (kSlots >= 6) g.z[i] = st.z(i);
    }
  }
}

struct SweepParams {
  double beta, gamma, h1, h2, h3, h4;
  const double* beta_g;   // per-graph penalties (device, G values) or nullptr
  const int32_t* active;  // per-graph run flags (device, G values) or nullptr = all run
  // stopping inside the per-graph kernel (launch_graph_sweeps_stop): every
  // check_every sweeps a graph stops once its residual e is below tol and
  // writes the sweeps it ran to done[graph]
  double tol = 0.0;
  int check_every = 0;
  int32_t* done = nullptr;
  // per-graph kernel (quaternion model): when non-null, each graph's state
  // p, q, lambda, t, s, z is copied to these arrays (same layout) before
  // its first sweep, so that the call can be undone per graph
  void* snap[6] = {nullptr, nullptr, nullptr, nullptr, nullptr, nullptr};
};

// Device view for the rotation-matrix (chordal) model: the same edge order
// and SoA layout, with 3x3 blocks in place of quaternions.  Edge record
//   nbr, tt = (tau t~_e, tau_e), R = kappa_e R~_e
// and the vertex constant cQ_i = 2 sum_out kappa (T and S sum their tau
// from the records they stream).
template <typename T>
struct DevChordal {
  int32_t n;
  const int32_t* gid;
  const int32_t* o_ptr;
  const int32_t* o_nbr;
  const P4<T>* o_tt;
  const R3<T>* o_R;
  const int32_t* i_ptr;
  const int32_t* i_nbr;
  const P4<T>* i_tt;
  const R3<T>* i_R;
  const T* cQ;
  R3<T>* P;
  R3<T>* Q;
  R3<T>* L;
  V3<T>* t;
  V3<T>* s;
  V3<T>* z;
  R3<T>* Q_prev;
  R3<T>* L_prev;
  V3<T>* t_prev;
  V3<T>* s_prev;
  V3<T>* z_prev;
};

// Launchers (sweep.hip).  Every launcher checks its own configuration and
// returns the HIP status of the launch.
template <typename T>
hipError_t launch_phase_sweeps(const DevGraph<T>& g, int k, const SweepParams& sp, int block,
                               hipStream_t st);
// lds != 0 lets every graph keep the part of its state that fits in LDS
// there for the whole launch (p, q; then t, s; then lambda, z, by graph
// size; at most 160 KiB per workgroup); lds == 0 keeps it all in memory.
template <typename T>
hipError_t launch_graph_sweeps(const DevGraph<T>& g, const int32_t* voff, const int32_t* order,
                               int G, int k, const SweepParams& sp, int block, int max_n, int lds,
                               hipStream_t st);
// The per-graph kernel running up to k sweeps (k a multiple of
// sp.check_every) with the stopping rule of App. E.1 evaluated in the
// kernel: after every check_every sweeps a graph computes its residual
// e = (|dlambda|^2 + |dz|^2)/beta + beta (|dq|^2 + |dt|^2) over the last
// sweep (FP64 sums of the stored values) and stops when e < sp.tol;
// sp.done[graph] receives the sweeps run.  Each check sweep ends with a
// plain S and records the residual history, so the state equals that of
// chunks of check_every sweeps run by separate calls.  block <= 1024.
template <typename T>
hipError_t launch_graph_sweeps_stop(const DevGraph<T>& g, const int32_t* voff,
                                    const int32_t* order, int G, int k, const SweepParams& sp,
                                    int block, int max_n, int lds, hipStream_t st);

// The per-phase schedule in one persistent cooperative launch (sweep_coop.hip):
// the same phases over all vertices, a device-wide barrier on bar[0] between
// phases (bar: 2 words of device memory owned by the handle; bar[1] is set
// to 1 by a launch whose barrier wait timed out).  Bitwise the state of
// launch_phase_sweeps.  coop_max_blocks: workgroups of a launch at `block`
// threads (co-resident, at most one per compute unit).
template <typename T>
hipError_t launch_coop_sweeps(const DevGraph<T>& g, int k, const SweepParams& sp, int block,
                              unsigned* bar, hipStream_t st);
template <typename T>
int coop_max_blocks(int block);

// Boundary preparation and state transfer (prep.hip), FP64.
// Device-to-device copy as a kernel (4-byte aligned, size a multiple of 4).
hipError_t launch_copy(void* dst, const void* src, size_t bytes, hipStream_t st);
// Projection onto SO(3) and conversion to a unit quaternion; bad[i] = 1
// where rotation i fails det > 0 or ||R^T R - I||_F <= 1e-2.
hipError_t launch_rot_to_quat(const double* R, int64_t count, Q4<double>* out, int canonical,
                              uint8_t* bad, hipStream_t st);
hipError_t launch_align(const Q4<double>* pv, Q4<double>* qe, const int32_t* ei,
                        const int32_t* ej, int64_t m, hipStream_t st);
// Stable sort of edge ids by key (tail or head).  Call once with tmp = nullptr
// to get the temporary size, then with a buffer of that size.
hipError_t sort_by_key(const int32_t* keys, int32_t* perm, int64_t m, int32_t n, int32_t* iota,
                       void* tmp, size_t* tmp_bytes, int32_t* keys_sorted, hipStream_t st);
hipError_t launch_ptr_from_sorted(const int32_t* keys_sorted, int64_t m, int32_t n, int32_t* ptr,
                                  hipStream_t st);
// The FP64 edges again in the order perm gives (row k = caller edge
// perm[k]): ei, ej, tm, kappa, tau always; q and X9 (9 doubles per edge)
// when given (non-null), else their outputs are left alone.
hipError_t launch_gather_edges_f64(const int32_t* perm, int64_t m, const int32_t* ei,
                                   const int32_t* ej, const Q4<double>* q, const double* tm,
                                   const double* kappa, const double* tau, const double* X9,
                                   int32_t* oi, int32_t* oj, Q4<double>* oq, double* otm,
                                   double* okappa, double* otau, double* oX9, hipStream_t st);
template <typename T>
hipError_t launch_fill_edges(const int32_t* perm, const int32_t* nbr_src, const Q4<double>* qe,
                             const double* tm, const double* kappa, const double* tau, int64_t m,
                             int32_t* nbr, P4<T>* tt, Q4<T>* w, hipStream_t st);
template <typename T>
hipError_t launch_vertex_consts(int32_t n, const int32_t* o_ptr, const int32_t* o_perm,
                                const int32_t* i_ptr, const int32_t* i_perm, const double* tm,
                                const double* kappa, const double* tau, T* cQ, T* cT, T* cS,
                                hipStream_t st);
template <typename T>
hipError_t launch_init_state(const DevGraph<T>& g, const Q4<double>* p0, const double* t0,
                             hipStream_t st);
template <typename T>
hipError_t launch_state_io(const DevGraph<T>& g, double* buf, int to_device, hipStream_t st);
template <typename T>
hipError_t launch_poses(const DevGraph<T>& g, double* R, double* t, hipStream_t st);

// Quaternion model with a full 3x3 translation information per edge
// (aniso.hip): the isotropic view plus the edge information matrices (two
// P4 per edge: xx xy xz yy | yz zz) in both orders, the edge record tt
// holding (t~, c_e) instead of (tau t~, tau).  The T and S updates form
// their matrices 2 sum_in S and 2 sum_out S from the records they stream.
template <typename T>
struct DevAniso {
  DevGraph<T> g;
  const V3<T>* o_Sa;
  const V3<T>* o_Sb;
  const V3<T>* i_Sa;
  const V3<T>* i_Sb;
};
template <typename T>
hipError_t launch_phase_sweeps_a(const DevAniso<T>& a, int k, const SweepParams& sp, int block,
                                 hipStream_t st);
template <typename T>
// lds != 0: each graph keeps the part of its state that fits in LDS there
// for the whole launch (as launch_graph_sweeps); block <= 512.
hipError_t launch_graph_sweeps_a(const DevAniso<T>& a, const int32_t* voff, const int32_t* order,
                                 int G, int k, const SweepParams& sp, int block, int max_n, int lds,
                                 hipStream_t st);
template <typename T>
hipError_t launch_fill_edges_a(const int32_t* perm, const double* tm, const double* S9, int64_t m,
                               P4<T>* tt, V3<T>* Sa, V3<T>* Sb, hipStream_t st);

// Chordal model (chordal.hip): sweeps, preparation and state transfer.
template <typename T>
hipError_t launch_phase_sweeps_c(const DevChordal<T>& g, int k, const SweepParams& sp, int block,
                                 hipStream_t st);
template <typename T>
// lds != 0: each graph keeps the part of its state that fits in LDS there
// for the whole launch (s, P, t, Q, z, Lambda in that order, by graph size).
hipError_t launch_graph_sweeps_c(const DevChordal<T>& g, const int32_t* voff, const int32_t* order,
                                 int G, int k, const SweepParams& sp, int block, int max_n, int lds,
                                 hipStream_t st);
// projection of 3x3 matrices onto SO(3) with the validity rule of
// launch_rot_to_quat (det > 0 and ||A^T A - I||_F <= 1e-2, else bad[i] = 1)
hipError_t launch_project_rot(const double* R, int64_t count, double* out, uint8_t* bad,
                              hipStream_t st);
template <typename T>
hipError_t launch_fill_edges_c(const int32_t* perm, const int32_t* nbr_src, const double* R9,
                               const double* tm, const double* kappa, const double* tau, int64_t m,
                               int32_t* nbr, P4<T>* tt, R3<T>* Rw, hipStream_t st);
template <typename T>
hipError_t launch_vertex_consts_c(int32_t n, const int32_t* o_ptr, const int32_t* o_perm,
                                  const double* kappa, T* cQ, hipStream_t st);
template <typename T>
hipError_t launch_init_state_c(const DevChordal<T>& g, const double* P0, const double* t0,
                               hipStream_t st);
// n x 36 doubles per vertex: P (9) Q (9) t (3) s (3) Lambda (9) z (3)
template <typename T>
hipError_t launch_state_io_c(const DevChordal<T>& g, double* buf, int to_device, hipStream_t st);
template <typename T>
hipError_t launch_poses_c(const DevChordal<T>& g, double* R, double* t, hipStream_t st);

// Restores the six state arrays of every vertex whose graph is flagged;
// words[k] = 4-byte words per vertex of array k (at most 32).
hipError_t launch_restore_words(int32_t n, const int32_t* gid, const int32_t* flag,
                                void* const* dst, const void* const* src, const int* words,
                                hipStream_t st);

// Chordal initialisation (cinit.hip): FP64 preconditioned conjugate
// gradients per graph on the relaxed rotation and the translation normal
// equations.  Edge arrays in caller order, reached through the CSR/CSC
// permutations.
struct CinitGraph {
  const int32_t* o_ptr;
  const int32_t* o_nbr;
  const int32_t* o_perm;
  const int32_t* i_ptr;
  const int32_t* i_nbr;
  const int32_t* i_perm;
  const double* wt;       // kappa (rotations) or tau (translations), caller order
  const double* R9;       // measured rotations, m x 9 row-major, caller order
  const double* tm;       // m x 3, caller order
  double* diag;           // n: sum of the weights at each vertex
  const uint8_t* anchor;  // n: 1 = held at its given value
  // the operator's edge data in out- and in-order (so a vertex reads its
  // edges contiguously): weight x R~ (m x 9) for the rotation solve, the
  // weight alone for the translation solve
  double* o_wR;
  double* i_wR;
  double* o_w;
  double* i_w;
};
struct CinitVec {  // W doubles per vertex each
  double* x;
  double* r;
  double* z;
  double* p;
  double* ap;
};
struct CinitChunks {  // vertex chunks, never straddling graphs
  const int64_t* beg;
  const int64_t* end;
  const int32_t* cgraph;  // graph of each chunk
  const int32_t* g_off;   // chunks of graph g: [g_off[g], g_off[g+1])
  int n_chunks;
  double* part;           // one partial per chunk
};
struct CinitScalars {  // one per graph
  double* rz0;
  double* rz;
  double* alpha;
  double* beta;
  int32_t* active;
  int32_t* iters;
};
hipError_t launch_cinit_diag(const CinitGraph& c, int32_t n, hipStream_t st);
// fills o_wR, i_wR (W = 9) or o_w, i_w (W = 3) from wt, R9 and the permutations
hipError_t launch_cinit_edges(const CinitGraph& c, int64_t m, int W, hipStream_t st);
hipError_t launch_cinit_rhs_t(const CinitGraph& c, int32_t n, const double* R, double* rhs,
                              hipStream_t st);
hipError_t launch_cinit_project(int32_t n, const uint8_t* anchor, const double* X,
                                const double* given, double* R, hipStream_t st);
hipError_t launch_cinit_qmat(int64_t m, const Q4<double>* q, double* R, hipStream_t st);
// Solves A x = b (b null: 0) for every graph, from the x given, W = 9 or 3;
// stops a graph when <r, z> <= tol^2 <r0, z0> or after max_iters; checks
// for global completion on the host every check_every iterations.
hipError_t launch_cinit_cg(const CinitGraph& c, const CinitVec& v, const CinitChunks& ch, int W,
                           const double* b, int max_iters, int check_every, double tol,
                           const CinitScalars& s, int G, int32_t* host_active, hipStream_t st);

// FP64 reductions (reduce.hip).  Items are split into chunks that never cross
// a graph boundary; chunk c covers [cbeg[c], cend[c]) of graph cgraph[c].
// Partial sums of a chunk are reduced in a fixed order, then each graph sums
// its chunks in order, so results are deterministic.
struct EdgeF64 {  // FP64 prepared edges for the cost, in any order within each graph
  const int32_t* ei;
  const int32_t* ej;
  const Q4<double>* q;
  const double* tm;
  const double* kappa;
  const double* tau;
  const double* R9;  // chordal model: projected measured rotations (m x 9), else unused
  const double* S9;  // information model: translation information per edge (m x 9), else null
};
// Per-graph reduction output, kRedVals doubles per graph:
enum RedIdx {
  kCost = 0,   // model (1) at (p, t)
  kSplit,      // f + g of eq. 2
  kPQ2,        // |p - q|^2
  kTS2,        // |t - s|^2
  kDL2,        // |lambda - lambda_prev|^2
  kDZ2,        // |z - z_prev|^2
  kDQ2,        // |q - q_prev|^2
  kDT2,        // |t - t_prev|^2
  kDS2,        // |s - s_prev|^2
  kLamPQ,      // <lambda, p - q>
  kZTS,        // <z, t - s>
  kRedVals
};
constexpr int kEdgeVals = 2;  // kCost, kSplit
constexpr int kVertVals = 9;  // kPQ2 .. kZTS
// ec_graph / vc_graph: graph of each edge / vertex chunk; with active given,
// chunks of graphs whose flag is 0 skip their work and report zeros.
template <typename T>
hipError_t launch_reduce(const DevGraph<T>& g, const EdgeF64& e, int have_prev,
                         const int32_t* ec_graph, const int64_t* ec_beg, const int64_t* ec_end,
                         int n_echunks, const int32_t* vc_graph, const int64_t* vc_beg,
                         const int64_t* vc_end, int n_vchunks, double* partial_e,
                         double* partial_v, const int32_t* g_ec_off, const int32_t* g_vc_off,
                         int G, double* out, const int32_t* active, hipStream_t st);

// The same reductions with partials and per-graph values in the library's
// static device array (pgo_evaluate_noalloc): kScratchDoubles doubles per
// device; scratch_address gives this device's array (looked up once per
// device).  A call needs 2 n_echunks + 9 n_vchunks + 11 G doubles of it.
// out receives kEvalVals doubles per graph: F, |p - q|, |t - s|, e,
// beta |dq|, beta |ds|, L_beta, Psi; beta is per graph, on the device.
constexpr size_t kScratchDoubles = size_t(1) << 18;  // 2 MiB
constexpr int kEvalVals = 8;
hipError_t scratch_address(int device, double** ptr);
template <typename T>
hipError_t launch_evaluate_noalloc(const DevGraph<T>& g, const EdgeF64& e, int have_prev,
                                   const int32_t* ec_graph, const int64_t* ec_beg,
                                   const int64_t* ec_end, int n_echunks, const int32_t* vc_graph,
                                   const int64_t* vc_beg, const int64_t* vc_end, int n_vchunks,
                                   const int32_t* g_ec_off, const int32_t* g_vc_off, int G,
                                   double* scr, const double* beta, double gamma, double* out,
                                   hipStream_t st);

template <typename T>
hipError_t launch_reduce_c(const DevChordal<T>& g, const EdgeF64& e, int have_prev,
                           const int32_t* ec_graph, const int64_t* ec_beg, const int64_t* ec_end,
                           int n_echunks, const int32_t* vc_graph, const int64_t* vc_beg,
                           const int64_t* vc_end, int n_vchunks, double* partial_e,
                           double* partial_v, const int32_t* g_ec_off, const int32_t* g_vc_off,
                           int G, double* out, const int32_t* active, hipStream_t st);

// ---------------------------------------------------------------------------
// Reverse mode (adjoint.hip)
// ---------------------------------------------------------------------------
template <typename T>
struct StateRef {
  const Q4<T>* p;
  const Q4<T>* q;
  const Q4<T>* lam;
  const V3<T>* t;
  const V3<T>* s;
  const V3<T>* z;
};

template <typename T>
struct AdjRef {
  Q4<T>* pb;
  Q4<T>* qb;
  Q4<T>* lb;
  P4<T>* tb;
  P4<T>* sb;
  P4<T>* zb;
  P4<T>* moS;     // S -> t of the head          (per out-position)
  P4<T>* miT3;    // T -> s of the tail          (per in-position)
  Q4<T>* miT4q;   // T -> q of the tail
  Q4<T>* miT4p;   // T -> p of the tail
  Q4<T>* moQ4;    // Q -> p of the head          (per out-position)
  P4<T>* moQ3;    // Q -> t of the head
  P4<T>* moP;     // P -> t of the head          (per out-position)
  Q4<T>* miP;     // P -> q of the tail          (per in-position)
  P4<double>* ga_o;  // d/d(tau t~) (xyz) and d/dtau (u), out-order
  Q4<double>* gw_o;  // d/d(kappa q~), out-order
  P4<double>* ga_i;  // in-order
  Q4<double>* gw_i;
  double* cqb;
  double* ctb;
  double* csb;
  const int32_t* in2out;
  const int32_t* out2in;
};

template <typename T>
hipError_t launch_reverse_sweep(const DevGraph<T>& g, const StateRef<T>& X, const StateRef<T>& Y,
                                const AdjRef<T>& A, const SweepParams& sp, int first,
                                hipStream_t st);
template <typename T>
hipError_t launch_reverse_finish(const DevGraph<T>& g, const AdjRef<T>& A, hipStream_t st);
template <typename T>
hipError_t launch_adj_io(int n, const AdjRef<T>& A, double* buf, int to_device, hipStream_t st);
template <typename T>
hipError_t launch_adj_zero_edges(int64_t m, const AdjRef<T>& A, hipStream_t st);
template <typename T>
hipError_t launch_adj_params(int64_t m, const AdjRef<T>& A, const int32_t* pos_out,
                             const int32_t* pos_in, const int32_t* ei, const int32_t* ej,
                             const double* tm, const double* kappa, const double* tau,
                             const Q4<double>* qe0, const double* omega, double* g_kappa,
                             double* g_tau, double* g_tm, double* g_omega, hipStream_t st);
hipError_t launch_perturb(int64_t m, const Q4<double>* qe0, const double* omega, Q4<double>* qe,
                          hipStream_t st);
hipError_t launch_edge_maps(int64_t m, const int32_t* o_perm, const int32_t* i_perm,
                            int32_t* pos_out, int32_t* pos_in, int32_t* in2out, int32_t* out2in,
                            hipStream_t st);

}  // namespace pgo
