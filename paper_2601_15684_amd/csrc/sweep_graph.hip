// The PRADMM sweep, one persistent workgroup per graph (the vertex updates
// are in sweep_core.hpp): all k sweeps of a call in one launch; the phase
// barrier is the workgroup barrier, so no grid-wide synchronisation exists.
// order[] lists graphs largest first (the hardware hands out workgroups in
// index order, which makes this a longest-first greedy schedule).
//
// A graph is updated by one workgroup only, so its state can stay on chip
// for all k sweeps (loaded once, written back once):
//   * thread t owns vertices v0 + t + r * blockDim (r < kVpt) for the whole
//     launch and keeps their owner-only values -- lambda, z, the slot
//     between phases and the constant cQ -- in registers (kVpt = 0: more vertices per thread
//     than registers hold; those values then stay in global memory);
//   * the first kSlots of p, q, t, s (read by the owner and gathered by the
//     neighbours) that fit the launch's LDS are kept there, every read of
//     them, the neighbour gathers included, served on chip.
// The 4096-graph batch (FP32, 1024 threads) keeps all of p, q, t, s in LDS
// for graphs up to 2925 poses, p, q, t up to 3723, p, q up to 5120.
#pragma clang fp contract(off)
#include <algorithm>

#include "sweep_core.hpp"

namespace pgo {

namespace {

// A vertex index the compiler cannot see through: the addresses derived
// from it are formed again in every phase instead of being hoisted out of
// the sweep loop, where one 64-bit address per array and vertex would hold
// a register pair for the whole launch.
__device__ __forceinline__ int vertex_of(int i) {
  asm volatile("" : "+v"(i));
  return i;
}

template <typename T>
struct Own {  // one vertex's owner-only values
  Q4<T> lam;
  Q4<T> xy;  // Y_i from T to S+P, X_i from S+P (or the opening P) to Q
  V3<T> z;
  T xm;      // magnitude of Y_i's terms (FP32 check)
  T cq;      // cQ_i (constant: loaded once, never stored)
};

// edges in flight per thread in the T and S passes when the owner-only
// values are in registers: two in FP32 (measured on the 4096-graph batch:
// 1, 2, 3, 4 give 31.9, 30.7, 31.9, 36.0 ms per 50 sweeps; three and more
// take registers the owner-only values hold), one in FP64 (two: 96.6
// against 95.0 ms)
#ifndef PGO_UNROLL_REG
#define PGO_UNROLL_REG 2
#endif
template <typename T>
constexpr int kUnrollReg = sizeof(T) == 4 ? PGO_UNROLL_REG : 1;
#ifndef PGO_UNROLL_Q
#define PGO_UNROLL_Q 2
#endif
constexpr int kUnrollQ = PGO_UNROLL_Q;

// Places the first kSlots of p, q, t, s of the graph's vertices [v0, v1)
// in LDS (laid out as sw_lds_bytes counts them), loads them and returns the
// view.  Every vertex's slots are written only by the thread that owns the
// vertex, which also loads and stores them.
template <int kSlots, typename T>
__device__ __forceinline__ SwState<T> sw_load(const DevGraph<T>& g, int v0, int v1,
                                              unsigned char* lds) {
  const size_t n = size_t(v1 - v0);
  SwState<T> st = sw_global(g);
  unsigned char* at = lds;
  unsigned char* ptr[kArrays];
#pragma unroll
  for (int a = 0; a < kArrays; ++a) {
    ptr[a] = at;
    if (a < kSlots) {
      st.b[a] = v0;
      at += (sw_elem_bytes<T>(a) * n + 15) & ~size_t(15);
    }
  }
  if (kSlots >= 1) st.p_ = reinterpret_cast<Q4<T>*>(ptr[0]);
  if (kSlots >= 2) st.q_ = reinterpret_cast<Q4<T>*>(ptr[1]);
  if (kSlots >= 3) st.t_ = reinterpret_cast<V3<T>*>(ptr[2]);
  if (kSlots >= 4) st.s_ = reinterpret_cast<V3<T>*>(ptr[3]);
  if (kSlots >= 1) {
    for (int i = v0 + int(threadIdx.x); i < v1; i += int(blockDim.x)) {
      st.p(i) = g.p[i];
      if (kSlots >= 2) st.q(i) = g.q[i];
      if (kSlots >= 3) st.t(i) = g.t[i];
      if (kSlots >= 4) st.s(i) = g.s[i];
    }
    __syncthreads();
  }
  return st;
}

template <int kSlots, typename T>
__device__ __forceinline__ void sw_store(const DevGraph<T>& g, const SwState<T>& st, int v0,
                                         int v1) {
  if (kSlots >= 1) {
    for (int i = v0 + int(threadIdx.x); i < v1; i += int(blockDim.x)) {
      g.p[i] = st.p(i);
      if (kSlots >= 2) g.q[i] = st.q(i);
      if (kSlots >= 3) g.t[i] = st.t(i);
      if (kSlots >= 4) g.s[i] = st.s(i);
    }
  }
}

// The stopping rule's reduction: the four squared changes of a check sweep
// are summed in FP64 per thread, then over the workgroup: wave shuffles,
// one slot per wave, thread 0 adding the slots in order (deterministic).
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

// k sweeps of the graph [v0, v1) (kStop: up to k, with the stopping rule
// evaluated every sp.check_every sweeps; done receives the sweeps run).
// kVpt > 0: thread t owns vertices v0 + t + r * blockDim, r < kVpt, and
// keeps their lambda and z in registers, and with kXyReg also the slot
// between phases (xy, xm); kVpt = 0: all owner-only values in memory.
template <int kVpt, bool kXyReg, int kSlots, bool kStop, typename T>
__device__ __forceinline__ void graph_run(const DevGraph<T>& g, int gr, int v0, int v1, int k,
                                          const SweepParams& sp, unsigned char* lds,
                                          double* red) {
  if (sp.snap[0]) {  // the state before the call, for undoing it (same owner mapping)
    for (int i = v0 + int(threadIdx.x); i < v1; i += int(blockDim.x)) {
      static_cast<Q4<T>*>(sp.snap[0])[i] = g.p[i];
      static_cast<Q4<T>*>(sp.snap[1])[i] = g.q[i];
      static_cast<Q4<T>*>(sp.snap[2])[i] = g.lam[i];
      static_cast<V3<T>*>(sp.snap[3])[i] = g.t[i];
      static_cast<V3<T>*>(sp.snap[4])[i] = g.s[i];
      static_cast<V3<T>*>(sp.snap[5])[i] = g.z[i];
    }
  }
  const SwState<T> st = sw_load<kSlots>(g, v0, v1, lds);
  const int tid = int(threadIdx.x), bd = int(blockDim.x);
  Own<T> o[kVpt > 0 ? kVpt : 1];
  // owner-only values to memory and back (around the rare FP64 islands)
  auto own_out = [&]() {
#pragma unroll
    for (int r = 0; r < kVpt; ++r) {
      const int i = vertex_of(v0 + tid + r * bd);
      if (i < v1) {
        g.lam[i] = o[r].lam;
        g.z[i] = o[r].z;
        if (kXyReg) {
          g.xy[i] = o[r].xy;
          g.xm[i] = o[r].xm;
        }
      }
    }
  };
  auto own_in = [&]() {
#pragma unroll
    for (int r = 0; r < kVpt; ++r) {
      const int i = vertex_of(v0 + tid + r * bd);
      if (i < v1) {
        o[r].lam = g.lam[i];
        o[r].z = g.z[i];
        o[r].cq = g.cQ[i];
        if (kXyReg) {
          o[r].xy = g.xy[i];
          o[r].xm = g.xm[i];
        }
      }
    }
  };
  if constexpr (kVpt > 0) {
#pragma unroll
    for (int r = 0; r < kVpt; ++r) {
      const int i = vertex_of(v0 + tid + r * bd);
      if (i < v1) {
        o[r].lam = g.lam[i];
        o[r].z = g.z[i];
        o[r].cq = g.cQ[i];
      }
    }
  }
  // Vertices whose FP32 P update cancelled get the FP64 island after the
  // thread's other vertices of the phase.  That is rare, so the thread's
  // owner-only values go to memory around it and come back after: the
  // island's registers never add to those the values hold.
  auto islands = [&](unsigned redo) {
    if constexpr (kVpt > 0) {
      own_out();
#pragma unroll
      for (int r = 0; r < kVpt; ++r) {
        const int i = vertex_of(v0 + tid + r * bd);
        if (redo & (1u << r)) g.xy[i] = p_island(g, st, i, sp, st.p(i), g.lam[i]);
      }
      own_in();
    }
  };
  auto phase_p = [&]() {  // the opening P
    if constexpr (kVpt > 0) {
      unsigned redo = 0;
#pragma unroll
      for (int r = 0; r < kVpt; ++r) {
        const int i = vertex_of(v0 + tid + r * bd);
        if (i < v1) {
          Q4<T> x;
          if (!vertex_P<kUnrollReg<T>>(g, st, i, sp, o[r].lam, x)) redo |= 1u << r;
          else if (kXyReg) o[r].xy = x;
          else g.xy[i] = x;
        }
      }
      if (redo) islands(redo);
    } else {
      for (int i = v0 + tid; i < v1; i += bd) phase_mem<0, T>(g, st, i, sp, false);
    }
  };
  auto phase_q = [&](bool save, double* d) {
    if constexpr (kVpt > 0) {
#pragma unroll
      for (int r = 0; r < kVpt; ++r) {
        const int i = vertex_of(v0 + tid + r * bd);
        if (i < v1) vertex_Q<kUnrollQ>(g, st, i, sp, save, o[r].lam, kXyReg ? o[r].xy : g.xy[i], o[r].cq, d);
      }
    } else {
      for (int i = v0 + tid; i < v1; i += bd) phase_mem<1, T>(g, st, i, sp, save, d);
    }
  };
  auto phase_t = [&](bool save, double* d) {
    if constexpr (kVpt > 0) {
#pragma unroll
      for (int r = 0; r < kVpt; ++r) {
        const int i = vertex_of(v0 + tid + r * bd);
        if (i < v1) {
          Q4<T> y;
          T ym;
          vertex_T<kUnrollReg<T>>(g, st, i, sp, save, o[r].z, y, ym, d);
          if (kXyReg) {
            o[r].xy = y;
            o[r].xm = ym;
          } else {
            g.xy[i] = y;
            if (sizeof(T) == 4) g.xm[i] = ym;
          }
        }
      }
    } else {
      for (int i = v0 + tid; i < v1; i += bd) phase_mem<2, T>(g, st, i, sp, save, d);
    }
  };
  auto phase_sp = [&]() {  // S of this sweep + P of the next
    if constexpr (kVpt > 0) {
      unsigned redo = 0;
#pragma unroll
      for (int r = 0; r < kVpt; ++r) {
        const int i = vertex_of(v0 + tid + r * bd);
        if (i < v1) {
          Q4<T> xy = kXyReg ? o[r].xy : g.xy[i];
          const T ym = kXyReg ? o[r].xm : (sizeof(T) == 4 ? g.xm[i] : T(0));
          if (!vertex_S<true, kUnrollReg<T>>(g, st, i, sp, false, o[r].z, o[r].lam, xy, ym))
            redo |= 1u << r;
          else if (kXyReg) o[r].xy = xy;
          else g.xy[i] = xy;
        }
      }
      if (redo) islands(redo);
    } else {
      for (int i = v0 + tid; i < v1; i += bd) phase_mem<4, T>(g, st, i, sp, false);
    }
  };
  auto phase_s = [&](double* d) {  // a plain S that records the residual history
    if constexpr (kVpt > 0) {
#pragma unroll
      for (int r = 0; r < kVpt; ++r) {
        const int i = vertex_of(v0 + tid + r * bd);
        Q4<T> unused = {};
        if (i < v1) vertex_S<false, kUnrollReg<T>>(g, st, i, sp, true, o[r].z, o[r].lam, unused, T(0), d);
      }
    } else {
      for (int i = v0 + tid; i < v1; i += bd) phase_mem<3, T>(g, st, i, sp, true, d);
    }
  };

  phase_p();
  __syncthreads();
  if constexpr (!kStop) {
    for (int it = 0; it < k; ++it) {
      const bool save = it == k - 1;
      phase_q(save, nullptr);
      __syncthreads();
      phase_t(save, nullptr);
      __syncthreads();
      if (save)
        phase_s(nullptr);
      else
        phase_sp();
      __syncthreads();
    }
  } else {
    const int C = sp.check_every;
    int done = k;
    for (int it = 0; it < k; ++it) {
      const bool check = (it + 1) % C == 0;
      // |dq|^2, |dlambda|^2, |dt|^2, |dz|^2 of this sweep (kept in registers:
      // every sweep adds to them, a check sweep uses them)
      double d[4] = {0.0, 0.0, 0.0, 0.0};
      phase_q(check, d);
      __syncthreads();
      phase_t(check, d);
      __syncthreads();
      if (!check) {
        phase_sp();
        __syncthreads();
        continue;
      }
      // a check sweep ends with a plain S, as the last sweep of any launch
      phase_s(d);
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
      phase_p();
      __syncthreads();
    }
    if (threadIdx.x == 0) sp.done[gr] = done;
  }
  sw_store<kSlots>(g, st, v0, v1);
  if constexpr (kVpt > 0) {
#pragma unroll
    for (int r = 0; r < kVpt; ++r) {
      const int i = vertex_of(v0 + tid + r * bd);
      if (i < v1) {
        g.lam[i] = o[r].lam;
        g.z[i] = o[r].z;
      }
    }
  }
}

// The variants one kernel holds (each adds compile time): owner-only
// values in registers for up to kVptA vertices per thread with the slot,
// kVptB without it, each with the LDS slot counts a 1024-thread workgroup
// meets on graphs of that size; everything else keeps the owner-only values
// in memory.
template <typename T>
struct Variants;
template <>
struct Variants<float> {
  static constexpr int kVptA = 3, kVptB = 5;
};
template <>
struct Variants<double> {
  static constexpr int kVptA = 1, kVptB = 2;
};

template <bool kStop, typename T>
__global__ void __launch_bounds__(1024) k_graph_sweeps(DevGraph<T> g,
                                                       const int32_t* __restrict__ voff,
                                                       const int32_t* __restrict__ order, int k,
                                                       SweepParams sp, int lds_bytes) {
  extern __shared__ unsigned char lds_raw[];
  const int gr = order[blockIdx.x];
  const int v0 = voff[gr], v1 = voff[gr + 1];
  if (sp.active && !sp.active[gr]) {
    if (kStop && threadIdx.x == 0) sp.done[gr] = 0;
    return;
  }
  if (sp.beta_g) sp.beta = sp.beta_g[gr];
  const size_t red_bytes = kStop ? sizeof(double) * kStopSlots : 0;
  double* red = reinterpret_cast<double*>(lds_raw);
  unsigned char* lds = lds_raw + red_bytes;
  const size_t n = size_t(v1 - v0), budget = size_t(lds_bytes) - red_bytes;
  int slots = 0;
  while (slots < kArrays && sw_lds_bytes<T>(slots + 1, n) <= budget) ++slots;
  constexpr int A = Variants<T>::kVptA, B = Variants<T>::kVptB;
  const size_t bd = blockDim.x;
  if (n <= A * bd && slots >= 3) {
    if (slots == 4) graph_run<A, true, 4, kStop, T>(g, gr, v0, v1, k, sp, lds, red);
    else graph_run<A, true, 3, kStop, T>(g, gr, v0, v1, k, sp, lds, red);
    return;
  }
  if (n <= B * bd && slots >= 2) {
    if (slots == 4) graph_run<B, false, 4, kStop, T>(g, gr, v0, v1, k, sp, lds, red);
    else if (slots == 3) graph_run<B, false, 3, kStop, T>(g, gr, v0, v1, k, sp, lds, red);
    else graph_run<B, false, 2, kStop, T>(g, gr, v0, v1, k, sp, lds, red);
    return;
  }
  switch (slots) {
    case 4: graph_run<0, false, 4, kStop, T>(g, gr, v0, v1, k, sp, lds, red); break;
    case 3: graph_run<0, false, 3, kStop, T>(g, gr, v0, v1, k, sp, lds, red); break;
    case 2: graph_run<0, false, 2, kStop, T>(g, gr, v0, v1, k, sp, lds, red); break;
    case 1: graph_run<0, false, 1, kStop, T>(g, gr, v0, v1, k, sp, lds, red); break;
    default: graph_run<0, false, 0, kStop, T>(g, gr, v0, v1, k, sp, lds, red); break;
  }
}

constexpr size_t kLdsBytes = 160 * 1024;

}  // namespace

template <typename T>
hipError_t launch_graph_sweeps_stop(const DevGraph<T>& g, const int32_t* voff,
                                    const int32_t* order, int G, int k, const SweepParams& sp,
                                    int block, int max_n, int lds, hipStream_t st) {
  if (G <= 0 || k <= 0) return hipSuccess;
  if (block <= 0 || block > 1024 || block % 64) return hipErrorInvalidValue;
  if (sp.check_every < 1 || k % sp.check_every || !sp.done) return hipErrorInvalidValue;
  const size_t red = sizeof(double) * kStopSlots;
  const size_t bytes =
      lds ? std::min(kLdsBytes, red + sw_lds_bytes<T>(kArrays, size_t(max_n))) : red;
  if (hipFuncSetAttribute(reinterpret_cast<const void*>(&k_graph_sweeps<true, T>),
                          hipFuncAttributeMaxDynamicSharedMemorySize, int(bytes)) != hipSuccess)
    return hipGetLastError();
  hipLaunchKernelGGL((k_graph_sweeps<true, T>), dim3(G), dim3(block), bytes, st, g, voff, order,
                     k, sp, int(bytes));
  return hipGetLastError();
}

template <typename T>
hipError_t launch_graph_sweeps(const DevGraph<T>& g, const int32_t* voff, const int32_t* order,
                               int G, int k, const SweepParams& sp, int block, int max_n,
                               int lds, hipStream_t st) {
  if (G <= 0 || k <= 0) return hipSuccess;
  if (block <= 0 || block > 1024 || block % 64) return hipErrorInvalidValue;
  // enough for p, q, t, s of the largest graph, within the 160 KiB of a CU
  size_t bytes = lds ? std::min(kLdsBytes, sw_lds_bytes<T>(kArrays, size_t(max_n))) : 0;
  if (bytes && hipFuncSetAttribute(reinterpret_cast<const void*>(&k_graph_sweeps<false, T>),
                                   hipFuncAttributeMaxDynamicSharedMemorySize,
                                   int(bytes)) != hipSuccess) {
    (void)hipGetLastError();  // clear a refused request; run without LDS residency
    bytes = 0;
  }
  hipLaunchKernelGGL((k_graph_sweeps<false, T>), dim3(G), dim3(block), bytes, st, g, voff, order,
                     k, sp, int(bytes));
  return hipGetLastError();
}

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
