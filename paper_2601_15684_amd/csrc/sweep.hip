// The PRADMM sweep, one launch per phase (the vertex updates are in
// sweep_core.hpp): every phase spreads all vertices of the handle over the
// whole GPU, the owner-only values (lambda, z and the slot between phases)
// live in global memory, and the k-sweep launch sequence is captured once
// into a HIP graph by the host.
#pragma clang fp contract(off)
#include "sweep_core.hpp"

namespace pgo {

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

// phase bodies: 0 P, 1 Q, 2 T, 3 S, 4 S of this sweep + P of the next
template <int PH, typename T>
__global__ void k_phase(DevGraph<T> g, SweepParams sp, int save) {
  const int i = xcd_block() * blockDim.x + threadIdx.x;
  if (i >= g.n) return;
  if (sp.active && !sp.active[g.gid[i]]) return;
  if (sp.beta_g) sp.beta = sp.beta_g[g.gid[i]];
  phase_mem<PH, T>(g, sw_global(g), i, sp, save != 0);
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

template hipError_t launch_phase_sweeps<float>(const DevGraph<float>&, int, const SweepParams&,
                                               int, hipStream_t);
template hipError_t launch_phase_sweeps<double>(const DevGraph<double>&, int,
                                                const SweepParams&, int, hipStream_t);

}  // namespace pgo
