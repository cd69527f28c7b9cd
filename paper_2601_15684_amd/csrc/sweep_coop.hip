// The PRADMM sweep in one persistent cooperative launch: every phase spreads
// the handle's vertices over all workgroups of the launch (as the per-phase
// launches do), and a device-wide barrier separates the phases in place of
// a kernel boundary.  A k-sweep call is one launch of 3k barriers instead of
// 3k + 1 launches, which is what a single mid-sized graph (a few thousand
// to a few hundred thousand poses) needs: too large for one workgroup, too
// small to hide a launch per phase.  The vertex updates are those of
// sweep_core.hpp, in the same order per vertex as the per-phase schedule,
// so both schedules give bitwise the same state.
#pragma clang fp contract(off)
#include <algorithm>

#include "sweep_core.hpp"

namespace pgo {

namespace {

constexpr int kXcds = 8;
// Spin limit of one barrier wait: seconds with the sleep below, where a
// phase takes microseconds to milliseconds.  A workgroup that waits this
// long stops waiting, marks the launch as failed (bar[1]) and writes NaN
// into the first vertex's translation, so the failure is visible to every
// later cost or merit check; the launch still ends.
constexpr unsigned kSpinLimit = 1u << 22;

// Workgroups are dispatched to the XCDs round-robin; this renumbering gives
// each XCD one contiguous range of workgroups (and so of vertices).
__device__ __forceinline__ int xcd_block() {
  const int b = blockIdx.x, nb = gridDim.x;
  const int xcd = b % kXcds, local = b / kXcds;
  const int per = nb / kXcds, rem = nb % kXcds;
  return xcd < rem ? xcd * (per + 1) + local : rem * (per + 1) + (xcd - rem) * per + local;
}

// Device-wide barrier on a counter that starts at 0 for the launch: every
// workgroup adds 1 per barrier and waits until the count reaches (barriers
// so far) x (workgroups).  Every wave first waits until its own stores are
// acknowledged (they are then in its XCD's L2), so after the workgroup
// barrier one release fence by the arriving thread writes all of the
// workgroup's results back to device scope; its acquire fence after the
// wait drops the CU's and the XCD's stale cached lines before any thread of
// the workgroup reads what others wrote.  (One write-back and one
// invalidation per workgroup and barrier: a fence in every wave costs an L2
// write-back per wave.)  The wait polls with relaxed device-scope loads, so
// no cache is invalidated while polling.  A workgroup whose earlier wait
// timed out (wait false) still arrives but no longer waits, so a broken
// launch ends after one spin limit per workgroup.
__device__ __forceinline__ bool grid_barrier(unsigned* bar, unsigned& goal, bool wait) {
  goal += gridDim.x;
  __builtin_amdgcn_s_waitcnt(0);
  __syncthreads();
  __shared__ int timed_out;
  if (threadIdx.x == 0) {
    timed_out = 0;
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
    __hip_atomic_fetch_add(bar, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    unsigned spins = 0;
    while (wait && __hip_atomic_load(bar, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) < goal) {
      if (++spins == kSpinLimit) {
        timed_out = 1;
        break;
      }
      __builtin_amdgcn_s_sleep(2);
    }
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
  }
  __syncthreads();
  return timed_out == 0;
}

template <int PH, typename T>
__device__ __forceinline__ void coop_phase(const DevGraph<T>& g, const SweepParams& sp, int lo,
                                           int hi, bool save) {
  const SwState<T> st = sw_global(g);
  for (int i = lo + int(threadIdx.x); i < hi; i += int(blockDim.x)) {
    if (sp.active && !sp.active[g.gid[i]]) continue;
    SweepParams spi = sp;
    if (sp.beta_g) spi.beta = sp.beta_g[g.gid[i]];
    phase_mem<PH, T>(g, st, i, spi, save);
  }
}

__global__ void k_coop_reset(unsigned* bar) {
  if (threadIdx.x == 0) bar[0] = 0u;
}

struct Fit {
  int block = 0, per_cu = 0;
};

}  // namespace

// One call of k sweeps: P, then k times (Q, T, S+P), the last S+P a plain S
// that records the residual history with the Q and T of the last sweep.
// Workgroup b (renumbered by XCD) owns vertices [b chunk, (b + 1) chunk).
template <typename T>
__global__ void k_coop_sweeps(DevGraph<T> g, SweepParams sp, int k, int chunk, unsigned* bar) {
  const int lo = xcd_block() * chunk;
  const int hi = min(g.n, lo + chunk);
  unsigned goal = 0;
  bool ok = true;
  coop_phase<0, T>(g, sp, lo, hi, false);
  for (int it = 0; it < k; ++it) {
    const bool last = it == k - 1;
    ok = grid_barrier(bar, goal, ok) && ok;
    coop_phase<1, T>(g, sp, lo, hi, last);
    ok = grid_barrier(bar, goal, ok) && ok;
    coop_phase<2, T>(g, sp, lo, hi, last);
    ok = grid_barrier(bar, goal, ok) && ok;
    if (last)
      coop_phase<3, T>(g, sp, lo, hi, true);
    else
      coop_phase<4, T>(g, sp, lo, hi, false);
  }
  if (!ok && threadIdx.x == 0) {
    __hip_atomic_store(bar + 1, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    g.t[0] = V3<T>{T(NAN), T(NAN), T(NAN)};
  }
}

// Workgroups of a launch: co-resident ones only (the barrier needs all of
// them running), and at most one per compute unit -- every workgroup writes
// its XCD's L2 back and invalidates it once per barrier, and those
// operations queue per XCD, so the barrier's cost grows with the workgroup
// count (measured: about 10 us per barrier with 100 workgroups, 30 us with
// 400).
template <typename T>
int coop_max_blocks(int block) {
  // (cached: the answer depends only on the kernel and the device)
  static thread_local Fit cache[2][17];
  int dev = 0, cus = 0;
  if (hipGetDevice(&dev) != hipSuccess ||
      hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess)
    return 0;
  Fit& f = cache[sizeof(T) == 8][block / 64];
  if (f.block != block) {
    int per = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per, k_coop_sweeps<T>, block, 0) !=
        hipSuccess)
      return 0;
    f = Fit{block, per};
  }
  return std::min(f.per_cu, 1) * cus;
}

template <typename T>
hipError_t launch_coop_sweeps(const DevGraph<T>& g, int k, const SweepParams& sp, int block,
                              unsigned* bar, hipStream_t st) {
  if (g.n <= 0 || k <= 0) return hipSuccess;
  if (block <= 0 || block > 1024 || block % 64 || !bar) return hipErrorInvalidValue;
  const int fit = coop_max_blocks<T>(block);
  if (fit <= 0) return hipErrorInvalidConfiguration;
  const int nb = std::min<int64_t>(fit, (int64_t(g.n) + block - 1) / block);
  const int chunk = (g.n + nb - 1) / nb;
  // the barrier count of one launch, 3k nb, stays below 2^31
  const int k_max = int((int64_t(1) << 31) / (3 * int64_t(nb)));
  for (int done = 0; done < k;) {
    const int kk = std::min(k - done, k_max);
    hipLaunchKernelGGL(k_coop_reset, dim3(1), dim3(64), 0, st, bar);
    DevGraph<T> ga = g;
    SweepParams spa = sp;
    int kka = kk, chunka = chunk;
    unsigned* bara = bar;
    void* args[] = {&ga, &spa, &kka, &chunka, &bara};
    const hipError_t e = hipLaunchCooperativeKernel(reinterpret_cast<void*>(k_coop_sweeps<T>),
                                                    dim3(nb), dim3(block), args, 0, st);
    if (e != hipSuccess) return e;
    done += kk;
  }
  return hipGetLastError();
}

template int coop_max_blocks<float>(int);
template int coop_max_blocks<double>(int);
template hipError_t launch_coop_sweeps<float>(const DevGraph<float>&, int, const SweepParams&, int,
                                              unsigned*, hipStream_t);
template hipError_t launch_coop_sweeps<double>(const DevGraph<double>&, int, const SweepParams&,
                                               int, unsigned*, hipStream_t);

}  // namespace pgo
