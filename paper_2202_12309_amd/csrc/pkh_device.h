// pkh_device.h -- device helpers shared by the stage kernels and the other
// kernels of the cycle.
#pragma once

#include "pkh_internal.h"
#include "pkh_physics.h"

namespace pkh {

// Load of a value the whole wave reads at one address, from memory that no
// thread writes while the kernel runs (block tables, neighbour lists, launch
// records): read through the constant address space it becomes a scalar
// load into SGPRs. A generic load inside a loop that also stores to global
// memory cannot be proven unclobbered, and its result, with everything
// derived from it, would occupy VGPRs.
template <class T>
__device__ __forceinline__ T load_uniform(const T* p) {
#if defined(__HIP_DEVICE_COMPILE__)
  return *(const __attribute__((address_space(4))) T*)p;
#else
  return *p;  // the host pass only parses device code
#endif
}

// Fold a workgroup's largest signal speed per cell width (mx >= 0) into the
// cycle's CFL reduction. Non-negative doubles order like their bit
// patterns; the maximum only grows within a cycle, so a workgroup whose
// value is already covered skips the atomic: launches with many
// workgroups would otherwise queue thousands of atomics on one address.
__device__ __forceinline__ void reduce_max_speed(DevTime* tm, double mx) {
  const unsigned long long b = (unsigned long long)__double_as_longlong(mx);
  if (__hip_atomic_load(&tm->smax_bits, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) < b) atomicMax(&tm->smax_bits, b);
}

// Padded index of cell (i, j, k) of block b, the cell at most one face step
// outside the block (-2 <= i < n1 + 2 with j, k active, and likewise for y
// and z): a cell beyond the block comes from the active cells of the
// same-level neighbour across that face when there is one (no kernel keeps
// ghost zones for same-level faces), else from the block's ghost zone,
// which the fill kernel writes for faces to other levels.
__device__ __forceinline__ int64_t nb_index(const Geom& g, const int32_t* nbr, int b, int i, int j, int k) {
  const int dx = i < 0 ? -1 : (i >= g.n1 ? 1 : 0);
  const int dy = j < 0 ? -1 : (j >= g.n2 ? 1 : 0);
  const int dz = k < 0 ? -1 : (k >= g.n3 ? 1 : 0);
  if (nbr && (dx | dy | dz)) {
    const int32_t nb = nbr[(int64_t)b * 27 + (dz + 1) * 9 + (dy + 1) * 3 + (dx + 1)];
    if (nb >= 0) {
      b = nb;
      i -= dx * g.n1;
      j -= dy * g.n2;
      k -= dz * g.n3;
    }
  }
  return (int64_t)b * g.bstride + ((int64_t)(k + NG) * g.p2 + (j + NG)) * g.p1 + (i + NG);
}

}  // namespace pkh
