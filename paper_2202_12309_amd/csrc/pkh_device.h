// pkh_device.h -- device helpers shared by the stage kernels and the other
// kernels of the cycle.
#pragma once

#include "pkh_internal.h"
#include "pkh_physics.h"

namespace pkh {

// Write an updated active cell (i, j, k) of a leaf into the ghost zones of
// the same-level neighbours that need it (cells within 2 of a face, edge or
// corner). nb27: the leaf's neighbour row.
__device__ __forceinline__ void push_ghosts(double* u, const int32_t* nb27, const Geom& g, int i,
                                            int j, int k, const double val[NV]) {
  const int dx = i < NG ? -1 : (i >= g.n1 - NG ? 1 : 0);
  const int dy = j < NG ? -1 : (j >= g.n2 - NG ? 1 : 0);
  const int dz = k < NG ? -1 : (k >= g.n3 - NG ? 1 : 0);
  auto put = [&](int ex, int ey, int ez) {
    const int32_t nb = nb27[(ez + 1) * 9 + (ey + 1) * 3 + (ex + 1)];
    if (nb < 0) return;
    double* d = u + (int64_t)nb * g.bstride +
                ((int64_t)(k - ez * g.n3 + NG) * g.p2 + (j - ey * g.n2 + NG)) * g.p1 + (i - ex * g.n1 + NG);
#pragma unroll
    for (int v = 0; v < NV; ++v) d[v * g.vstride] = val[v];
  };
  if (dx) put(dx, 0, 0);
  if (dy) {
    put(0, dy, 0);
    if (dx) put(dx, dy, 0);
  }
  if (dz) {
    put(0, 0, dz);
    if (dx) put(dx, 0, dz);
    if (dy) {
      put(0, dy, dz);
      if (dx) put(dx, dy, dz);
    }
  }
}


// Index of cell s (-2 <= s < n1 + 2) of x-row (j, k) of block b in a padded
// state: cells beyond the block come from the active cells of the same-level
// x neighbour when there is one (the stage kernels keep no x ghost zone for
// those), else from the block's ghost zone.
__device__ __forceinline__ int64_t xrow_cell(const Geom& g, const int32_t* nbr, int b, int j, int k, int s) {
  int bb = b, ss = s;
  if (nbr && (s < 0 || s >= g.n1)) {
    const int32_t nb = nbr[(int64_t)b * 27 + (s < 0 ? 12 : 14)];
    if (nb >= 0) {
      bb = nb;
      ss = s < 0 ? s + g.n1 : s - g.n1;
    }
  }
  return (int64_t)bb * g.bstride + ((int64_t)(k + NG) * g.p2 + (j + NG)) * g.p1 + NG + ss;
}

// The stage kernels' push: only the y and z face regions. The stage kernels
// read the x halo from the x neighbours' active cells and never read edge or
// corner ghost regions, so those are left to the full exchange.
__device__ __forceinline__ void push_yz_ghosts(double* u, const int32_t* nb27, const Geom& g, int i,
                                               int j, int k, const double val[NV]) {
  const int dy = j < NG ? -1 : (j >= g.n2 - NG ? 1 : 0);
  const int dz = k < NG ? -1 : (k >= g.n3 - NG ? 1 : 0);
  auto put = [&](int ey, int ez) {
    const int32_t nb = nb27[(ez + 1) * 9 + (ey + 1) * 3 + 1];
    if (nb < 0) return;
    double* d = u + (int64_t)nb * g.bstride +
                ((int64_t)(k - ez * g.n3 + NG) * g.p2 + (j - ey * g.n2 + NG)) * g.p1 + (i + NG);
#pragma unroll
    for (int v = 0; v < NV; ++v) d[v * g.vstride] = val[v];
  };
  if (dy) put(dy, 0);
  if (dz) put(0, dz);
}

}  // namespace pkh
