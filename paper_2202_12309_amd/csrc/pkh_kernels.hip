// pkh_kernels.hip -- gfx950 kernels of the block-AMR Euler cycle.
//
// Method (Parthenon, arXiv:2202.12309, Sec. 4.1): two-stage second-order
// finite-volume update, piecewise-linear reconstruction with the MC limiter
// on primitive variables, HLLE fluxes with Einfeldt's Roe-averaged wave
// speeds, flux-divergence update. Ghost zones (Sec. 3.7) are filled on the
// device from neighbouring leaves: copy, restriction (volume average of 8
// fine cells) or linear prolongation with minmod slopes of the composite
// coarse field. Fine-coarse flux correction (Sec. 3.7) is applied as a
// reflux of the coarse cells after each stage. The CFL timestep and the
// conserved totals are device reductions (Sec. 3.10).
//
// Layout: every state array is [block][var][k][j][i] with ghost width 2 on
// each side, i (x) contiguous. One launch covers every block of the mesh.
#include <math.h>

#include <algorithm>
#include <mutex>

#include "pkh_amr.h"
#include "pkh_device.h"

// waves per SIMD the reverse pencils are compiled for: at 1 they take 412
// VGPRs without spilling; at 2 the 256-register cap spills (156 B a lane)
// and a reverse stage of the 128^3 workload took 20 % longer
#ifndef PKH_ADJ_PENCIL_WAVES
#define PKH_ADJ_PENCIL_WAVES 1
#endif

namespace pkh {

// ---------------------------------------------------------------------------
// Fill-in-one ghost exchange: one thread per (block, ghost cell), all five
// variables; ghost cells enumerated in memory order of the padded block.
// ---------------------------------------------------------------------------

__device__ __forceinline__ void ghost_coord(int q, const Geom& g, int& i, int& j, int& k) {
  const int e1 = g.n1 + 2 * NG;  // x extent with ghosts (the row pitch may be larger)
  const int plane = e1 * g.p2;
  if (q < 4 * plane) {
    const int s = q / plane, r = q - s * plane;
    k = s < 2 ? s - NG : g.n3 + s - 2;
    j = r / e1 - NG;
    i = r - (j + NG) * e1 - NG;
    return;
  }
  q -= 4 * plane;
  const int rows = 4 * e1;
  if (q < g.n3 * rows) {
    k = q / rows;
    const int r = q - k * rows;
    const int s = r / e1;
    i = r - s * e1 - NG;
    j = s < 2 ? s - NG : g.n2 + s - 2;
    return;
  }
  q -= g.n3 * rows;
  const int kj = q >> 2, s = q & 3;
  k = kj / g.n2;
  j = kj - k * g.n2;
  i = s < 2 ? s - NG : g.n1 + s - 2;
}

// Value of ghost cell (i, j, k) of leaf b from the leaf data (copy,
// restriction or prolongation); a ghost cell beyond a wall takes the value
// of its image inside the domain, with the image's momentum signs.
// skip_same leaves cells inside the domain whose source is a same-level
// leaf alone.
__device__ __forceinline__ void fill_cell(double* u, const BlockInfo* blocks, const Geom& g, const LevelMaps& M,
                                          DevTime* tm, int b, int i, int j, int k, int skip_same) {
  const BlockInfo bi = blocks[b];
  const int L = bi.level;
  const int n[3] = {g.n1, g.n2, g.n3};
  int J[3] = {bi.lx * g.n1 + i, bi.ly * g.n2 + j, bi.lz * g.n3 + k};
  const int code = cell_in_domain(g, L, J);
  const int bl[3] = {J[0] / n[0], J[1] / n[1], J[2] / n[2]};
  double* dst = u + (int64_t)b * g.bstride + pad_index(g, i, j, k);
  int err = 0;
  double val[NV];
  const int32_t id = leaf_at(M, L, bl[0], bl[1], bl[2]);
  if (id >= 0) {  // same level: copy
    if (skip_same && !(code & 8)) return;
    const double* src = u + (int64_t)id * g.bstride +
                        pad_index(g, J[0] - bl[0] * n[0], J[1] - bl[1] * n[1], J[2] - bl[2] * n[2]);
#pragma unroll
    for (int v = 0; v < NV; ++v) val[v] = src[v * g.vstride];
  } else if (L > 0 && leaf_at(M, L - 1, bl[0] >> 1, bl[1] >> 1, bl[2] >> 1) >= 0) {
    prolong_val(u, blocks, M, g, L, J[0], J[1], J[2], val, &err);
  } else {
    comp_val_inside(u, blocks, M, g, L, J, val, &err);
  }
  apply_image_signs(code, val);
#pragma unroll
  for (int v = 0; v < NV; ++v) dst[v * g.vstride] = val[v];
  if (err) atomicOr(&tm->err, 2);
}

// Every ghost region (all 26) of every leaf.
__global__ void __launch_bounds__(256) fill_kernel(double* u, const BlockInfo* blocks, int nblocks,
                                                   Geom g, LevelMaps M, DevTime* tm, int skip_same) {
  const int ngc = 4 * (g.n1 + 2 * NG) * g.p2 + 4 * g.n3 * (g.n1 + 2 * NG) + 4 * g.n3 * g.n2;
  const int q = blockIdx.x * blockDim.x + threadIdx.x;
  const int b = blockIdx.y;
  if (q >= ngc || b >= nblocks) return;
  int i, j, k;
  ghost_coord(q, g, i, j, k);
  fill_cell(u, blocks, g, M, tm, b, i, j, k, skip_same);
}

__global__ void __launch_bounds__(256) fill_faces_kernel(double* u, Geom g, DevTime* tm,
                                                         const int32_t* __restrict__ jf,
                                                         const uint2* __restrict__ plan) {
  fill_faces_item(u, g, tm, jf, plan, blockIdx.x, blockIdx.y);
}

hipError_t launch_fill_faces(double* u, const Geom& g, DevTime* tm, const int32_t* jf, const uint2* plan,
                             int32_t njf, hipStream_t s) {
  if (njf <= 0) return hipSuccess;
  dim3 grid(fill_faces_stride(g) / 256, njf);
  hipLaunchKernelGGL(fill_faces_kernel, grid, dim3(256), 0, s, u, g, tm, jf, plan);
  return hipGetLastError();
}

// The face-fill plan: for every thread of every face record, the location
// its value is read from (fill_faces_loc), so the fill after each stage
// reads it instead of walking the level maps. Threads with no cell get
// LOC_NONE.
__global__ void __launch_bounds__(256) fill_plan_kernel(uint2* plan, const BlockInfo* blocks, Geom g, LevelMaps M,
                                                        const int32_t* __restrict__ jf) {
  const int f = blockIdx.y, q = blockIdx.x * 256 + threadIdx.x;
  uint2 e = make_uint2(LOC_NONE, 0u);
  fill_faces_loc(blocks, g, M, reinterpret_cast<const int2*>(jf)[f], q, &e);
  plan[(int64_t)f * fill_faces_stride(g) + q] = e;
}

hipError_t launch_fill_plan(uint2* plan, const BlockInfo* blocks, const Geom& g, const LevelMaps& maps,
                            const int32_t* jf, int32_t njf, hipStream_t s) {
  if (njf <= 0) return hipSuccess;
  dim3 grid(fill_faces_stride(g) / 256, njf);
  hipLaunchKernelGGL(fill_plan_kernel, grid, dim3(256), 0, s, plan, blocks, g, maps, jf);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Remote faces of a partitioned mesh (the buffers of Sec. 3.7 for faces
// whose neighbour lives in another part): pack the sender's two cell layers
// next to the face, and after the transfer unpack them into the receiver's
// ghost layers. One thread per (layer, face cell), all five variables.
// ---------------------------------------------------------------------------

__global__ void __launch_bounds__(256) remote_pack_kernel(const double* __restrict__ u, Geom g,
                                                          const RemoteFace* __restrict__ rf,
                                                          double* __restrict__ buf, int64_t slot) {
  const RemoteFace r = rf[blockIdx.y];
  const int d = r.face >> 1, hi = r.face & 1;
  const int n[3] = {g.n1, g.n2, g.n3};
  const int t1 = d == 0 ? 1 : 0, t2 = d == 2 ? 1 : 2;
  const int area = n[t1] * n[t2];
  const int q = blockIdx.x * blockDim.x + threadIdx.x;
  if (q >= 2 * area) return;
  const int s = q / area, rr = q - s * area;
  int c[3];
  c[t1] = rr % n[t1];
  c[t2] = rr / n[t1];
  // the receiver's ghost layer n + s (high face) or s - 2 (low face) is the
  // sender's cell layer s or n - 2 + s
  c[d] = hi ? s : n[d] - NG + s;
  const double* src = u + (int64_t)r.send * g.bstride + pad_index(g, c[0], c[1], c[2]);
  double* dst = buf + (int64_t)blockIdx.y * slot + q;
#pragma unroll
  for (int v = 0; v < NV; ++v) dst[(int64_t)v * 2 * area] = src[v * g.vstride];
}

__global__ void __launch_bounds__(256) remote_unpack_kernel(double* __restrict__ u, Geom g,
                                                            const RemoteFace* __restrict__ rf,
                                                            const double* __restrict__ buf, int64_t slot) {
  const RemoteFace r = rf[blockIdx.y];
  const int d = r.face >> 1, hi = r.face & 1;
  const int n[3] = {g.n1, g.n2, g.n3};
  const int t1 = d == 0 ? 1 : 0, t2 = d == 2 ? 1 : 2;
  const int area = n[t1] * n[t2];
  const int q = blockIdx.x * blockDim.x + threadIdx.x;
  if (q >= 2 * area) return;
  const int s = q / area, rr = q - s * area;
  int c[3];
  c[t1] = rr % n[t1];
  c[t2] = rr / n[t1];
  c[d] = hi ? n[d] + s : s - NG;
  double* dst = u + (int64_t)r.recv * g.bstride + pad_index(g, c[0], c[1], c[2]);
  const double* src = buf + (int64_t)blockIdx.y * slot + q;
#pragma unroll
  for (int v = 0; v < NV; ++v) dst[v * g.vstride] = src[(int64_t)v * 2 * area];
}

hipError_t launch_remote_pack(const double* u, const RemoteFace* rf, int32_t nrf, const Geom& g, double* buf,
                              int64_t slot, hipStream_t s) {
  if (nrf <= 0) return hipSuccess;
  const int area = std::max(std::max(g.n1 * g.n2, g.n1 * g.n3), g.n2 * g.n3);
  hipLaunchKernelGGL(remote_pack_kernel, dim3((2 * area + 255) / 256, nrf), dim3(256), 0, s, u, g, rf, buf, slot);
  return hipGetLastError();
}

hipError_t launch_remote_unpack(double* u, const RemoteFace* rf, int32_t nrf, const Geom& g, const double* buf,
                                int64_t slot, hipStream_t s) {
  if (nrf <= 0) return hipSuccess;
  const int area = std::max(std::max(g.n1 * g.n2, g.n1 * g.n3), g.n2 * g.n3);
  hipLaunchKernelGGL(remote_unpack_kernel, dim3((2 * area + 255) / 256, nrf), dim3(256), 0, s, u, g, rf, buf,
                     slot);
  return hipGetLastError();
}

hipError_t launch_fill(double* u, const BlockInfo* blocks, int32_t nblocks, const Geom& g,
                       const LevelMaps& maps, DevTime* tm, int32_t skip_same, hipStream_t s) {
  const int ngc = 4 * (g.n1 + 2 * NG) * g.p2 + 4 * g.n3 * (g.n1 + 2 * NG) + 4 * g.n3 * g.n2;
  dim3 grid((ngc + 255) / 256, nblocks);
  hipLaunchKernelGGL(fill_kernel, grid, dim3(256), 0, s, u, blocks, nblocks, g, maps, tm,
                     (int)skip_same);
  return hipGetLastError();
}


__global__ void __launch_bounds__(256) flux_correct_kernel(double* u, const BlockInfo* blocks,
                                                           const FineFace* ff, const int32_t* ff_first,
                                                           const int32_t* cblocks, Geom g, DevTime* tm,
                                                           double beta, int do_dt, const double* fbuf) {
  __shared__ double sRed[4];
  flux_correct_item(u, blocks, ff, ff_first, cblocks, g, tm, tm->dt, beta, do_dt, fbuf, blockIdx.x, blockIdx.y,
                    sRed);
}

hipError_t launch_flux_correct(double* u, const BlockInfo* blocks, const FineFace* ff,
                               const int32_t* ff_first, const int32_t* cblocks, int32_t ncblocks,
                               const Geom& g, DevTime* tm, double beta, int32_t do_dt,
                               const double* fbuf, const int32_t* nbr, hipStream_t s) {
  if (ncblocks == 0) return hipSuccess;
  const int nshell = 2 * g.n1 * g.n2 + (g.n3 - 2) * (2 * g.n1 + 2 * (g.n2 - 2));
  dim3 grid((nshell + 255) / 256, ncblocks);
  hipLaunchKernelGGL(flux_correct_kernel, grid, dim3(256), 0, s, u, blocks, ff, ff_first, cblocks,
                     g, tm, beta, do_dt, fbuf);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// CFL reduction over the active cells (after exchange / regrid / upload).
// ---------------------------------------------------------------------------

template <typename S>
__global__ void __launch_bounds__(256) dt_kernel(const S* u, const BlockInfo* blocks,
                                                 int nblocks, Geom g, DevTime* tm) {
  __shared__ double sRed[4];
  const int ncell = g.n1 * g.n2 * g.n3;
  const int b = blockIdx.y;
  const int q = blockIdx.x * blockDim.x + threadIdx.x;
  double smax = 0.0;
  bool bad = false;
  if (q < ncell && b < nblocks) {
    const BlockInfo bi = blocks[b];
    const int i = q % g.n1, j = (q / g.n1) % g.n2, k = q / (g.n1 * g.n2);
    const S* cell = u + (int64_t)b * g.bstride + pad_index(g, i, j, k);
    double uc[NV], wn[NV];
#pragma unroll
    for (int v = 0; v < NV; ++v) uc[v] = cell[v * g.vstride];
    bad = !to_prim(uc, g.gamma, wn);
    const double cs = sqrt(g.gamma * wn[4] / wn[0]);
    smax = fmax(fmax((fabs(wn[1]) + cs) * bi.idx[0], (fabs(wn[2]) + cs) * bi.idx[1]),
                (fabs(wn[3]) + cs) * bi.idx[2]);
  }
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) smax = fmax(smax, __shfl_xor(smax, off));
  if ((threadIdx.x & 63) == 0) sRed[threadIdx.x >> 6] = smax;
  __syncthreads();
  if (threadIdx.x == 0) {
    const double mx = fmax(fmax(sRed[0], sRed[1]), fmax(sRed[2], sRed[3]));
    reduce_max_speed(tm, mx);
  }
  if (bad) atomicOr(&tm->err, 1);
}

template <typename S>
static hipError_t launch_dt_t(const S* u, const BlockInfo* blocks, int32_t nblocks, const Geom& g,
                              DevTime* tm, hipStream_t s) {
  const int ncell = g.n1 * g.n2 * g.n3;
  dim3 grid((ncell + 255) / 256, nblocks);
  hipLaunchKernelGGL(dt_kernel<S>, grid, dim3(256), 0, s, u, blocks, nblocks, g, tm);
  return hipGetLastError();
}
hipError_t launch_dt(const double* u, const BlockInfo* blocks, int32_t nblocks, const Geom& g,
                     DevTime* tm, hipStream_t s) {
  return launch_dt_t(u, blocks, nblocks, g, tm, s);
}
hipError_t launch_dt(const float* u, const BlockInfo* blocks, int32_t nblocks, const Geom& g,
                     DevTime* tm, hipStream_t s) {
  return launch_dt_t(u, blocks, nblocks, g, tm, s);
}

// Device clock: END closes a cycle (t += dt, cycle++, next dt from the
// reduction); BEGIN opens one (dt = next dt clamped to t_end, reduction
// reset); FROM_SMAX only turns the reduction into the next dt.
__global__ void clock_kernel(DevTime* tm, int mode, double t_end) {
  if (threadIdx.x != 0 || blockIdx.x != 0) return;
  if (mode & (CLOCK_END | CLOCK_FROM_SMAX)) {
    const double smax = __longlong_as_double((long long)tm->smax_bits);
    tm->dt_next = tm->cfl / smax;
  }
  if (mode & CLOCK_END) {
    tm->t += tm->dt;
    tm->cycle += 1;
  }
  if (mode & CLOCK_BEGIN) {
    double dt = tm->dt_next;
    if (isfinite(t_end) && dt > t_end - tm->t) dt = fmax(t_end - tm->t, 0.0);
    tm->dt = dt;
    tm->smax_bits = 0ull;
  }
}

hipError_t launch_clock(DevTime* tm, int32_t mode, double t_end, hipStream_t s) {
  hipLaunchKernelGGL(clock_kernel, dim3(1), dim3(64), 0, s, tm, (int)mode, t_end);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Upload / download between the active-only FP64 layout and padded blocks
// (stored as double, or as float: rounded to nearest on upload).
// ---------------------------------------------------------------------------

template <typename S>
__global__ void __launch_bounds__(256) scatter_kernel(S* u, const double* src, int64_t total,
                                                      Geom g) {
  const int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (q >= total) return;
  const int i = q % g.n1;
  int64_t r = q / g.n1;
  const int j = r % g.n2;
  r /= g.n2;
  const int k = r % g.n3;
  r /= g.n3;  // r = block*5 + v
  u[r * g.vstride + pad_index(g, i, j, k)] = static_cast<S>(src[q]);
}

template <typename S>
__global__ void __launch_bounds__(256) gather_kernel(double* dst, const S* u, int64_t total,
                                                     Geom g) {
  const int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (q >= total) return;
  const int i = q % g.n1;
  int64_t r = q / g.n1;
  const int j = r % g.n2;
  r /= g.n2;
  const int k = r % g.n3;
  r /= g.n3;
  dst[q] = u[r * g.vstride + pad_index(g, i, j, k)];
}

template <typename S>
static hipError_t launch_scatter_t(S* u, const double* src, int32_t nblocks, const Geom& g, hipStream_t s) {
  const int64_t total = (int64_t)nblocks * NV * g.n1 * g.n2 * g.n3;
  hipLaunchKernelGGL(scatter_kernel<S>, dim3((unsigned)((total + 255) / 256)), dim3(256), 0, s, u, src,
                     total, g);
  return hipGetLastError();
}
hipError_t launch_scatter(double* u, const double* src, int32_t nblocks, const Geom& g, hipStream_t s) {
  return launch_scatter_t(u, src, nblocks, g, s);
}
hipError_t launch_scatter(float* u, const double* src, int32_t nblocks, const Geom& g, hipStream_t s) {
  return launch_scatter_t(u, src, nblocks, g, s);
}

template <typename S>
static hipError_t launch_gather_t(double* dst, const S* u, int32_t nblocks, const Geom& g, hipStream_t s) {
  const int64_t total = (int64_t)nblocks * NV * g.n1 * g.n2 * g.n3;
  hipLaunchKernelGGL(gather_kernel<S>, dim3((unsigned)((total + 255) / 256)), dim3(256), 0, s, dst, u,
                     total, g);
  return hipGetLastError();
}
hipError_t launch_gather(double* dst, const double* u, int32_t nblocks, const Geom& g, hipStream_t s) {
  return launch_gather_t(dst, u, nblocks, g, s);
}
hipError_t launch_gather(double* dst, const float* u, int32_t nblocks, const Geom& g, hipStream_t s) {
  return launch_gather_t(dst, u, nblocks, g, s);
}

// ---------------------------------------------------------------------------
// Conserved totals: per-block sums in a fixed order (per-thread strided sums,
// a butterfly of wave shuffles, the block's waves in index order), then one
// workgroup sums the block partials the same way (bitwise reproducible).
// ---------------------------------------------------------------------------

// Sum over the 64 lanes of a wave by an xor butterfly: lanes l and l^off add
// the same two values at each step, so every lane ends with the same sum,
// formed in a fixed order.
__device__ __forceinline__ double wave_sum(double x) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) x += __shfl_xor(x, off);
  return x;
}

template <typename S>
__global__ void __launch_bounds__(256) block_sum_kernel(double* partial, const S* u,
                                                        const BlockInfo* blocks, Geom g) {
  __shared__ double sh[NV][4];
  const int b = blockIdx.x;
  const BlockInfo bi = blocks[b];
  const int ncell = g.n1 * g.n2 * g.n3;
  double acc[NV] = {0, 0, 0, 0, 0};
  for (int q = threadIdx.x; q < ncell; q += 256) {
    const int i = q % g.n1, j = (q / g.n1) % g.n2, k = q / (g.n1 * g.n2);
    const S* cell = u + (int64_t)b * g.bstride + pad_index(g, i, j, k);
#pragma unroll
    for (int v = 0; v < NV; ++v) acc[v] += static_cast<double>(cell[v * g.vstride]);
  }
#pragma unroll
  for (int v = 0; v < NV; ++v) acc[v] = wave_sum(acc[v]);
  if ((threadIdx.x & 63) == 0)
#pragma unroll
    for (int v = 0; v < NV; ++v) sh[v][threadIdx.x >> 6] = acc[v];
  __syncthreads();
  if (threadIdx.x < NV) {
    const int v = threadIdx.x;
    const double dV = 1.0 / (bi.idx[0] * bi.idx[1] * bi.idx[2]);
    partial[(int64_t)b * NV + v] = ((sh[v][0] + sh[v][1]) + (sh[v][2] + sh[v][3])) * dV;
  }
}

__global__ void __launch_bounds__(256) final_sum_kernel(double* out, const double* partial,
                                                        int nblocks) {
  __shared__ double sh[NV][4];
  double acc[NV] = {0, 0, 0, 0, 0};
  for (int b = threadIdx.x; b < nblocks; b += 256)
#pragma unroll
    for (int v = 0; v < NV; ++v) acc[v] += partial[(int64_t)b * NV + v];
#pragma unroll
  for (int v = 0; v < NV; ++v) acc[v] = wave_sum(acc[v]);
  if ((threadIdx.x & 63) == 0)
#pragma unroll
    for (int v = 0; v < NV; ++v) sh[v][threadIdx.x >> 6] = acc[v];
  __syncthreads();
  if (threadIdx.x < NV) {
    const int v = threadIdx.x;
    out[v] = (sh[v][0] + sh[v][1]) + (sh[v][2] + sh[v][3]);
  }
}

template <typename S>
static hipError_t launch_totals_t(double* partial, double* out, const S* u, const BlockInfo* blocks,
                                  int32_t nblocks, const Geom& g, hipStream_t s) {
  hipLaunchKernelGGL(block_sum_kernel<S>, dim3(nblocks), dim3(256), 0, s, partial, u, blocks, g);
  hipLaunchKernelGGL(final_sum_kernel, dim3(1), dim3(256), 0, s, out, partial, nblocks);
  return hipGetLastError();
}
hipError_t launch_totals(double* partial, double* out, const double* u, const BlockInfo* blocks,
                         int32_t nblocks, const Geom& g, hipStream_t s) {
  return launch_totals_t(partial, out, u, blocks, nblocks, g, s);
}
hipError_t launch_totals(double* partial, double* out, const float* u, const BlockInfo* blocks,
                         int32_t nblocks, const Geom& g, hipStream_t s) {
  return launch_totals_t(partial, out, u, blocks, nblocks, g, s);
}

// Scratch of the totals for callers that cannot allocate: the per-leaf
// partial sums and the five results in a file-scope device array, one copy
// per GPU for the life of the process. Host code never passes the array's
// name to a kernel (on the host it is only a stand-in for the symbol): the
// device address of each GPU's copy is looked up once, with that GPU
// current, and kept per device.
static __device__ __align__(256) double scratch[(int64_t)TOTALS_SCRATCH_LEAVES * NV + 8];

namespace {
std::mutex g_scratch_mu;
double* g_scratch_ptr[64] = {};
}  // namespace

hipError_t totals_scratch(int device, double** ptr) {
  if (device < 0 || device >= 64) return hipErrorInvalidDevice;
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if (!g_scratch_ptr[device]) {
    int cur = -1;
    hipError_t e = hipGetDevice(&cur);
    if (e != hipSuccess) return e;
    if (cur != device && (e = hipSetDevice(device)) != hipSuccess) return e;
    void* p = nullptr;
    e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (cur != device) {
      const hipError_t e2 = hipSetDevice(cur);
      if (e == hipSuccess) e = e2;
    }
    if (e != hipSuccess) return e;
    g_scratch_ptr[device] = static_cast<double*>(p);
  }
  *ptr = g_scratch_ptr[device];
  return hipSuccess;
}

hipError_t launch_totals_scratch(const double* u, const BlockInfo* blocks, int32_t nblocks, const Geom& g,
                                 double* scr, hipStream_t s) {
  if (nblocks < 1 || nblocks > TOTALS_SCRATCH_LEAVES) return hipErrorInvalidValue;
  return launch_totals_t(scr, scr + (int64_t)TOTALS_SCRATCH_LEAVES * NV, u, blocks, nblocks, g, s);
}
hipError_t launch_totals_scratch(const float* u, const BlockInfo* blocks, int32_t nblocks, const Geom& g,
                                 double* scr, hipStream_t s) {
  if (nblocks < 1 || nblocks > TOTALS_SCRATCH_LEAVES) return hipErrorInvalidValue;
  return launch_totals_t(scr, scr + (int64_t)TOTALS_SCRATCH_LEAVES * NV, u, blocks, nblocks, g, s);
}

// ---------------------------------------------------------------------------
// Jump refinement indicator: per leaf, the largest relative jump
// |q(i+e_d) - q(i-e_d)| / (q(i+e_d) + q(i-e_d)) over active cells and
// directions, on the ghost-filled state, of q = pressure (quantity 0) or
// density (quantity 1). Evaluated without contraction and with correctly
// rounded division, so a threshold test on it decides the same way as the
// plain expression evaluated on a CPU.
// ---------------------------------------------------------------------------

__device__ double pressure_nc(const double* c, int64_t vs, double gm1) {
#pragma clang fp contract(off)
  const double rho = c[0], m1 = c[vs], m2 = c[2 * vs], m3 = c[3 * vs], e = c[4 * vs];
  const double ke = 0.5 * ((m1 * m1 + m2 * m2) + m3 * m3) / rho;
  return gm1 * (e - ke);
}

__global__ void __launch_bounds__(256) eta_kernel(double* eta, const double* u, const int32_t* nbr, Geom g,
                                                  int quantity) {
#pragma clang fp contract(off)
  __shared__ double sRed[4];
  const int b = blockIdx.x;
  const int ncell = g.n1 * g.n2 * g.n3;
  const double gm1 = g.gamma - 1.0;
  double mx = 0.0;
  for (int q = threadIdx.x; q < ncell; q += 256) {
    const int i = q % g.n1, j = (q / g.n1) % g.n2, k = q / (g.n1 * g.n2);
#pragma unroll
    for (int d = 0; d < 3; ++d) {
      // neighbours beyond the block: the face neighbour's active cells
      const int ip = i + (d == 0), jp = j + (d == 1), kp = k + (d == 2);
      const int im = i - (d == 0), jm = j - (d == 1), km = k - (d == 2);
      const double* cp = u + nb_index(g, nbr, b, ip, jp, kp);
      const double* cm = u + nb_index(g, nbr, b, im, jm, km);
      const double pp = quantity ? cp[0] : pressure_nc(cp, g.vstride, gm1);
      const double pm = quantity ? cm[0] : pressure_nc(cm, g.vstride, gm1);
      mx = fmax(mx, fabs(pp - pm) / (pp + pm));
    }
  }
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) mx = fmax(mx, __shfl_xor(mx, off));
  if ((threadIdx.x & 63) == 0) sRed[threadIdx.x >> 6] = mx;
  __syncthreads();
  if (threadIdx.x == 0) eta[b] = fmax(fmax(sRed[0], sRed[1]), fmax(sRed[2], sRed[3]));
}

// The same indicator with each cell's quantity evaluated once: the
// workgroup walks the block's z planes and keeps three planes of q (each
// with its one-cell x/y face ring) in LDS, so a cell's six neighbours are
// LDS reads instead of six evaluations from memory. The same expressions
// in the same order give the same bits as eta_kernel.
__device__ __forceinline__ double eta_q(const double* u, const int32_t* nbr, const Geom& g, int b, int i, int j,
                                        int k, int quantity, double gm1) {
  const double* c = u + nb_index(g, nbr, b, i, j, k);
  return quantity ? c[0] : pressure_nc(c, g.vstride, gm1);
}

__global__ void __launch_bounds__(256) eta_planes_kernel(double* eta, const double* u, const int32_t* nbr, Geom g,
                                                         int quantity) {
#pragma clang fp contract(off)
  extern __shared__ double sq[];  // 3 planes of (n1 + 2) x (n2 + 2)
  __shared__ double sRed[4];
  const int b = blockIdx.x;
  const int r1 = g.n1 + 2, pl = r1 * (g.n2 + 2);
  const int ring = 2 * g.n1 + 2 * g.n2;
  const double gm1 = g.gamma - 1.0;
  // q of plane k: its active cells, plus the x/y face ring when `ring` is
  // set (only the plane being evaluated needs it), into slot (k + 3) % 3
  auto fill = [&](int k, bool with_ring) {
    double* dst = sq + ((k + 3) % 3) * pl;
    const int ncell = g.n1 * g.n2 + (with_ring ? ring : 0);
    for (int q = threadIdx.x; q < ncell; q += 256) {
      int i, j;
      if (q < g.n1 * g.n2) {
        i = q % g.n1;
        j = q / g.n1;
      } else {
        const int r = q - g.n1 * g.n2;
        if (r < 2 * g.n1) {
          i = r % g.n1;
          j = r < g.n1 ? -1 : g.n2;
        } else {
          const int t = r - 2 * g.n1;
          j = t % g.n2;
          i = t < g.n2 ? -1 : g.n1;
        }
      }
      dst[(j + 1) * r1 + (i + 1)] = eta_q(u, nbr, g, b, i, j, k, quantity, gm1);
    }
  };
  fill(-1, false);
  fill(0, true);
  double mx = 0.0;
  for (int k = 0; k < g.n3; ++k) {
    fill(k + 1, k + 1 < g.n3);  // the ring of plane k + 1 is needed when it is evaluated
    __syncthreads();
    const double* qm = sq + ((k + 2) % 3) * pl;
    const double* q0 = sq + (k % 3) * pl;
    const double* qp = sq + ((k + 1) % 3) * pl;
    for (int q = threadIdx.x; q < g.n1 * g.n2; q += 256) {
      const int i = q % g.n1, j = q / g.n1;
      const int c = (j + 1) * r1 + (i + 1);
      const double px[3] = {q0[c + 1], q0[c + r1], qp[c]};
      const double pm[3] = {q0[c - 1], q0[c - r1], qm[c]};
#pragma unroll
      for (int d = 0; d < 3; ++d) mx = fmax(mx, fabs(px[d] - pm[d]) / (px[d] + pm[d]));
    }
    __syncthreads();  // plane k - 1's slot is refilled next
  }
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) mx = fmax(mx, __shfl_xor(mx, off));
  if ((threadIdx.x & 63) == 0) sRed[threadIdx.x >> 6] = mx;
  __syncthreads();
  if (threadIdx.x == 0) eta[b] = fmax(fmax(sRed[0], sRed[1]), fmax(sRed[2], sRed[3]));
}

hipError_t launch_eta(double* eta, const double* u, const int32_t* nbr, int32_t nblocks, const Geom& g,
                      int32_t quantity, hipStream_t s) {
  const size_t lds = 3 * sizeof(double) * (size_t)(g.n1 + 2) * (g.n2 + 2);
  if (lds <= 48 * 1024)
    hipLaunchKernelGGL(eta_planes_kernel, dim3(nblocks), dim3(256), lds, s, eta, u, nbr, g, (int)quantity);
  else
    hipLaunchKernelGGL(eta_kernel, dim3(nblocks), dim3(256), 0, s, eta, u, nbr, g, (int)quantity);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Regrid data: each new leaf is a copy, a child (prolongation of the
// composite field at the parent's level on the old mesh) or a merged parent
// (restriction of its children).
// ---------------------------------------------------------------------------

__global__ void __launch_bounds__(256) regrid_kernel(double* unew, const BlockInfo* bnew,
                                                     const int32_t* kind, const int32_t* src,
                                                     const double* uold, const BlockInfo* bold,
                                                     LevelMaps M, Geom g, DevTime* tm) {
  const int ncell = g.n1 * g.n2 * g.n3;
  const int r = blockIdx.y;
  const int q = blockIdx.x * blockDim.x + threadIdx.x;
  if (q >= ncell) return;
  const int i = q % g.n1, j = (q / g.n1) % g.n2, k = q / (g.n1 * g.n2);
  const BlockInfo bn = bnew[r];
  const int kd = kind[r], s = src[r];
  double* dst = unew + (int64_t)r * g.bstride + pad_index(g, i, j, k);
  const int J0 = bn.lx * g.n1 + i, J1 = bn.ly * g.n2 + j, J2 = bn.lz * g.n3 + k;
  int err = 0;
  double val[NV];
  if (kd == 0) {
#pragma unroll
    for (int v = 0; v < NV; ++v) val[v] = uold[(int64_t)s * g.bstride + v * g.vstride + pad_index(g, i, j, k)];
  } else if (kd == 1) {
    prolong_val(uold, bold, M, g, bn.level, J0, J1, J2, val, &err);
  } else {
    comp_val(uold, bold, M, g, bn.level, J0, J1, J2, val, &err);
  }
#pragma unroll
  for (int v = 0; v < NV; ++v) dst[v * g.vstride] = val[v];
  if (err) atomicOr(&tm->err, 2);
}

hipError_t launch_regrid_data(double* unew, const BlockInfo* bnew, const int32_t* kind,
                              const int32_t* src, int32_t nnew, const double* uold,
                              const BlockInfo* bold, const LevelMaps& old_maps, const Geom& g,
                              DevTime* tm, hipStream_t s) {
  const int ncell = g.n1 * g.n2 * g.n3;
  dim3 grid((ncell + 255) / 256, nnew);
  hipLaunchKernelGGL(regrid_kernel, grid, dim3(256), 0, s, unew, bnew, kind, src, uold, bold,
                     old_maps, g, tm);
  return hipGetLastError();
}

}  // namespace pkh

// ===========================================================================
// Reverse mode of one stage, U_out = U_base - c * D(U_in), w.r.t. U_in
// (the identity through U_base is added by the caller): with
// lam = dL/dU_out, the face adjoint of face f along d is
// mu_f = c/dx_d * (lam(f) - lam(f-1)) (only the block's own active cells),
// propagated back through HLLE, the face reconstruction and the primitive
// recovery to the cells of the face stencil, including ghost cells; the
// ghost contributions are then returned to the leaves they were copied
// from (the transpose of the same-level ghost exchange).
// ===========================================================================

namespace pkh {

// One thread per pencil (active transverse position) of a block along D;
// it walks the pencil's padded cells with a window of states and a ring of
// four cell accumulators, so each cell's primitive adjoint is complete when
// emitted. Each direction writes its own array (every padded cell of its
// pencils), so the three directions run in one launch.
template <int RECON, int D>
__device__ __forceinline__ void adj_pencil(const double* __restrict__ U, const double* __restrict__ lam,
                                           double* __restrict__ wbar, const BlockInfo* blocks,
                                           const int32_t* __restrict__ nbr, int nblocks, const Geom& g,
                                           const double* dtp, double beta, int64_t gid) {
  const int n[3] = {g.n1, g.n2, g.n3};
  constexpr int T1 = D == 0 ? 1 : 0, T2 = D == 2 ? 1 : 2;
  const int nt1 = n[T1], nt2 = n[T2], nd = n[D];
  const int64_t per = (int64_t)nt1 * nt2;
  const int b = (int)(gid / per);
  if (b >= nblocks) return;
  const int rem = (int)(gid - (int64_t)b * per);
  const int a1 = rem % nt1, a2 = rem / nt1;
  const BlockInfo bi = blocks[b];
  const double gam = g.gamma, gm1 = gam - 1.0, igm1 = 1.0 / gm1;
  const double coef = beta * (*dtp) * bi.idx[D];
  const int pst[3] = {1, g.p1, g.p1 * g.p2};  // padded strides
  const int ast[3] = {1, g.n1, g.n1 * g.n2};  // active strides
  int c3[3];
  c3[T1] = a1;
  c3[T2] = a2;
  c3[D] = 0;
  const int64_t pbase = (int64_t)b * g.bstride + ((int64_t)(c3[2] + NG) * g.p2 + (c3[1] + NG)) * g.p1 +
                        (c3[0] + NG);  // padded index of the pencil's cell 0
  const int64_t ncell = (int64_t)g.n1 * g.n2 * g.n3;
  const int64_t abase = (int64_t)b * NV * ncell + (int64_t)c3[2] * ast[2] + (int64_t)c3[1] * ast[1] + c3[0];
  const int ps = pst[D], as = ast[D];

  auto loadu = [&](int s, double u[NV]) {
    int64_t at = pbase + (int64_t)s * ps;
    if (s < 0 || s >= nd) {
      int cc[3] = {c3[0], c3[1], c3[2]};
      cc[D] = s;
      at = nb_index(g, nbr, b, cc[0], cc[1], cc[2]);
    }
#pragma unroll
    for (int v = 0; v < NV; ++v) u[v] = U[at + (int64_t)v * g.vstride];
  };
  auto loadl = [&](int s, double l[NV]) {
#pragma unroll
    for (int v = 0; v < NV; ++v) l[v] = (s >= 0 && s < nd) ? lam[abase + (int64_t)v * ncell + (int64_t)s * as] : 0.0;
  };
  auto emit = [&](int s, const double acc[NV]) {
    double* o = wbar + pbase + (int64_t)s * ps;
#pragma unroll
    for (int v = 0; v < NV; ++v) o[(int64_t)v * g.vstride] = acc[v];
  };
  // face f lies between cells f-1 and f; its flux enters cell f-1 with +coef
  // and cell f with -coef, so its adjoint is coef * (lam(f) - lam(f-1))
  double un[NV], lp[NV], ln[NV];
  const double zero5[NV] = {0, 0, 0, 0, 0};

  if constexpr (!RECON) {
    // donor cell: the face states are the cell states, so each cell's
    // derived state is formed once and its adjoint reversed once, after both
    // of its faces have been swept
    FState Qa, Qb;
    double gQa[8], gQb[8];
    auto state_of = [&](const double u[NV], FState& q) {
      double w[NV];
      to_prim(u, gam, w);
      q = FState{w[0], w[1], w[2], w[3], w[4], 0, 0, 0};
      complete_state(q, gam, igm1);
    };
    loadu(-1, un);
    state_of(un, Qa);
    loadu(0, un);
    state_of(un, Qb);
    loadu(1, un);  // next cell, one iteration ahead
    loadl(-1, lp);
    loadl(0, ln);
#pragma unroll
    for (int k = 0; k < 8; ++k) gQa[k] = gQb[k] = 0.0;
    emit(-2, zero5);
    for (int f = 0; f <= nd; ++f) {
      double mu[NV];
#pragma unroll
      for (int v = 0; v < NV; ++v) mu[v] = coef * (ln[v] - lp[v]);
#pragma unroll
      for (int v = 0; v < NV; ++v) lp[v] = ln[v];
      loadl(f + 1, ln);
      hlle_rev<D>(Qa, Qb, gm1, mu, gQa, gQb);
      double gw[NV] = {0, 0, 0, 0, 0};
      complete_state_rev(Qa, gam, igm1, gQa, gw);
      emit(f - 1, gw);
      if (f < nd) {
        Qa = Qb;
#pragma unroll
        for (int k = 0; k < 8; ++k) {
          gQa[k] = gQb[k];
          gQb[k] = 0.0;
        }
        state_of(un, Qb);
        if (f + 2 <= nd) loadu(f + 2, un);
      }
    }
    double gw[NV] = {0, 0, 0, 0, 0};
    complete_state_rev(Qb, gam, igm1, gQb, gw);
    emit(nd, gw);
    emit(nd + 1, zero5);
  } else {
    // PLM: window of primitives of cells f-1, f, f+1; the limited slope of
    // each cell and its branch derivatives are formed once, when the cell's
    // right neighbour arrives, and used by both faces of the cell
    double W0[NV], W1[NV], W2[NV];  // cells f-1, f, f+1
    double Sp[NV], Gap[NV], Gbp[NV];  // slope of cell f-1 and d slope / d (dl, dr)
    double acc0[NV], acc1[NV], acc2[NV], acc3[NV];  // cells f-2 .. f+1
    {
      double Wm[NV];
      loadu(-2, un);
      to_prim(un, gam, Wm);
      loadu(-1, un);
      to_prim(un, gam, W1);
      loadu(0, un);
      to_prim(un, gam, W2);
#pragma unroll
      for (int v = 0; v < NV; ++v) {
        const double dl = W1[v] - Wm[v], dr = W2[v] - W1[v];
        Sp[v] = mc_slope(dl, dr);
        mc_branch(dl, dr, Gap[v], Gbp[v]);
      }
    }
    loadu(1, un);
    loadl(-1, lp);
    loadl(0, ln);
#pragma unroll
    for (int v = 0; v < NV; ++v) acc0[v] = acc1[v] = acc2[v] = acc3[v] = 0.0;
    for (int f = 0; f <= nd; ++f) {
#pragma unroll
      for (int v = 0; v < NV; ++v) {
        W0[v] = W1[v];
        W1[v] = W2[v];
      }
      to_prim(un, gam, W2);
      if (f + 2 <= nd + 1) loadu(f + 2, un);
      double mu[NV];
#pragma unroll
      for (int v = 0; v < NV; ++v) mu[v] = coef * (ln[v] - lp[v]);
#pragma unroll
      for (int v = 0; v < NV; ++v) lp[v] = ln[v];
      loadl(f + 1, ln);
      double Sc[NV], Gac[NV], Gbc[NV];
      double wl[NV], wr[NV];
#pragma unroll
      for (int v = 0; v < NV; ++v) {
        const double dl = W1[v] - W0[v], dr = W2[v] - W1[v];
        Sc[v] = mc_slope(dl, dr);
        mc_branch(dl, dr, Gac[v], Gbc[v]);
        wl[v] = W0[v] + 0.5 * Sp[v];
        wr[v] = W1[v] - 0.5 * Sc[v];
      }
      FState L{wl[0], wl[1], wl[2], wl[3], wl[4], 0, 0, 0};
      FState R{wr[0], wr[1], wr[2], wr[3], wr[4], 0, 0, 0};
      complete_state(L, gam, igm1);
      complete_state(R, gam, igm1);
      double gL[8] = {0, 0, 0, 0, 0, 0, 0, 0}, gR[8] = {0, 0, 0, 0, 0, 0, 0, 0};
      hlle_rev<D>(L, R, gm1, mu, gL, gR);
      double gl[NV] = {0, 0, 0, 0, 0}, gr[NV] = {0, 0, 0, 0, 0};
      complete_state_rev(L, gam, igm1, gL, gl);
      complete_state_rev(R, gam, igm1, gR, gr);
#pragma unroll
      for (int v = 0; v < NV; ++v) {
        // wl = W(f-1) + s(f-1)/2, s(f-1) = MC(W(f-1) - W(f-2), W(f) - W(f-1))
        acc0[v] -= gl[v] * 0.5 * Gap[v];
        acc1[v] += gl[v] * (1.0 + 0.5 * Gap[v] - 0.5 * Gbp[v]);
        acc2[v] += gl[v] * 0.5 * Gbp[v];
        // wr = W(f) - s(f)/2, s(f) = MC(W(f) - W(f-1), W(f+1) - W(f))
        acc1[v] += gr[v] * 0.5 * Gac[v];
        acc2[v] += gr[v] * (1.0 - 0.5 * Gac[v] + 0.5 * Gbc[v]);
        acc3[v] -= gr[v] * 0.5 * Gbc[v];
        Sp[v] = Sc[v];
        Gap[v] = Gac[v];
        Gbp[v] = Gbc[v];
      }
      emit(f - 2, acc0);
#pragma unroll
      for (int v = 0; v < NV; ++v) {
        acc0[v] = acc1[v];
        acc1[v] = acc2[v];
        acc2[v] = acc3[v];
        acc3[v] = 0.0;
      }
    }
    emit(nd - 1, acc0);
    emit(nd, acc1);
    emit(nd + 1, acc2);
  }
}

// ---------------------------------------------------------------------------
// x direction of the reverse sweep and the closing of each cell, one pass
// face-parallel along rows. A pencil walk along x would put every lane of a
// wave on a different row of the contiguous dimension; here lane i of an
// n1-wide lane segment owns cell i of one row and the face below it (face
// i, between cells i-1 and i), so loads and stores are coalesced. Neighbour
// states and the contributions a face makes to cells i-2 .. i+1 move between
// lanes by shuffles within the segment. Everything that crosses a block's x
// face - the face itself (with the face adjoints of both blocks combined)
// and the parts of the two faces beside it that reach across - is computed
// once per boundary row beforehand, alongside the y and z pencils, into a
// side buffer of 20 doubles per row. The row pass then completes each cell:
// its x part, the side-buffer part, its y and z parts and those of its
// ghost copies in the y and z neighbours, the primitive-to-conserved
// adjoint at its state, and the identity terms of the cycle.
// ---------------------------------------------------------------------------

// Side-buffer slot q of row `row` (slot-major, rows fastest). For the x
// face between the row of block X and the same row of its x-upper
// neighbour R, indexed by X's row: slots 0, 1 hold the parts for X's cells
// n1-2, n1-1, slots 2, 3 those for R's cells 0, 1.
__device__ __forceinline__ int64_t xside_at(int64_t nrows, int q, int64_t row) {
  return (int64_t)q * nrows + row;
}

// Adjoint of one PLM face normal to D from the primitives of cells f-2 ..
// f+1 (Wa .. Wd) and the face adjoint mu: the parts c0 .. c3 of the four
// cells' primitive adjoints.
template <int D>
__device__ __forceinline__ void plm_face_rev(const double Wa[NV], const double Wb[NV], const double Wc[NV],
                                             const double Wd[NV], const double mu[NV], double gam,
                                             double c0[NV], double c1[NV], double c2[NV], double c3[NV]) {
  const double gm1 = gam - 1.0, igm1 = 1.0 / gm1;
  double ga0[NV], gb0[NV], ga1[NV], gb1[NV], wl[NV], wr[NV];
#pragma unroll
  for (int v = 0; v < NV; ++v) {
    const double s0 = mc_slope(Wb[v] - Wa[v], Wc[v] - Wb[v]);
    mc_branch(Wb[v] - Wa[v], Wc[v] - Wb[v], ga0[v], gb0[v]);
    const double s1 = mc_slope(Wc[v] - Wb[v], Wd[v] - Wc[v]);
    mc_branch(Wc[v] - Wb[v], Wd[v] - Wc[v], ga1[v], gb1[v]);
    wl[v] = Wb[v] + 0.5 * s0;
    wr[v] = Wc[v] - 0.5 * s1;
  }
  FState L{wl[0], wl[1], wl[2], wl[3], wl[4], 0, 0, 0};
  FState R{wr[0], wr[1], wr[2], wr[3], wr[4], 0, 0, 0};
  complete_state(L, gam, igm1);
  complete_state(R, gam, igm1);
  double gL[8] = {0, 0, 0, 0, 0, 0, 0, 0}, gR[8] = {0, 0, 0, 0, 0, 0, 0, 0};
  hlle_rev<D>(L, R, gm1, mu, gL, gR);
  double gl[NV] = {0, 0, 0, 0, 0}, gr[NV] = {0, 0, 0, 0, 0};
  complete_state_rev(L, gam, igm1, gL, gl);
  complete_state_rev(R, gam, igm1, gR, gr);
#pragma unroll
  for (int v = 0; v < NV; ++v) {
    c0[v] = -gl[v] * 0.5 * ga0[v];
    c1[v] = gl[v] * (1.0 + 0.5 * ga0[v] - 0.5 * gb0[v]) + gr[v] * 0.5 * ga1[v];
    c2[v] = gl[v] * 0.5 * gb0[v] + gr[v] * (1.0 - 0.5 * ga1[v] + 0.5 * gb1[v]);
    c3[v] = -gr[v] * 0.5 * gb1[v];
  }
}

// The crossing parts at the x face above row `row` of block X (cells n1-1 |
// 0 of X and R). PLM: the face itself with both face adjoints, the k3 part
// of X's face n1-1 and the k0 part of R's face 1. Donor cell: the face
// itself.
template <int RECON>
__device__ __forceinline__ void adj_xside(const double* __restrict__ U, const double* __restrict__ lam,
                                          double* __restrict__ xl, const BlockInfo* blocks,
                                          const int32_t* __restrict__ nbr, int nblocks, const Geom& g,
                                          const double* dtp, double beta, int64_t row) {
  const int64_t rpb = (int64_t)g.n2 * g.n3;
  const int64_t nrows = rpb * nblocks;
  if (row >= nrows) return;
  const int b = (int)(row / rpb);
  const int r = (int)(row - (int64_t)b * rpb);
  const int j = r % g.n2, k = r / g.n2;
  const int nd = g.n1;
  const int32_t rb = nbr[(int64_t)b * 27 + 14];
  if (rb < 0) {  // a face to another level: not part of a single-level sweep
#pragma unroll
    for (int q = 0; q < 4 * NV; ++q) xl[xside_at(nrows, q, row)] = 0.0;
    return;
  }
  const double gam = g.gamma, gm1 = gam - 1.0, igm1 = 1.0 / gm1;
  const double coef = beta * (*dtp) * blocks[b].idx[0];
  const int64_t ncell = (int64_t)g.n1 * g.n2 * g.n3;
  const int64_t lx = (int64_t)b * NV * ncell + ((int64_t)k * g.n2 + j) * g.n1;
  const int64_t lr = (int64_t)rb * NV * ncell + ((int64_t)k * g.n2 + j) * g.n1;
  auto loadw = [&](int s, double w[NV]) {
    const int64_t at = nb_index(g, nbr, b, s, j, k);
    double u[NV];
#pragma unroll
    for (int v = 0; v < NV; ++v) u[v] = U[at + (int64_t)v * g.vstride];
    to_prim(u, gam, w);
  };
  double muB[NV];
#pragma unroll
  for (int v = 0; v < NV; ++v) muB[v] = coef * (lam[lr + (int64_t)v * ncell] - lam[lx + (int64_t)v * ncell + nd - 1]);
  double o0[NV], o1[NV], o2[NV], o3[NV];
  if constexpr (RECON) {
    double W0[NV], W1[NV], W2[NV], W3[NV], W4[NV], W5[NV];  // cells n1-3 .. n1+2
    loadw(nd - 3, W0);
    loadw(nd - 2, W1);
    loadw(nd - 1, W2);
    loadw(nd, W3);
    loadw(nd + 1, W4);
    loadw(nd + 2, W5);
    double muA[NV], muC[NV], t0[NV], t1[NV], t2[NV], t3[NV];
#pragma unroll
    for (int v = 0; v < NV; ++v) {
      muA[v] = coef * (lam[lx + (int64_t)v * ncell + nd - 1] - lam[lx + (int64_t)v * ncell + nd - 2]);
      muC[v] = coef * (lam[lr + (int64_t)v * ncell + 1] - lam[lr + (int64_t)v * ncell]);
    }
    plm_face_rev<0>(W1, W2, W3, W4, muB, gam, o0, o1, o2, o3);
    plm_face_rev<0>(W0, W1, W2, W3, muA, gam, t0, t1, t2, t3);
#pragma unroll
    for (int v = 0; v < NV; ++v) o2[v] += t3[v];  // X's face n1-1 -> R's cell 0
    plm_face_rev<0>(W2, W3, W4, W5, muC, gam, t0, t1, t2, t3);
#pragma unroll
    for (int v = 0; v < NV; ++v) o1[v] += t0[v];  // R's face 1 -> X's cell n1-1
  } else {
    double wa[NV], wb[NV];
    loadw(nd - 1, wa);
    loadw(nd, wb);
    FState Qa{wa[0], wa[1], wa[2], wa[3], wa[4], 0, 0, 0};
    FState Qb{wb[0], wb[1], wb[2], wb[3], wb[4], 0, 0, 0};
    complete_state(Qa, gam, igm1);
    complete_state(Qb, gam, igm1);
    double gL[8] = {0, 0, 0, 0, 0, 0, 0, 0}, gR[8] = {0, 0, 0, 0, 0, 0, 0, 0};
    hlle_rev<0>(Qa, Qb, gm1, muB, gL, gR);
#pragma unroll
    for (int v = 0; v < NV; ++v) o0[v] = o1[v] = o2[v] = o3[v] = 0.0;
    // the reverse of the derived state is linear in its adjoint, so the
    // face's parts of the two cells are reversed here on their own
    complete_state_rev(Qa, gam, igm1, gL, o1);
    complete_state_rev(Qb, gam, igm1, gR, o2);
  }
#pragma unroll
  for (int v = 0; v < NV; ++v) {
    xl[xside_at(nrows, 0 * NV + v, row)] = o0[v];
    xl[xside_at(nrows, 1 * NV + v, row)] = o1[v];
    xl[xside_at(nrows, 2 * NV + v, row)] = o2[v];
    xl[xside_at(nrows, 3 * NV + v, row)] = o3[v];
  }
}

// Lane shuffles within segments of W lanes (one row each); a lane whose
// source falls outside its segment gets its own value back.
template <int W>
__device__ __forceinline__ double shup(double x, int d) {
  return __shfl_up(x, d, W);
}
template <int W>
__device__ __forceinline__ double shdn(double x, int d) {
  return __shfl_down(x, d, W);
}

// The row pass. out = add0 + add1 + (dD/dU_in)^T-term of lam at every
// active cell (add0, add1 may be null); wyz: the y and z primitive-adjoint
// arrays (padded, wstride apart); xl: the side buffer.
template <int RECON, int N1>
__global__ void __launch_bounds__(256) adj_xrow_kernel(const double* __restrict__ U,
                                                       const double* __restrict__ lam,
                                                       const double* __restrict__ wyz, int64_t wstride,
                                                       const double* __restrict__ xl,
                                                       const BlockInfo* blocks,
                                                       const int32_t* __restrict__ nbr, int nblocks, Geom g,
                                                       const double* dtp, double beta, double* __restrict__ out,
                                                       const double* __restrict__ add0,
                                                       const double* __restrict__ add1) {
  static_assert(N1 == 8 || N1 == 16 || N1 == 32 || N1 == 64, "row width");
  const int i = (int)(threadIdx.x % N1);
  const int64_t row = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) / N1;
  const int64_t rpb = (int64_t)g.n2 * g.n3;
  const int64_t nrows = rpb * nblocks;
  // every lane of a segment shares the row, so whole segments leave together
  if (row >= nrows) return;
  const int b = (int)(row / rpb);
  const int r = (int)(row - (int64_t)b * rpb);
  const int j = r % g.n2, k = r / g.n2;
  const double gam = g.gamma, gm1 = gam - 1.0, igm1 = 1.0 / gm1;
  const double coef = beta * (*dtp) * blocks[b].idx[0];
  const int64_t pbase = (int64_t)b * g.bstride + ((int64_t)(k + NG) * g.p2 + (j + NG)) * g.p1 + NG;
  const int64_t ncell = (int64_t)g.n1 * g.n2 * g.n3;
  const int64_t abase = (int64_t)b * NV * ncell + ((int64_t)k * g.n2 + j) * g.n1;
  const int32_t* nb27 = nbr + (int64_t)b * 27;
  auto loadu = [&](int s, double u[NV]) {
    const int64_t at = (s >= 0 && s < N1) ? pbase + s : nb_index(g, nbr, b, s, j, k);
#pragma unroll
    for (int v = 0; v < NV; ++v) u[v] = U[at + (int64_t)v * g.vstride];
  };
  // face i adjoint: coef * (lam(i) - lam(i-1)); face 0 crosses the block's
  // x face and is left to the side buffer (mu = 0 here)
  double mu[NV];
#pragma unroll
  for (int v = 0; v < NV; ++v) {
    const double l0 = lam[abase + (int64_t)v * ncell + i];
    const double lm = shup<N1>(l0, 1);
    mu[v] = i > 0 ? coef * (l0 - lm) : 0.0;
  }
  const bool first = i == 0, last = i == N1 - 1;
  double uown[NV], gw[NV];
  loadu(i, uown);

  if constexpr (RECON) {
    // own cell, and the cell beyond the segment an edge lane needs for the
    // states of its face: lane 0 cell -2, lane 1 cell -1, last lane cell n1
    double W[NV], Wx[NV], ux[NV];
    to_prim(uown, gam, W);
    loadu(i == 0 ? -2 : (i == 1 ? -1 : N1), ux);
    to_prim(ux, gam, Wx);
    double Wm1[NV], Wm2[NV], Wp1[NV];
#pragma unroll
    for (int v = 0; v < NV; ++v) {
      const double a1 = shup<N1>(W[v], 1), a2 = shup<N1>(W[v], 2), p1 = shdn<N1>(W[v], 1);
      const double gm = shdn<N1>(Wx[v], 1);  // lane 0 <- lane 1's cell -1
      Wm1[v] = first ? gm : a1;
      Wm2[v] = first ? Wx[v] : (i == 1 ? Wx[v] : a2);
      Wp1[v] = last ? Wx[v] : p1;
    }
    double c0[NV], c1[NV], c2[NV], c3[NV];
    plm_face_rev<0>(Wm2, Wm1, W, Wp1, mu, gam, c0, c1, c2, c3);
    // the in-block parts of cell i: faces i-1 .. i+2 of this row; the
    // parts reaching across a block face are in the side buffer
#pragma unroll
    for (int v = 0; v < NV; ++v) {
      const double f1 = shdn<N1>(c1[v], 1), f0 = shdn<N1>(c0[v], 2), b3 = shup<N1>(c3[v], 1);
      double a = c2[v] + (first ? 0.0 : b3);
      a += last ? 0.0 : f1;
      a += (i >= N1 - 2) ? 0.0 : f0;
      gw[v] = a;
    }
  } else {
    // donor cell: face i joins cells i-1 and i
    double W[NV];
    to_prim(uown, gam, W);
    FState Q{W[0], W[1], W[2], W[3], W[4], 0, 0, 0};
    complete_state(Q, gam, igm1);
    const FState Qm{shup<N1>(Q.r, 1),  shup<N1>(Q.v0, 1), shup<N1>(Q.v1, 1), shup<N1>(Q.v2, 1),
                    shup<N1>(Q.p, 1),  shup<N1>(Q.sr, 1), shup<N1>(Q.c, 1),  shup<N1>(Q.h, 1)};
    double gL[8] = {0, 0, 0, 0, 0, 0, 0, 0}, gR[8] = {0, 0, 0, 0, 0, 0, 0, 0};
    hlle_rev<0>(Qm, Q, gm1, mu, gL, gR);  // lane 0: mu = 0 (its Qm is its own state)
    double gQ[8];
#pragma unroll
    for (int q = 0; q < 8; ++q) {
      const double nb = shdn<N1>(gL[q], 1);
      gQ[q] = gR[q] + (last ? 0.0 : nb);
    }
#pragma unroll
    for (int v = 0; v < NV; ++v) gw[v] = 0.0;
    complete_state_rev(Q, gam, igm1, gQ, gw);
  }
  // parts across the block's x faces
  if (i >= N1 - 2) {
#pragma unroll
    for (int v = 0; v < NV; ++v) gw[v] += xl[xside_at(nrows, (i - (N1 - 2)) * NV + v, row)];
  }
  if (i < 2 && nb27[12] >= 0) {
    const int64_t lrow = (int64_t)nb27[12] * rpb + r;
#pragma unroll
    for (int v = 0; v < NV; ++v) gw[v] += xl[xside_at(nrows, (2 + i) * NV + v, lrow)];
  }
  // y and z parts of the cell and of its ghost copies in the y and z neighbours
  const int64_t own = pbase + i;
#pragma unroll
  for (int v = 0; v < NV; ++v)
    gw[v] += wyz[own + (int64_t)v * g.vstride] + wyz[wstride + own + (int64_t)v * g.vstride];
  auto add_copy = [&](int dy, int dz) {
    const int32_t nb = nb27[(dz + 1) * 9 + (dy + 1) * 3 + 1];
    if (nb < 0) return;
    const double* wd = wyz + (dy ? 0 : wstride);
    const int64_t o = (int64_t)nb * g.bstride + pad_index(g, i, j - dy * g.n2, k - dz * g.n3);
#pragma unroll
    for (int v = 0; v < NV; ++v) gw[v] += wd[o + (int64_t)v * g.vstride];
  };
  if (j < NG) add_copy(-1, 0);
  if (j >= g.n2 - NG) add_copy(1, 0);
  if (k < NG) add_copy(0, -1);
  if (k >= g.n3 - NG) add_copy(0, 1);
  double gu[NV];
  prim_rev(uown, gam, gw, gu);
  const int64_t ao = abase + i;
#pragma unroll
  for (int v = 0; v < NV; ++v) {
    double o = gu[v];
    if (add0) o += add0[ao + (int64_t)v * ncell];
    if (add1) o += add1[ao + (int64_t)v * ncell];
    out[ao + (int64_t)v * ncell] = o;
  }
}

// One launch for the y and z pencils (blockIdx.y = 0, 1); the x-face side
// buffer in a launch of its own, whose register demand (beyond 256 VGPRs)
// would otherwise hold the pencils to one wave per SIMD.
template <int RECON>
__global__ void __launch_bounds__(256, PKH_ADJ_PENCIL_WAVES) adj_pencils_kernel(const double* __restrict__ U,
                                                          const double* __restrict__ lam,
                                                          double* __restrict__ wyz, int64_t wstride,
                                                          const BlockInfo* blocks, const int32_t* nbr, int nblocks,
                                                          Geom g, const double* dtp, double beta) {
  const int64_t gid = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (blockIdx.y == 0)
    adj_pencil<RECON, 1>(U, lam, wyz, blocks, nbr, nblocks, g, dtp, beta, gid);
  else
    adj_pencil<RECON, 2>(U, lam, wyz + wstride, blocks, nbr, nblocks, g, dtp, beta, gid);
}

template <int RECON>
__global__ void __launch_bounds__(256) adj_xside_kernel(const double* __restrict__ U,
                                                        const double* __restrict__ lam, double* __restrict__ xl,
                                                        const BlockInfo* blocks, const int32_t* nbr, int nblocks,
                                                        Geom g, const double* dtp, double beta) {
  const int64_t gid = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  adj_xside<RECON>(U, lam, xl, blocks, nbr, nblocks, g, dtp, beta, gid);
}

template <int RECON>
static void launch_xrow(int n1, dim3 grid, hipStream_t s, const double* U, const double* lam, const double* wyz,
                        int64_t wstride, const double* xl, const BlockInfo* blocks, const int32_t* nbr,
                        int nblocks, const Geom& g, const double* dtp, double beta, double* out,
                        const double* add0, const double* add1) {
#define PKH_XROW(N)                                                                                            \
  hipLaunchKernelGGL((adj_xrow_kernel<RECON, N>), grid, dim3(256), 0, s, U, lam, wyz, wstride, xl, blocks, nbr, \
                     nblocks, g, dtp, beta, out, add0, add1)
  switch (n1) {
    case 8:
      PKH_XROW(8);
      break;
    case 16:
      PKH_XROW(16);
      break;
    case 32:
      PKH_XROW(32);
      break;
    default:
      PKH_XROW(64);
  }
#undef PKH_XROW
}

bool adj_xrow_supported(int n1) { return n1 == 8 || n1 == 16 || n1 == 32 || n1 == 64; }

hipError_t launch_adj_stage(int recon, const double* U, const double* lam, double* wyz, double* xside,
                            const BlockInfo* blocks, int32_t nblocks, const Geom& g,
                            const int32_t* nbr, const double* dtp, double beta, double* out,
                            const double* add0, const double* add1, hipStream_t s) {
  // y and z pencils with the x-face side buffer, then the rows (x and the
  // closing of every cell)
  if (!adj_xrow_supported(g.n1) || xside == nullptr) return hipErrorInvalidValue;
  const int64_t nrows = (int64_t)nblocks * g.n2 * g.n3;
  const int64_t npen = std::max(std::max((int64_t)nblocks * g.n1 * g.n3, (int64_t)nblocks * g.n1 * g.n2), nrows);
  const int64_t wstride = (int64_t)nblocks * g.bstride;
  const dim3 gr((unsigned)((nrows * g.n1 + 255) / 256)), gp((unsigned)((npen + 255) / 256), 2),
      gx((unsigned)((npen + 255) / 256));
  if (recon) {
    hipLaunchKernelGGL(adj_pencils_kernel<1>, gp, dim3(256), 0, s, U, lam, wyz, wstride, blocks, nbr, nblocks, g,
                       dtp, beta);
    hipLaunchKernelGGL(adj_xside_kernel<1>, gx, dim3(256), 0, s, U, lam, xside, blocks, nbr, nblocks, g, dtp, beta);
    launch_xrow<1>(g.n1, gr, s, U, lam, wyz, wstride, xside, blocks, nbr, nblocks, g, dtp, beta, out, add0, add1);
  } else {
    hipLaunchKernelGGL(adj_pencils_kernel<0>, gp, dim3(256), 0, s, U, lam, wyz, wstride, blocks, nbr, nblocks, g,
                       dtp, beta);
    hipLaunchKernelGGL(adj_xside_kernel<0>, gx, dim3(256), 0, s, U, lam, xside, blocks, nbr, nblocks, g, dtp, beta);
    launch_xrow<0>(g.n1, gr, s, U, lam, wyz, wstride, xside, blocks, nbr, nblocks, g, dtp, beta, out, add0, add1);
  }
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Face-wise reverse mode of one stage, for meshes with level jumps or walls
// (also valid on single-level meshes): U_out = U_base - beta dt D(U_in) with
// the fine-coarse flux correction of every stage, differentiated w.r.t. the
// active cells of U_in through the ghost faces the stage reads.
//  1. Each face whose flux enters some update gets its adjoint
//     mu = beta dt (lam_up w_up / dx_up - lam_lo w_lo / dx_lo); a coarse
//     cell beside finer leaves sees each fine sub-face with weight 1/4 (its
//     own flux there is replaced, so it gets none). The face is handled by
//     the leaf on its fine side, by the lower leaf of a same-level pair, and
//     by the leaf itself at a wall.
//  2. mu goes back through HLLE (frozen wave-speed cases), the face states
//     (frozen MC cases) and the primitive recovery to the stencil cells:
//     atomically added into a padded primitive-adjoint array, cells beyond a
//     same-level face into the neighbour's active cells, cells beyond a
//     level jump or wall into the leaf's own ghost zone.
//  3. Primitive adjoints become conserved ones at the forward states.
//  4. Every ghost-zone adjoint moves to the active cells its forward value
//     came from: the image cell at a wall; 1/8 to each of 8 fine cells for a
//     restriction; for a prolongation the transposed linear map with the
//     forward's minmod cases, onto the composite coarse field (coarse leaf
//     cells, or 1/8 to each fine cell of a restricted composite value).
//  5. out = add0 + add1 + the active-cell adjoints.
// ---------------------------------------------------------------------------

// Neighbour kind across face f of leaf bi: 0 same level, 1 coarser, 2 finer,
// 3 wall.
__device__ __forceinline__ int face_kind(const BlockInfo& bi, const int32_t* nb27, const Geom& g, int f) {
  const int d = f >> 1, s = f & 1;
  if (g.bc[2 * d] != BC_PERIODIC) {
    const int lo = d == 0 ? bi.lx : (d == 1 ? bi.ly : bi.lz);
    if ((s == 0 && lo == 0) || (s == 1 && lo == (g.nrb[d] << bi.level) - 1)) return 3;
  }
  const int q = (d == 2 ? (s ? 2 : 0) : 1) * 9 + (d == 1 ? (s ? 2 : 0) : 1) * 3 + (d == 0 ? (s ? 2 : 0) : 1);
  if (nb27[q] >= 0) return 0;
  if ((bi.finer_mask >> f) & 1) return 2;
  return 1;
}

// lam of the coarse cell beside fine leaf bi (level L >= 1) across its face
// along d on side s, at the fine cell's transverse position c (leaf
// coordinates, c[d] the fine cell next to the face); writes the coarse
// leaf's 1/dx_d to *idd. False if no coarse leaf covers it.
__device__ bool coarse_lam(const double* lam, const BlockInfo* blocks, const LevelMaps& M, const Geom& g,
                           const BlockInfo& bi, int d, int s, const int c[3], double out[NV], double* idd) {
  const int n[3] = {g.n1, g.n2, g.n3};
  const int lo[3] = {bi.lx, bi.ly, bi.lz};
  int J[3];
#pragma unroll
  for (int e = 0; e < 3; ++e) J[e] = lo[e] * n[e] + c[e] + (e == d ? (s ? 1 : -1) : 0);
  const int L = bi.level;
#pragma unroll
  for (int e = 0; e < 3; ++e) J[e] = wrap_i(J[e], (g.nrb[e] * n[e]) << L) >> 1;
  const int32_t id = leaf_at(M, L - 1, J[0] / n[0], J[1] / n[1], J[2] / n[2]);
  if (id < 0) return false;
  const BlockInfo bc = blocks[id];
  const int64_t cs = (int64_t)n[0] * n[1] * n[2];
  const int64_t o = (int64_t)id * NV * cs + ((int64_t)(J[2] - bc.lz * n[2]) * n[1] + (J[1] - bc.ly * n[1])) * n[0] +
                    (J[0] - bc.lx * n[0]);
#pragma unroll
  for (int v = 0; v < NV; ++v) out[v] = lam[o + v * cs];
  *idd = d == 0 ? bc.idx[0] : (d == 1 ? bc.idx[1] : bc.idx[2]);
  return true;
}

template <int RECON>
__global__ void __launch_bounds__(256) adjf_face_kernel(const double* __restrict__ U, const double* __restrict__ lam,
                                                        double* gw, const BlockInfo* blocks, const int32_t* nbr,
                                                        LevelMaps M, Geom g, const double* dtp, double beta,
                                                        int64_t nfaces, DevTime* tm) {
  const int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (q >= nfaces) return;
  const int n[3] = {g.n1, g.n2, g.n3};
  const int64_t fx = (int64_t)(n[0] + 1) * n[1] * n[2], fy = (int64_t)n[0] * (n[1] + 1) * n[2],
                fz = (int64_t)n[0] * n[1] * (n[2] + 1);
  const int64_t per = fx + fy + fz;
  const int b = (int)(q / per);
  int64_t r = q - (int64_t)b * per;
  const int d = r < fx ? 0 : (r < fx + fy ? 1 : 2);
  r -= d == 0 ? 0 : (d == 1 ? fx : fx + fy);
  const int e0 = n[0] + (d == 0), e1 = n[1] + (d == 1);
  int c[3];  // the face's upper cell (leaf coordinates); c[d] in [0, n_d]
  c[0] = (int)(r % e0);
  c[1] = (int)((r / e0) % e1);
  c[2] = (int)(r / ((int64_t)e0 * e1));
  const BlockInfo bi = blocks[b];
  const int32_t* nb27 = nbr + (int64_t)b * 27;
  const int cd = c[d], nd = n[d];
  int klo = -1, kup = -1;  // neighbour kinds where the face is a block face
  if (cd == 0) {
    klo = face_kind(bi, nb27, g, 2 * d);
    if (klo == 0 || klo == 2) return;  // handled by the same-level or finer leaf
  } else if (cd == nd) {
    kup = face_kind(bi, nb27, g, 2 * d + 1);
    if (kup == 2) return;
  }
  const double dt = *dtp;
  const double bdt = beta * dt;
  const double idd = d == 0 ? bi.idx[0] : (d == 1 ? bi.idx[1] : bi.idx[2]);
  const int64_t cs = (int64_t)n[0] * n[1] * n[2];
  auto lam_at = [&](int bb, int i, int j, int k, double out[NV]) {
    const int64_t o = (int64_t)bb * NV * cs + ((int64_t)k * n[1] + j) * n[0] + i;
#pragma unroll
    for (int v = 0; v < NV; ++v) out[v] = lam[o + v * cs];
  };
  double mu[NV];
  double lup[NV], llo[NV];
  double wup = 0.0, wlo = 0.0;
#pragma unroll
  for (int v = 0; v < NV; ++v) lup[v] = llo[v] = 0.0;
  int err = 0;
  // upper cell
  if (cd < nd) {
    lam_at(b, c[0], c[1], c[2], lup);
    wup = idd;
  } else if (kup == 0) {
    const int qn = (d == 2 ? 2 : 1) * 9 + (d == 1 ? 2 : 1) * 3 + (d == 0 ? 2 : 1);
    lam_at(nb27[qn], d == 0 ? 0 : c[0], d == 1 ? 0 : c[1], d == 2 ? 0 : c[2], lup);
    wup = idd;
  } else if (kup == 1) {
    int cc[3] = {c[0], c[1], c[2]};
    cc[d] = nd - 1;
    double ic;
    if (coarse_lam(lam, blocks, M, g, bi, d, 1, cc, lup, &ic)) wup = 0.25 * ic; else err = 1;
  }
  // lower cell
  if (cd > 0) {
    int cc[3] = {c[0], c[1], c[2]};
    cc[d] -= 1;
    lam_at(b, cc[0], cc[1], cc[2], llo);
    wlo = idd;
  } else if (klo == 1) {
    double ic;
    if (coarse_lam(lam, blocks, M, g, bi, d, 0, c, llo, &ic)) wlo = 0.25 * ic; else err = 1;
  }
  if (err) atomicOr(&tm->err, 2);
  bool any = false;
#pragma unroll
  for (int v = 0; v < NV; ++v) {
    mu[v] = bdt * (wup * lup[v] - wlo * llo[v]);
    any |= mu[v] != 0.0;
  }
  if (!any) return;
  // stencil cells i-2, i-1, i, i+1 along d (DC: i-1, i)
  const double gam = g.gamma, gm1 = gam - 1.0, igm1 = 1.0 / gm1;
  int64_t idx[4];
  double w[4][NV];
#pragma unroll
  for (int t = 0; t < 4; ++t) {
    if (!RECON && (t == 0 || t == 3)) continue;
    int cc[3] = {c[0], c[1], c[2]};
    cc[d] += t - 2;
    idx[t] = nb_index(g, nbr, b, cc[0], cc[1], cc[2]);
    double u[NV];
#pragma unroll
    for (int v = 0; v < NV; ++v) u[v] = U[idx[t] + v * g.vstride];
    to_prim(u, gam, w[t]);
  }
  FState L, R;
  double wl[NV], wr[NV];
#pragma unroll
  for (int v = 0; v < NV; ++v) {
    if (RECON) {
      wl[v] = w[1][v] + mc_half(w[1][v] - w[0][v], w[2][v] - w[1][v]);
      wr[v] = w[2][v] - mc_half(w[2][v] - w[1][v], w[3][v] - w[2][v]);
    } else {
      wl[v] = w[1][v];
      wr[v] = w[2][v];
    }
  }
  L = FState{wl[0], wl[1], wl[2], wl[3], wl[4], 0, 0, 0};
  R = FState{wr[0], wr[1], wr[2], wr[3], wr[4], 0, 0, 0};
  complete_state(L, gam, igm1);
  complete_state(R, gam, igm1);
  double gL[8] = {0, 0, 0, 0, 0, 0, 0, 0}, gR[8] = {0, 0, 0, 0, 0, 0, 0, 0};
  hlle_rev<-1>(L, R, gm1, mu, gL, gR, d);
  double gwl[NV] = {0, 0, 0, 0, 0}, gwr[NV] = {0, 0, 0, 0, 0};
  complete_state_rev(L, gam, igm1, gL, gwl);
  complete_state_rev(R, gam, igm1, gR, gwr);
  double gq[4][NV];
#pragma unroll
  for (int t = 0; t < 4; ++t)
#pragma unroll
    for (int v = 0; v < NV; ++v) gq[t][v] = 0.0;
#pragma unroll
  for (int v = 0; v < NV; ++v) {
    if (RECON) {
      double ga, gb;
      mc_branch(w[1][v] - w[0][v], w[2][v] - w[1][v], ga, gb);
      gq[1][v] += gwl[v] * (1.0 + 0.5 * ga - 0.5 * gb);
      gq[0][v] -= gwl[v] * 0.5 * ga;
      gq[2][v] += gwl[v] * 0.5 * gb;
      mc_branch(w[2][v] - w[1][v], w[3][v] - w[2][v], ga, gb);
      gq[2][v] += gwr[v] * (1.0 - 0.5 * ga + 0.5 * gb);
      gq[1][v] += gwr[v] * 0.5 * ga;
      gq[3][v] -= gwr[v] * 0.5 * gb;
    } else {
      gq[1][v] = gwl[v];
      gq[2][v] = gwr[v];
    }
  }
#pragma unroll
  for (int t = 0; t < 4; ++t) {
    if (!RECON && (t == 0 || t == 3)) continue;
#pragma unroll
    for (int v = 0; v < NV; ++v)
      if (gq[t][v] != 0.0) atomicAdd(&gw[idx[t] + v * g.vstride], gq[t][v]);
  }
}

// Primitive adjoints to conserved ones at the forward state, in place, over
// every padded cell that received any.
__global__ void __launch_bounds__(256) adjf_prim_kernel(const double* __restrict__ U, double* gw, int64_t ncells,
                                                        Geom g) {
  const int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (q >= ncells) return;
  const int64_t b = q / g.vstride, c = q - b * g.vstride;
  const int64_t o = b * g.bstride + c;
  double gp[NV];
  bool any = false;
#pragma unroll
  for (int v = 0; v < NV; ++v) {
    gp[v] = gw[o + v * g.vstride];
    any |= gp[v] != 0.0;
  }
  if (!any) return;
  double u[NV], gu[NV];
#pragma unroll
  for (int v = 0; v < NV; ++v) u[v] = U[o + v * g.vstride];
  prim_rev(u, g.gamma, gp, gu);
#pragma unroll
  for (int v = 0; v < NV; ++v) gw[o + v * g.vstride] = gu[v];
}

// Add weight * x (image signs of code applied) to the composite level-L
// field at global cell J (any integers within a domain length): the level-L
// leaf's cell, or 1/8 to each of the 8 level-(L+1) cells below it.
__device__ void comp_scatter(double* gu, const BlockInfo* blocks, const LevelMaps& M, const Geom& g, int L,
                             int J0, int J1, int J2, const double x[NV], double weight, int* err) {
  int J[3] = {J0, J1, J2};
  const int code = cell_in_domain(g, L, J);
  double y[NV];
#pragma unroll
  for (int v = 0; v < NV; ++v) y[v] = weight * x[v];
  apply_image_signs(code, y);
  const int n[3] = {g.n1, g.n2, g.n3};
  const int32_t id = leaf_at(M, L, J[0] / n[0], J[1] / n[1], J[2] / n[2]);
  if (id >= 0) {
    const BlockInfo bc = blocks[id];
    double* p = gu + (int64_t)id * g.bstride +
                pad_index(g, J[0] - bc.lx * n[0], J[1] - bc.ly * n[1], J[2] - bc.lz * n[2]);
#pragma unroll
    for (int v = 0; v < NV; ++v)
      if (y[v] != 0.0) atomicAdd(&p[v * g.vstride], y[v]);
    return;
  }
  if (L + 1 > M.maxl) {
    *err = 1;
    return;
  }
  for (int cc = 0; cc < 8; ++cc) {
    const int F0 = 2 * J[0] + (cc & 1), F1 = 2 * J[1] + ((cc >> 1) & 1), F2 = 2 * J[2] + ((cc >> 2) & 1);
    const int32_t fid = leaf_at(M, L + 1, F0 / n[0], F1 / n[1], F2 / n[2]);
    if (fid < 0) {
      *err = 1;
      return;
    }
    const BlockInfo bf = blocks[fid];
    double* p = gu + (int64_t)fid * g.bstride + pad_index(g, F0 - bf.lx * n[0], F1 - bf.ly * n[1], F2 - bf.lz * n[2]);
#pragma unroll
    for (int v = 0; v < NV; ++v)
      if (y[v] != 0.0) atomicAdd(&p[v * g.vstride], 0.125 * y[v]);
  }
}

// Transposed ghost fill of the face records jf (level jumps and walls): one
// thread per ghost cell of a face slab; gu holds conserved adjoints.
__global__ void __launch_bounds__(256) adjf_ghost_kernel(const double* __restrict__ U, double* gu,
                                                         const BlockInfo* blocks, Geom g, LevelMaps M, DevTime* tm,
                                                         const int32_t* __restrict__ jf) {
  const int2 rec = reinterpret_cast<const int2*>(jf)[blockIdx.y];
  const int b = rec.x, d = (rec.y & 7) >> 1, hi = rec.y & 1, wall = (rec.y >> 3) & 7;
  const int n[3] = {g.n1, g.n2, g.n3};
  const int t1 = d == 0 ? 1 : 0, t2 = d == 2 ? 1 : 2;
  const int area = n[t1] * n[t2];
  const int q = blockIdx.x * blockDim.x + threadIdx.x;
  if (q >= 2 * area) return;
  const int s = q / area, r = q - s * area;
  int c[3];
  c[t1] = r % n[t1];
  c[t2] = r / n[t1];
  c[d] = hi ? n[d] + s : s - NG;
  double* ub = gu + (int64_t)b * g.bstride;
  double x[NV];
  bool any = false;
#pragma unroll
  for (int v = 0; v < NV; ++v) {
    x[v] = ub[pad_index(g, c[0], c[1], c[2]) + v * g.vstride];
    any |= x[v] != 0.0;
  }
  if (!any) return;
  int err = 0;
  if (wall) {
    int src[3] = {c[0], c[1], c[2]};
    src[d] = wall == BC_OUTFLOW ? (hi ? n[d] - 1 : 0) : (hi ? 2 * n[d] - 1 - c[d] : -1 - c[d]);
    double* p = ub + pad_index(g, src[0], src[1], src[2]);
#pragma unroll
    for (int v = 0; v < NV; ++v)
      atomicAdd(&p[v * g.vstride], (wall == BC_REFLECT && v == 1 + d) ? -x[v] : x[v]);
    return;
  }
  const BlockInfo bi = blocks[b];
  const int L = bi.level;
  int bl[3] = {bi.lx, bi.ly, bi.lz};
  bl[d] = wrap_i(bl[d] + (hi ? 1 : -1), g.nrb[d] << L);
  const bool coarser = L > 0 && leaf_at(M, L - 1, bl[0] >> 1, bl[1] >> 1, bl[2] >> 1) >= 0;
  const int lo[3] = {bi.lx, bi.ly, bi.lz};
  int J[3];
#pragma unroll
  for (int e = 0; e < 3; ++e) J[e] = wrap_i(lo[e] * n[e] + c[e], (g.nrb[e] * n[e]) << L);
  if (coarser) {
    // x = C(I) + 1/4 sum_e sigma_e s_e, s_e = minmod(C(I) - C(I-e), C(I+e) - C(I))
    const int I[3] = {J[0] >> 1, J[1] >> 1, J[2] >> 1};
    double c0[NV], cm[3][NV], cp[3][NV];
    comp_val(U, blocks, M, g, L - 1, I[0], I[1], I[2], c0, &err);
#pragma unroll
    for (int e = 0; e < 3; ++e) {
      comp_val(U, blocks, M, g, L - 1, I[0] - (e == 0), I[1] - (e == 1), I[2] - (e == 2), cm[e], &err);
      comp_val(U, blocks, M, g, L - 1, I[0] + (e == 0), I[1] + (e == 1), I[2] + (e == 2), cp[e], &err);
    }
    double a0[NV], am[3][NV], ap[3][NV];
#pragma unroll
    for (int v = 0; v < NV; ++v) {
      double k0 = 1.0;
#pragma unroll
      for (int e = 0; e < 3; ++e) {
        const double sg = (J[e] & 1) ? 0.25 : -0.25;
        const double da = c0[v] - cm[e][v], db = cp[e][v] - c0[v];
        am[e][v] = ap[e][v] = 0.0;
        if (da * db > 0.0) {
          if (fabs(da) <= fabs(db)) {  // s = da
            k0 += sg;
            am[e][v] = -sg * x[v];
          } else {  // s = db
            k0 -= sg;
            ap[e][v] = sg * x[v];
          }
        }
      }
      a0[v] = k0 * x[v];
    }
    comp_scatter(gu, blocks, M, g, L - 1, I[0], I[1], I[2], a0, 1.0, &err);
#pragma unroll
    for (int e = 0; e < 3; ++e) {
      comp_scatter(gu, blocks, M, g, L - 1, I[0] - (e == 0), I[1] - (e == 1), I[2] - (e == 2), am[e], 1.0, &err);
      comp_scatter(gu, blocks, M, g, L - 1, I[0] + (e == 0), I[1] + (e == 1), I[2] + (e == 2), ap[e], 1.0, &err);
    }
  } else {
    // restriction of the 8 fine cells below J
    comp_scatter(gu, blocks, M, g, L, J[0], J[1], J[2], x, 1.0, &err);
  }
  if (err) atomicOr(&tm->err, 2);
}

// out (upload layout) = add0 + add1 + the active cells of gu.
__global__ void __launch_bounds__(256) adjf_out_kernel(const double* __restrict__ gu, double* out,
                                                       const double* add0, const double* add1, int64_t total,
                                                       Geom g) {
  const int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (q >= total) return;
  const int i = q % g.n1;
  int64_t r = q / g.n1;
  const int j = r % g.n2;
  r /= g.n2;
  const int k = r % g.n3;
  r /= g.n3;  // r = block*5 + v
  double x = gu[r * g.vstride + pad_index(g, i, j, k)];
  if (add0) x += add0[q];
  if (add1) x += add1[q];
  out[q] = x;
}

hipError_t launch_adj_stage_facewise(int recon, const double* U, const double* lam, double* gw,
                                     const BlockInfo* blocks, int32_t nblocks, const Geom& g, const int32_t* nbr,
                                     const LevelMaps& maps, const int32_t* jf, int32_t njf, const double* dtp,
                                     double beta, double* out, const double* add0, const double* add1,
                                     DevTime* tm, hipStream_t s) {
  hipError_t e = hipMemsetAsync(gw, 0, (size_t)nblocks * g.bstride * sizeof(double), s);
  if (e != hipSuccess) return e;
  const int64_t nfaces = (int64_t)nblocks * ((int64_t)(g.n1 + 1) * g.n2 * g.n3 + (int64_t)g.n1 * (g.n2 + 1) * g.n3 +
                                             (int64_t)g.n1 * g.n2 * (g.n3 + 1));
  const dim3 gf((unsigned)((nfaces + 255) / 256));
  if (recon)
    hipLaunchKernelGGL(adjf_face_kernel<1>, gf, dim3(256), 0, s, U, lam, gw, blocks, nbr, maps, g, dtp, beta,
                       nfaces, tm);
  else
    hipLaunchKernelGGL(adjf_face_kernel<0>, gf, dim3(256), 0, s, U, lam, gw, blocks, nbr, maps, g, dtp, beta,
                       nfaces, tm);
  const int64_t ncells = (int64_t)nblocks * g.vstride;
  hipLaunchKernelGGL(adjf_prim_kernel, dim3((unsigned)((ncells + 255) / 256)), dim3(256), 0, s, U, gw, ncells, g);
  if (njf > 0) {
    const int area = std::max(std::max(g.n1 * g.n2, g.n1 * g.n3), g.n2 * g.n3);
    hipLaunchKernelGGL(adjf_ghost_kernel, dim3((2 * area + 255) / 256, njf), dim3(256), 0, s, U, gw, blocks, g, maps,
                       tm, jf);
  }
  const int64_t total = (int64_t)nblocks * NV * g.n1 * g.n2 * g.n3;
  hipLaunchKernelGGL(adjf_out_kernel, dim3((unsigned)((total + 255) / 256)), dim3(256), 0, s, gw, out, add0, add1,
                     total, g);
  return hipGetLastError();
}

// Device clock for recomputation: dt of the current cycle from a record.
__global__ void tape_dt_kernel(DevTime* tm, const double* dts, int c, int record) {
  if (threadIdx.x != 0 || blockIdx.x != 0) return;
  if (record)
    const_cast<double*>(dts)[c] = tm->dt;
  else
    tm->dt = dts[c];
}

hipError_t launch_tape_dt(DevTime* tm, double* dts, int32_t c, int32_t record, hipStream_t s) {
  hipLaunchKernelGGL(tape_dt_kernel, dim3(1), dim3(64), 0, s, tm, (const double*)dts, (int)c, (int)record);
  return hipGetLastError();
}

}  // namespace pkh

namespace pkh {

// Device clocks of many meshes in one launch (thread per mesh); modes as
// for clock_kernel.
__global__ void clock_group_kernel(DevTime* const* tms, int n, int mode, double t_end) {
  const int q = blockIdx.x * blockDim.x + threadIdx.x;
  if (q >= n) return;
  DevTime* tm = tms[q];
  if (mode & (CLOCK_END | CLOCK_FROM_SMAX)) {
    const double smax = __longlong_as_double((long long)tm->smax_bits);
    tm->dt_next = tm->cfl / smax;
  }
  if (mode & CLOCK_END) {
    tm->t += tm->dt;
    tm->cycle += 1;
  }
  if (mode & CLOCK_BEGIN) {
    double dt = tm->dt_next;
    if (isfinite(t_end) && dt > t_end - tm->t) dt = fmax(t_end - tm->t, 0.0);
    tm->dt = dt;
    tm->smax_bits = 0ull;
  }
}

hipError_t launch_clock_group(DevTime* const* tms, int32_t n, int32_t mode, double t_end, hipStream_t s) {
  hipLaunchKernelGGL(clock_group_kernel, dim3((n + 63) / 64), dim3(64), 0, s, tms, (int)n, (int)mode, t_end);
  return hipGetLastError();
}

}  // namespace pkh
