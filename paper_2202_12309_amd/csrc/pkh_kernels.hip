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

#include "pkh_internal.h"

namespace pkh {

// ---------------------------------------------------------------------------
// Pointwise physics
// ---------------------------------------------------------------------------

__device__ __forceinline__ bool to_prim(const double u[NV], double gam, double w[NV]) {
  const double ir = 1.0 / u[0];
  w[0] = u[0];
  w[1] = u[1] * ir;
  w[2] = u[2] * ir;
  w[3] = u[3] * ir;
  w[4] = (gam - 1.0) * (u[4] - 0.5 * (u[1] * w[1] + u[2] * w[2] + u[3] * w[3]));
  return (w[0] > 0.0) && (w[4] > 0.0);  // false also for NaN
}

// Monotonised-central limited slope (van Leer 1977).
__device__ __forceinline__ double mc_slope(double dl, double dr) {
  const double m = fmin(fmin(2.0 * fabs(dl), 2.0 * fabs(dr)), 0.5 * fabs(dl + dr));
  return (dl * dr > 0.0) ? copysign(m, dl) : 0.0;
}

__device__ __forceinline__ double minmod(double a, double b) {
  const double m = fmin(fabs(a), fabs(b));
  return (a * b > 0.0) ? copysign(m, a) : 0.0;
}

// HLLE flux normal to direction D from primitive states; Einfeldt (1988)
// bounds b+ = max(u_roe + a_roe, u_R + c_R, 0), b- = min(u_roe - a_roe,
// u_L - c_L, 0).
template <int D>
__device__ __forceinline__ void hlle(const double wl[NV], const double wr[NV], double gam,
                                     double f[NV]) {
  const double gm1 = gam - 1.0;
  const double igm1 = 1.0 / gm1;
  const double rl = wl[0], pl = wl[4], rr = wr[0], pr = wr[4];
  const double ul = wl[1 + D], ur = wr[1 + D];
  const double irl = 1.0 / rl, irr = 1.0 / rr;
  const double v2l = wl[1] * wl[1] + wl[2] * wl[2] + wl[3] * wl[3];
  const double v2r = wr[1] * wr[1] + wr[2] * wr[2] + wr[3] * wr[3];
  const double el = pl * igm1 + 0.5 * rl * v2l;
  const double er = pr * igm1 + 0.5 * rr * v2r;
  const double hl = (el + pl) * irl, hr = (er + pr) * irr;
  const double cl = sqrt(gam * pl * irl), cr = sqrt(gam * pr * irr);
  const double sl = sqrt(rl), sr = sqrt(rr);
  const double r = sl / (sl + sr), r1 = 1.0 - r;
  const double vb0 = r * wl[1] + r1 * wr[1];
  const double vb1 = r * wl[2] + r1 * wr[2];
  const double vb2 = r * wl[3] + r1 * wr[3];
  const double hb = r * hl + r1 * hr;
  const double ab = sqrt(gm1 * (hb - 0.5 * (vb0 * vb0 + vb1 * vb1 + vb2 * vb2)));
  const double vbn = D == 0 ? vb0 : (D == 1 ? vb1 : vb2);
  const double bp = fmax(fmax(vbn + ab, ur + cr), 0.0);
  const double bm = fmin(fmin(vbn - ab, ul - cl), 0.0);
  const double ib = 1.0 / (bp - bm);
  const double bpm = bp * bm;
  const double ml = rl * ul, mr = rr * ur;  // mass fluxes
  // mass
  f[0] = (bp * ml - bm * mr + bpm * (rr - rl)) * ib;
  // momentum
#pragma unroll
  for (int c = 0; c < 3; ++c) {
    double fl = ml * wl[1 + c], fr = mr * wr[1 + c];
    if (c == D) {
      fl += pl;
      fr += pr;
    }
    f[1 + c] = (bp * fl - bm * fr + bpm * (rr * wr[1 + c] - rl * wl[1 + c])) * ib;
  }
  // energy
  f[4] = (bp * (el + pl) * ul - bm * (er + pr) * ur + bpm * (er - el)) * ib;
}

// ---------------------------------------------------------------------------
// Stage kernel: U_out = U_base - beta*dt * D(U_in) over every block.
//
// A workgroup owns TJ rows of N1 cells of one block and streams through z.
// Per z-plane it stages the plane's primitives (TJ+4 rows incl. halo, full
// padded row width, one contiguous run of memory per variable) in LDS,
// computes every x- and y-face flux of the plane once (LDS), and keeps a
// register window of the column's primitives for the z faces. A cell is
// finished once its upper z face is known; its x/y divergence waits in a
// short register queue.
// ---------------------------------------------------------------------------

template <int RECON, int N1, int TJ>
__global__ void __launch_bounds__(N1 * TJ) stage_kernel(StageLaunch a) {
  constexpr int NT = N1 * TJ;
  constexpr int P1 = N1 + 2 * NG;
  constexpr int RW = TJ + 2 * NG;
  constexpr int PLANE = RW * P1;
  constexpr int NX = TJ * (N1 + 1);
  constexpr int NY = (TJ + 1) * N1;
  constexpr int LAG = RECON ? 1 : 0;  // z face m is computed at plane m + LAG
  constexpr int WN = RECON ? 4 : 2;   // z window length
  constexpr int QN = 1 + LAG;         // x/y divergence queue length
  constexpr int NWAVE = (NT + 63) / 64;

  __shared__ double sW[NV][PLANE];
  __shared__ double sFx[NV][NX];
  __shared__ double sFy[NV][NY];
  __shared__ double sRed[NWAVE];

  const Geom& g = a.g;
  const int ntj = g.n2 / TJ;
  const int nwg = gridDim.x;
  int wg = blockIdx.x;
  // XCD-aware order: workgroups are dealt round-robin to the 8 XCDs; map
  // consecutive tiles of a block (which share halo rows) to one XCD's L2.
  if ((nwg & 7) == 0) wg = (wg & 7) * (nwg >> 3) + (wg >> 3);
  const int blk = wg / ntj;
  if (blk >= a.nblocks) return;
  const int j0 = (wg - blk * ntj) * TJ;
  const int tid = threadIdx.x;
  const int ti = tid % N1, tj = tid / N1;

  const BlockInfo bi = a.blocks[blk];
  const double gam = g.gamma;
  const double coef = a.beta * a.tm->dt;
  const int64_t vs = g.vstride;
  const double* __restrict__ in = a.uin + (int64_t)blk * g.bstride;
  const double* base = a.ubase + (int64_t)blk * g.bstride;
  double* out = a.uout + (int64_t)blk * g.bstride;
  const int n2 = g.n2, n3 = g.n3;
  const int j = j0 + tj;
  const int fsz = NV * max(max(g.n1 * n2, g.n1 * n3), n2 * n3);  // face slot stride
  double* fbuf = a.fbuf;

  double w[WN][NV];
  double dq[QN][NV];
  double fzp[NV];
  bool bad = false;
  double smax = 0.0;
  const int mask = bi.finer_mask;

#pragma unroll
  for (int s = 0; s < WN; ++s)
#pragma unroll
    for (int v = 0; v < NV; ++v) w[s][v] = 0.0;
#pragma unroll
  for (int s = 0; s < QN; ++s)
#pragma unroll
    for (int v = 0; v < NV; ++v) dq[s][v] = 0.0;
#pragma unroll
  for (int v = 0; v < NV; ++v) fzp[v] = 0.0;

  for (int p = -1 - LAG; p < n3 + 1 + LAG; ++p) {
    // --- stage plane p (rows j0-2 .. j0+TJ+1) as primitives in LDS
    const int64_t pofs = ((int64_t)(p + NG) * g.p2 + j0) * P1;
    for (int c = tid; c < PLANE; c += NT) {
      double u[NV], wp[NV];
#pragma unroll
      for (int v = 0; v < NV; ++v) u[v] = in[v * vs + pofs + c];
      bad |= !to_prim(u, gam, wp);
#pragma unroll
      for (int v = 0; v < NV; ++v) sW[v][c] = wp[v];
    }
    __syncthreads();

    // --- z window
#pragma unroll
    for (int s = 0; s < WN - 1; ++s)
#pragma unroll
      for (int v = 0; v < NV; ++v) w[s][v] = w[s + 1][v];
#pragma unroll
    for (int v = 0; v < NV; ++v) w[WN - 1][v] = sW[v][(tj + NG) * P1 + ti + NG];

    // --- z face m between cells m-1 and m, then finish cell m-1
    const int m = p - LAG;
    if (m >= 0 && m <= n3) {
      double wl[NV], wr[NV], fz[NV];
#pragma unroll
      for (int v = 0; v < NV; ++v) {
        if constexpr (RECON) {
          wl[v] = w[1][v] + 0.5 * mc_slope(w[1][v] - w[0][v], w[2][v] - w[1][v]);
          wr[v] = w[2][v] - 0.5 * mc_slope(w[2][v] - w[1][v], w[3][v] - w[2][v]);
        } else {
          wl[v] = w[0][v];
          wr[v] = w[1][v];
        }
      }
      hlle<2>(wl, wr, gam, fz);
      if (m == 0 && bi.fslot[ZLO] >= 0) {
#pragma unroll
        for (int v = 0; v < NV; ++v)
          fbuf[(int64_t)bi.fslot[ZLO] * fsz + ((int64_t)v * n2 + j) * N1 + ti] = fz[v];
      }
      if (m == n3 && bi.fslot[ZHI] >= 0) {
#pragma unroll
        for (int v = 0; v < NV; ++v)
          fbuf[(int64_t)bi.fslot[ZHI] * fsz + ((int64_t)v * n2 + j) * N1 + ti] = fz[v];
      }
      if (m >= 1) {
        const int k = m - 1;
        const int64_t o = ((int64_t)(k + NG) * g.p2 + (j + NG)) * P1 + ti + NG;
        double un[NV];
#pragma unroll
        for (int v = 0; v < NV; ++v) {
          const double du = dq[0][v] + (fz[v] - fzp[v]) * bi.idx[2];
          un[v] = base[v * vs + o] - coef * du;
          out[v * vs + o] = un[v];
        }
        if (a.do_dt) {
          const bool skip = ((mask >> XLO) & 1 && ti == 0) || ((mask >> XHI) & 1 && ti == N1 - 1) ||
                            ((mask >> YLO) & 1 && j == 0) || ((mask >> YHI) & 1 && j == n2 - 1) ||
                            ((mask >> ZLO) & 1 && k == 0) || ((mask >> ZHI) & 1 && k == n3 - 1);
          if (!skip) {
            double wn[NV];
            bad |= !to_prim(un, gam, wn);
            const double cs = sqrt(gam * wn[4] / wn[0]);
            const double s = fmax(fmax((fabs(wn[1]) + cs) * bi.idx[0], (fabs(wn[2]) + cs) * bi.idx[1]),
                                  (fabs(wn[3]) + cs) * bi.idx[2]);
            smax = fmax(smax, s);
          }
        }
      }
#pragma unroll
      for (int v = 0; v < NV; ++v) fzp[v] = fz[v];
    }

    // --- x and y faces of plane p, divergence into the queue
    if (p >= 0 && p < n3) {
      for (int f = tid; f < NX + NY; f += NT) {
        double wl[NV], wr[NV], fl[NV];
        if (f < NX) {
          const int r = f / (N1 + 1), i = f - r * (N1 + 1);
          const int c0 = (r + NG) * P1 + i;  // cell i-2 of row r
#pragma unroll
          for (int v = 0; v < NV; ++v) {
            const double qm2 = sW[v][c0], qm1 = sW[v][c0 + 1], q0 = sW[v][c0 + 2], qp1 = sW[v][c0 + 3];
            if constexpr (RECON) {
              wl[v] = qm1 + 0.5 * mc_slope(qm1 - qm2, q0 - qm1);
              wr[v] = q0 - 0.5 * mc_slope(q0 - qm1, qp1 - q0);
            } else {
              wl[v] = qm1;
              wr[v] = q0;
            }
          }
          hlle<0>(wl, wr, gam, fl);
#pragma unroll
          for (int v = 0; v < NV; ++v) sFx[v][f] = fl[v];
          const int slot = (i == 0) ? bi.fslot[XLO] : ((i == N1) ? bi.fslot[XHI] : -1);
          if (slot >= 0) {
#pragma unroll
            for (int v = 0; v < NV; ++v)
              fbuf[(int64_t)slot * fsz + ((int64_t)v * n3 + p) * n2 + j0 + r] = fl[v];
          }
        } else {
          const int f2 = f - NX;
          const int r = f2 / N1, i = f2 - r * N1;
          const int c0 = r * P1 + i + NG;  // row r-2 of the tile, column i
#pragma unroll
          for (int v = 0; v < NV; ++v) {
            const double qm2 = sW[v][c0], qm1 = sW[v][c0 + P1], q0 = sW[v][c0 + 2 * P1],
                         qp1 = sW[v][c0 + 3 * P1];
            if constexpr (RECON) {
              wl[v] = qm1 + 0.5 * mc_slope(qm1 - qm2, q0 - qm1);
              wr[v] = q0 - 0.5 * mc_slope(q0 - qm1, qp1 - q0);
            } else {
              wl[v] = qm1;
              wr[v] = q0;
            }
          }
          hlle<1>(wl, wr, gam, fl);
#pragma unroll
          for (int v = 0; v < NV; ++v) sFy[v][f2] = fl[v];
          const int jf = j0 + r;
          const int slot = (jf == 0) ? bi.fslot[YLO] : ((jf == n2) ? bi.fslot[YHI] : -1);
          if (slot >= 0) {
#pragma unroll
            for (int v = 0; v < NV; ++v)
              fbuf[(int64_t)slot * fsz + ((int64_t)v * n3 + p) * N1 + i] = fl[v];
          }
        }
      }
      __syncthreads();
#pragma unroll
      for (int s = 0; s < QN - 1; ++s)
#pragma unroll
        for (int v = 0; v < NV; ++v) dq[s][v] = dq[s + 1][v];
#pragma unroll
      for (int v = 0; v < NV; ++v)
        dq[QN - 1][v] = (sFx[v][tj * (N1 + 1) + ti + 1] - sFx[v][tj * (N1 + 1) + ti]) * bi.idx[0] +
                        (sFy[v][(tj + 1) * N1 + ti] - sFy[v][tj * N1 + ti]) * bi.idx[1];
    } else {
      // keep the queue aligned with plane numbers on the leading planes
#pragma unroll
      for (int s = 0; s < QN - 1; ++s)
#pragma unroll
        for (int v = 0; v < NV; ++v) dq[s][v] = dq[s + 1][v];
    }
    __syncthreads();
  }

  if (a.do_dt) {
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) smax = fmax(smax, __shfl_xor(smax, off));
    if ((tid & 63) == 0) sRed[tid >> 6] = smax;
    __syncthreads();
    if (tid == 0) {
      double mx = sRed[0];
      for (int q = 1; q < NWAVE; ++q) mx = fmax(mx, sRed[q]);
      atomicMax(&a.tm->smax_bits, (unsigned long long)__double_as_longlong(mx));
    }
  }
  if (bad) atomicOr(&a.tm->err, 1);
}

template <int RECON, int N1, int TJ>
static hipError_t launch_stage_t(const StageLaunch& a, hipStream_t s) {
  const int ntj = a.g.n2 / TJ;
  int64_t nwg = (int64_t)a.nblocks * ntj;
  nwg = (nwg + 7) / 8 * 8;
  hipLaunchKernelGGL((stage_kernel<RECON, N1, TJ>), dim3((unsigned)nwg), dim3(N1 * TJ), 0, s, a);
  return hipGetLastError();
}

template <int N1, int TJ>
static hipError_t launch_stage_n(const StageLaunch& a, hipStream_t s) {
  return a.recon ? launch_stage_t<1, N1, TJ>(a, s) : launch_stage_t<0, N1, TJ>(a, s);
}

hipError_t launch_stage(const StageLaunch& a, hipStream_t s) {
  switch (a.g.n1) {
    case 8:
      return launch_stage_n<8, 8>(a, s);
    case 16:
      return launch_stage_n<16, 8>(a, s);
    case 32:
      return launch_stage_n<32, 8>(a, s);
    case 64:
      return launch_stage_n<64, 4>(a, s);
    default:
      return hipErrorInvalidValue;
  }
}

// ---------------------------------------------------------------------------
// Composite-field lookups shared by the ghost fill and the regrid kernels.
// ---------------------------------------------------------------------------

__device__ __forceinline__ int wrap_i(int a, int n) {
  a %= n;
  return a < 0 ? a + n : a;
}

__device__ __forceinline__ int32_t leaf_at(const LevelMaps& M, int L, int bx, int by, int bz) {
  return M.map[M.off[L] + ((int64_t)bz * M.nb[L][1] + by) * M.nb[L][0] + bx];
}

__device__ __forceinline__ int64_t pad_index(const Geom& g, int i, int j, int k) {
  return ((int64_t)(k + NG) * g.p2 + (j + NG)) * g.p1 + (i + NG);
}

// Composite value at level L, global cell J (any integers; wrapped here):
// leaf value at level L; restriction of the level-(L+1) leaves; or, while
// regridding, the containing coarser cell (injection).
__device__ double comp_val(const double* u, const BlockInfo* blocks, const LevelMaps& M,
                           const Geom& g, int L, int J0, int J1, int J2, int v, int* err) {
  const int n[3] = {g.n1, g.n2, g.n3};
  int J[3] = {J0, J1, J2}, b[3];
#pragma unroll
  for (int d = 0; d < 3; ++d) {
    J[d] = wrap_i(J[d], (g.nrb[d] * n[d]) << L);
    b[d] = J[d] / n[d];
  }
  int32_t id = leaf_at(M, L, b[0], b[1], b[2]);
  if (id >= 0)
    return u[(int64_t)id * g.bstride + v * g.vstride +
             pad_index(g, J[0] - b[0] * n[0], J[1] - b[1] * n[1], J[2] - b[2] * n[2])];
  for (int Lc = L - 1; Lc >= 0; --Lc) {
    const int sh = L - Lc;
    id = leaf_at(M, Lc, b[0] >> sh, b[1] >> sh, b[2] >> sh);
    if (id >= 0) {
      const BlockInfo bc = blocks[id];
      return u[(int64_t)id * g.bstride + v * g.vstride +
               pad_index(g, (J[0] >> sh) - bc.lx * n[0], (J[1] >> sh) - bc.ly * n[1],
                         (J[2] >> sh) - bc.lz * n[2])];
    }
  }
  if (L + 1 > M.maxl) {
    *err = 1;
    return 0.0;
  }
  double f[8];
#pragma unroll
  for (int c = 0; c < 8; ++c) {
    const int F0 = 2 * J[0] + (c & 1), F1 = 2 * J[1] + ((c >> 1) & 1), F2 = 2 * J[2] + ((c >> 2) & 1);
    const int32_t fid = leaf_at(M, L + 1, F0 / n[0], F1 / n[1], F2 / n[2]);
    if (fid < 0) {
      *err = 1;
      return 0.0;
    }
    const BlockInfo bf = blocks[fid];
    f[c] = u[(int64_t)fid * g.bstride + v * g.vstride +
             pad_index(g, F0 - bf.lx * n[0], F1 - bf.ly * n[1], F2 - bf.lz * n[2])];
  }
  return 0.125 * (((f[0] + f[1]) + (f[2] + f[3])) + ((f[4] + f[5]) + (f[6] + f[7])));
}

// Linear prolongation to fine cell F (level L) from the composite field at
// level L-1 with minmod slopes; the fine centre sits a quarter coarse width
// from the coarse centre along each axis.
__device__ double prolong_val(const double* u, const BlockInfo* blocks, const LevelMaps& M,
                              const Geom& g, int L, int F0, int F1, int F2, int v, int* err) {
  const int I0 = F0 >> 1, I1 = F1 >> 1, I2 = F2 >> 1;  // F >= 0 here
  const double c0 = comp_val(u, blocks, M, g, L - 1, I0, I1, I2, v, err);
  const double s0 = minmod(c0 - comp_val(u, blocks, M, g, L - 1, I0 - 1, I1, I2, v, err),
                           comp_val(u, blocks, M, g, L - 1, I0 + 1, I1, I2, v, err) - c0);
  const double s1 = minmod(c0 - comp_val(u, blocks, M, g, L - 1, I0, I1 - 1, I2, v, err),
                           comp_val(u, blocks, M, g, L - 1, I0, I1 + 1, I2, v, err) - c0);
  const double s2 = minmod(c0 - comp_val(u, blocks, M, g, L - 1, I0, I1, I2 - 1, v, err),
                           comp_val(u, blocks, M, g, L - 1, I0, I1, I2 + 1, v, err) - c0);
  const double t0 = (F0 & 1) ? s0 : -s0;
  const double t1 = (F1 & 1) ? s1 : -s1;
  const double t2 = (F2 & 1) ? s2 : -s2;
  return c0 + 0.25 * ((t0 + t1) + t2);
}

// ---------------------------------------------------------------------------
// Fill-in-one ghost exchange: one thread per (block, ghost cell), all five
// variables; ghost cells enumerated in memory order of the padded block.
// ---------------------------------------------------------------------------

__device__ __forceinline__ void ghost_coord(int q, const Geom& g, int& i, int& j, int& k) {
  const int plane = g.p1 * g.p2;
  if (q < 4 * plane) {
    const int s = q / plane, r = q - s * plane;
    k = s < 2 ? s - NG : g.n3 + s - 2;
    j = r / g.p1 - NG;
    i = r - (j + NG) * g.p1 - NG;
    return;
  }
  q -= 4 * plane;
  const int rows = 4 * g.p1;
  if (q < g.n3 * rows) {
    k = q / rows;
    const int r = q - k * rows;
    const int s = r / g.p1;
    i = r - s * g.p1 - NG;
    j = s < 2 ? s - NG : g.n2 + s - 2;
    return;
  }
  q -= g.n3 * rows;
  const int kj = q >> 2, s = q & 3;
  k = kj / g.n2;
  j = kj - k * g.n2;
  i = s < 2 ? s - NG : g.n1 + s - 2;
}

__global__ void __launch_bounds__(256) fill_kernel(double* u, const BlockInfo* blocks, int nblocks,
                                                   Geom g, LevelMaps M, DevTime* tm) {
  const int ngc = 4 * g.p1 * g.p2 + 4 * g.n3 * g.p1 + 4 * g.n3 * g.n2;
  const int q = blockIdx.x * blockDim.x + threadIdx.x;
  const int b = blockIdx.y;
  if (q >= ngc || b >= nblocks) return;
  int i, j, k;
  ghost_coord(q, g, i, j, k);
  const BlockInfo bi = blocks[b];
  const int L = bi.level;
  const int n[3] = {g.n1, g.n2, g.n3};
  int J[3] = {bi.lx * g.n1 + i, bi.ly * g.n2 + j, bi.lz * g.n3 + k}, bl[3];
#pragma unroll
  for (int d = 0; d < 3; ++d) {
    J[d] = wrap_i(J[d], (g.nrb[d] * n[d]) << L);
    bl[d] = J[d] / n[d];
  }
  double* dst = u + (int64_t)b * g.bstride + pad_index(g, i, j, k);
  const int32_t id = leaf_at(M, L, bl[0], bl[1], bl[2]);
  if (id >= 0) {  // same level: copy
    const double* src = u + (int64_t)id * g.bstride +
                        pad_index(g, J[0] - bl[0] * n[0], J[1] - bl[1] * n[1], J[2] - bl[2] * n[2]);
#pragma unroll
    for (int v = 0; v < NV; ++v) dst[v * g.vstride] = src[v * g.vstride];
    return;
  }
  int err = 0;
  if (L > 0 && leaf_at(M, L - 1, bl[0] >> 1, bl[1] >> 1, bl[2] >> 1) >= 0) {
    for (int v = 0; v < NV; ++v)
      dst[v * g.vstride] = prolong_val(u, blocks, M, g, L, J[0], J[1], J[2], v, &err);
  } else {
    for (int v = 0; v < NV; ++v)
      dst[v * g.vstride] = comp_val(u, blocks, M, g, L, J[0], J[1], J[2], v, &err);
  }
  if (err) atomicOr(&tm->err, 2);
}

hipError_t launch_fill(double* u, const BlockInfo* blocks, int32_t nblocks, const Geom& g,
                       const LevelMaps& maps, DevTime* tm, hipStream_t s) {
  const int ngc = 4 * g.p1 * g.p2 + 4 * g.n3 * g.p1 + 4 * g.n3 * g.n2;
  dim3 grid((ngc + 255) / 256, nblocks);
  hipLaunchKernelGGL(fill_kernel, grid, dim3(256), 0, s, u, blocks, nblocks, g, maps, tm);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Flux correction as reflux: on each coarse face bordering finer leaves the
// coarse flux is replaced by the area mean of the 4 fine fluxes,
// U += +-beta*dt/dx * (F_own - F_fine). One thread per cell of a coarse
// block that has such faces; the cell applies all of its faces in x, y, z
// order, then (corrector stage) contributes to the CFL reduction the stage
// kernel skipped for it.
// ---------------------------------------------------------------------------

__global__ void __launch_bounds__(256) flux_correct_kernel(double* u, const BlockInfo* blocks,
                                                           const FineFace* ff,
                                                           const int32_t* ff_first,
                                                           const int32_t* cblocks, Geom g,
                                                           DevTime* tm, double beta, int do_dt,
                                                           const double* fbuf) {
  __shared__ double sRed[4];
  const int c = blockIdx.y;
  const int b = cblocks[c];
  const BlockInfo bi = blocks[b];
  const int ncell = g.n1 * g.n2 * g.n3;
  const int q = blockIdx.x * blockDim.x + threadIdx.x;
  double smax = 0.0;
  bool bad = false;
  if (q < ncell) {
    const int i = q % g.n1, j = (q / g.n1) % g.n2, k = q / (g.n1 * g.n2);
    const int n[3] = {g.n1, g.n2, g.n3};
    const int cc[3] = {i, j, k};
    const int fsz = NV * max(max(g.n1 * g.n2, g.n1 * g.n3), g.n2 * g.n3);
    bool touched = false;
    double* cell = u + (int64_t)b * g.bstride + pad_index(g, i, j, k);
    double uc[NV];
#pragma unroll
    for (int v = 0; v < NV; ++v) uc[v] = cell[v * g.vstride];
    const double coef = beta * tm->dt;
    for (int e = ff_first[c]; e < ff_first[c + 1]; ++e) {
      const FineFace rec = ff[e];
      const int d = rec.face >> 1, s = rec.face & 1;
      if (cc[d] != (s ? n[d] - 1 : 0)) continue;
      touched = true;
      const int t1 = d == 0 ? 1 : 0, t2 = d == 2 ? 1 : 2;
      const int a1 = cc[t1], a2 = cc[t2];
      const int h1 = a1 >= n[t1] / 2, h2 = a2 >= n[t2] / 2;
      const int fs = rec.fine_slot[h1 + 2 * h2];
      const int f1 = 2 * a1 - h1 * n[t1], f2 = 2 * a2 - h2 * n[t2];
      const double sg = s ? 1.0 : -1.0;
      for (int v = 0; v < NV; ++v) {
        const double own = fbuf[(int64_t)rec.own_slot * fsz + ((int64_t)v * n[t2] + a2) * n[t1] + a1];
        const double* fb = fbuf + (int64_t)fs * fsz + (int64_t)v * n[t2] * n[t1];
        const double fine = 0.25 * ((fb[f2 * n[t1] + f1] + fb[f2 * n[t1] + f1 + 1]) +
                                    (fb[(f2 + 1) * n[t1] + f1] + fb[(f2 + 1) * n[t1] + f1 + 1]));
        uc[v] += sg * coef * (own - fine) * bi.idx[d];
      }
    }
    if (touched) {
#pragma unroll
      for (int v = 0; v < NV; ++v) cell[v * g.vstride] = uc[v];
      if (do_dt) {
        double wn[NV];
        bad = !to_prim(uc, g.gamma, wn);
        const double cs = sqrt(g.gamma * wn[4] / wn[0]);
        smax = fmax(fmax((fabs(wn[1]) + cs) * bi.idx[0], (fabs(wn[2]) + cs) * bi.idx[1]),
                    (fabs(wn[3]) + cs) * bi.idx[2]);
      }
    }
  }
  if (do_dt) {
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) smax = fmax(smax, __shfl_xor(smax, off));
    if ((threadIdx.x & 63) == 0) sRed[threadIdx.x >> 6] = smax;
    __syncthreads();
    if (threadIdx.x == 0) {
      const double mx = fmax(fmax(sRed[0], sRed[1]), fmax(sRed[2], sRed[3]));
      atomicMax(&tm->smax_bits, (unsigned long long)__double_as_longlong(mx));
    }
  }
  if (bad) atomicOr(&tm->err, 1);
}

hipError_t launch_flux_correct(double* u, const BlockInfo* blocks, const FineFace* ff,
                               const int32_t* ff_first, const int32_t* cblocks, int32_t ncblocks,
                               const Geom& g, DevTime* tm, double beta, int32_t do_dt,
                               const double* fbuf, hipStream_t s) {
  if (ncblocks == 0) return hipSuccess;
  const int ncell = g.n1 * g.n2 * g.n3;
  dim3 grid((ncell + 255) / 256, ncblocks);
  hipLaunchKernelGGL(flux_correct_kernel, grid, dim3(256), 0, s, u, blocks, ff, ff_first, cblocks,
                     g, tm, beta, do_dt, fbuf);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// CFL reduction over the active cells (after exchange / regrid / upload).
// ---------------------------------------------------------------------------

__global__ void __launch_bounds__(256) dt_kernel(const double* u, const BlockInfo* blocks,
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
    const double* cell = u + (int64_t)b * g.bstride + pad_index(g, i, j, k);
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
    atomicMax(&tm->smax_bits, (unsigned long long)__double_as_longlong(mx));
  }
  if (bad) atomicOr(&tm->err, 1);
}

hipError_t launch_dt(const double* u, const BlockInfo* blocks, int32_t nblocks, const Geom& g,
                     DevTime* tm, hipStream_t s) {
  const int ncell = g.n1 * g.n2 * g.n3;
  dim3 grid((ncell + 255) / 256, nblocks);
  hipLaunchKernelGGL(dt_kernel, grid, dim3(256), 0, s, u, blocks, nblocks, g, tm);
  return hipGetLastError();
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
// Upload / download between the active-only layout and padded blocks.
// ---------------------------------------------------------------------------

__global__ void __launch_bounds__(256) scatter_kernel(double* u, const double* src, int64_t total,
                                                      Geom g) {
  const int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (q >= total) return;
  const int i = q % g.n1;
  int64_t r = q / g.n1;
  const int j = r % g.n2;
  r /= g.n2;
  const int k = r % g.n3;
  r /= g.n3;  // r = block*5 + v
  u[r * g.vstride + pad_index(g, i, j, k)] = src[q];
}

__global__ void __launch_bounds__(256) gather_kernel(double* dst, const double* u, int64_t total,
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

hipError_t launch_scatter(double* u, const double* src, int32_t nblocks, const Geom& g,
                          hipStream_t s) {
  const int64_t total = (int64_t)nblocks * NV * g.n1 * g.n2 * g.n3;
  hipLaunchKernelGGL(scatter_kernel, dim3((unsigned)((total + 255) / 256)), dim3(256), 0, s, u, src,
                     total, g);
  return hipGetLastError();
}

hipError_t launch_gather(double* dst, const double* u, int32_t nblocks, const Geom& g,
                         hipStream_t s) {
  const int64_t total = (int64_t)nblocks * NV * g.n1 * g.n2 * g.n3;
  hipLaunchKernelGGL(gather_kernel, dim3((unsigned)((total + 255) / 256)), dim3(256), 0, s, dst, u,
                     total, g);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Conserved totals: per-block sums in a fixed order, then one workgroup sums
// the block partials in a fixed order (bitwise reproducible).
// ---------------------------------------------------------------------------

__global__ void __launch_bounds__(256) block_sum_kernel(double* partial, const double* u,
                                                        const BlockInfo* blocks, Geom g) {
  __shared__ double sh[NV][256];
  const int b = blockIdx.x;
  const BlockInfo bi = blocks[b];
  const int ncell = g.n1 * g.n2 * g.n3;
  double acc[NV] = {0, 0, 0, 0, 0};
  for (int q = threadIdx.x; q < ncell; q += 256) {
    const int i = q % g.n1, j = (q / g.n1) % g.n2, k = q / (g.n1 * g.n2);
    const double* cell = u + (int64_t)b * g.bstride + pad_index(g, i, j, k);
#pragma unroll
    for (int v = 0; v < NV; ++v) acc[v] += cell[v * g.vstride];
  }
#pragma unroll
  for (int v = 0; v < NV; ++v) sh[v][threadIdx.x] = acc[v];
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w)
#pragma unroll
      for (int v = 0; v < NV; ++v) sh[v][threadIdx.x] += sh[v][threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x < NV) {
    const double dV = 1.0 / (bi.idx[0] * bi.idx[1] * bi.idx[2]);
    partial[(int64_t)b * NV + threadIdx.x] = sh[threadIdx.x][0] * dV;
  }
}

__global__ void __launch_bounds__(256) final_sum_kernel(double* out, const double* partial,
                                                        int nblocks) {
  __shared__ double sh[NV][256];
  double acc[NV] = {0, 0, 0, 0, 0};
  for (int b = threadIdx.x; b < nblocks; b += 256)
#pragma unroll
    for (int v = 0; v < NV; ++v) acc[v] += partial[(int64_t)b * NV + v];
#pragma unroll
  for (int v = 0; v < NV; ++v) sh[v][threadIdx.x] = acc[v];
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w)
#pragma unroll
      for (int v = 0; v < NV; ++v) sh[v][threadIdx.x] += sh[v][threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x < NV) out[threadIdx.x] = sh[threadIdx.x][0];
}

hipError_t launch_totals(double* partial, double* out, const double* u, const BlockInfo* blocks,
                         int32_t nblocks, const Geom& g, hipStream_t s) {
  hipLaunchKernelGGL(block_sum_kernel, dim3(nblocks), dim3(256), 0, s, partial, u, blocks, g);
  hipLaunchKernelGGL(final_sum_kernel, dim3(1), dim3(256), 0, s, out, partial, nblocks);
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
  for (int v = 0; v < NV; ++v) {
    double val;
    if (kd == 0) {
      val = uold[(int64_t)s * g.bstride + v * g.vstride + pad_index(g, i, j, k)];
    } else if (kd == 1) {
      val = prolong_val(uold, bold, M, g, bn.level, J0, J1, J2, v, &err);
    } else {
      val = comp_val(uold, bold, M, g, bn.level, J0, J1, J2, v, &err);
    }
    dst[v * g.vstride] = val;
  }
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
