// pkh_stage.hip -- the stage kernel of the Euler cycle for gfx950.
//
// Method (Parthenon, arXiv:2202.12309, Sec. 4.1): one stage of the two-stage
// second-order finite-volume update, U_out = U_base - beta dt D(U_in), with
// donor-cell (predictor) or piecewise-linear MC-limited (corrector)
// reconstruction on primitive variables and HLLE fluxes with Einfeldt's
// Roe-averaged wave speeds, over every block of a mesh in one launch.
//
// Layout: every state array is [block][var][k][j][i] with ghost width 2 on
// each side, i (x) contiguous.
#include <math.h>

#include <algorithm>
#include <type_traits>

#include "pkh_amr.h"
#include "pkh_device.h"

// Launch options: the corrector prefetches the next plane's inputs and the
// U^n values of its next update one plane ahead (measured at 256^3: 0.94 ms
// against 1.11 ms with neither prefetch at three waves per SIMD); waves per
// SIMD the launch bounds ask for (PKH_CORR_WAVES_256: the corrector on
// 256-thread tiles of 32-cell rows, see stage_waves).
#ifndef PKH_CORR_PF
#define PKH_CORR_PF 1
#endif
#ifndef PKH_CORR_BPF
#define PKH_CORR_BPF 1
#endif
#ifndef PKH_CORR_WAVES
#define PKH_CORR_WAVES 2
#endif
#ifndef PKH_PRED_WAVES
#define PKH_PRED_WAVES 2
#endif
#ifndef PKH_CORR_WAVES_256
#define PKH_CORR_WAVES_256 3
#endif
// issue the next plane's loads after the update (1) or right after staging (0)
#ifndef PKH_PF_LATE
#define PKH_PF_LATE 1
#endif
// with PKH_PF_LATE: the halo loads start after the first face solve (1)
#ifndef PKH_PF_SPLIT
#define PKH_PF_SPLIT 1
#endif
// planes of inputs kept in flight ahead of the one being computed
#ifndef PKH_CORR_PFD
#define PKH_CORR_PFD 1
#endif
#ifndef PKH_PRED_PFD
#define PKH_PRED_PFD 1
#endif

namespace pkh {

// ---------------------------------------------------------------------------
// Stage kernel: U_out = U_base - beta*dt * D(U_in) over every block.
//
// A workgroup owns TJ rows of N1 cells of one block and streams through z.
// Each thread loads its own cell of every plane (and, with the others, the
// 2-cell halo of the tile), keeps its column's states in a register window
// for the z faces, and stages the plane's face-state inputs in LDS for the
// x and y faces, each of which is solved once. The predictor (donor cell)
// stages per-cell HLLE inputs (sqrt(rho), c, h) so no face recomputes them;
// the corrector stages primitives and reconstructs per face (PLM-MC). A
// cell is finished once its upper z face is known; its x/y divergence waits
// in a short register queue. Halo cells beyond a same-level face are read
// from the neighbour's active cells.
//
// S is the storage type of the state arrays: double, or float for FP32
// storage (values widened on load, every operation in FP64, the result
// rounded once when stored; the CFL reduction sees the stored value).
// ---------------------------------------------------------------------------

// LDS doubles one tile of a stage uses: the staged plane (NQ values per
// cell of (TJ+4) x (N1+4)), the x and y face fluxes, one slot per wave.
template <int RECON, int N1, int TJ>
constexpr int stage_lds_doubles() {
  return (RECON ? 5 : 8) * (TJ + 2 * NG) * (N1 + 2 * NG) + NV * TJ * (N1 + 1) + NV * (TJ + 1) * N1 +
         (N1 * TJ + 63) / 64;
}

// One tile (TJ rows of block blk starting at row j0) of a stage with
// timestep dt, in LDS at lds (stage_lds_doubles doubles); rot rotates which
// wave takes the tile's remainder faces; tid is the thread's index in the
// workgroup.
template <int RECON, int N1, int TJ, typename S = double>
__device__ __forceinline__ void stage_tile(const StageLaunch& a, int blk, int j0, int rot, double dt,
                                           double* __restrict__ lds, int tid) {
  constexpr int NT = N1 * TJ;
  constexpr int P1 = N1 + 2 * NG;
  constexpr int RW = TJ + 2 * NG;
  constexpr int PLANE = RW * P1;
  // halo cells the faces read: HW rows below and above the tile over the
  // active columns, and HW cells beyond each end of the interior rows (HW =
  // 2 for the piecewise-linear faces, 1 for donor cell)
  constexpr int HW = RECON ? 2 : 1;
  constexpr int NHALO = 2 * HW * N1 + 2 * HW * TJ;
  constexpr int NX = TJ * (N1 + 1);
  constexpr int NY = (TJ + 1) * N1;
  constexpr int LAG = RECON ? 1 : 0;  // z face m is computed at plane m + LAG
  constexpr int WN = RECON ? 4 : 2;   // z window length
  constexpr int QN = 1 + LAG;         // x/y divergence queue length
  constexpr int UQN = RECON ? 1 : 2;  // predictor: conserved own-cell queue length
  constexpr int NQ = RECON ? 5 : 8;   // staged values per cell
  constexpr int NWAVE = (NT + 63) / 64;
  constexpr bool PF = !RECON || PKH_CORR_PF;  // prefetch the next plane into registers
  constexpr bool BPF = RECON && PKH_CORR_BPF; // corrector: U^n of the next update one plane ahead
  constexpr int PFD = PF ? (RECON ? PKH_CORR_PFD : PKH_PRED_PFD) : 1;  // planes in flight
  static_assert(NT % 64 == 0, "whole waves");

  static_assert(stage_lds_doubles<RECON, N1, TJ>() == NQ * PLANE + NV * NX + NV * NY + NWAVE, "LDS layout");
  double(*__restrict__ sQ)[PLANE] = reinterpret_cast<double(*)[PLANE]>(lds);
  double(*__restrict__ sFx)[NX] = reinterpret_cast<double(*)[NX]>(lds + NQ * PLANE);
  double(*__restrict__ sFy)[NY] = reinterpret_cast<double(*)[NY]>(lds + NQ * PLANE + NV * NX);
  double* __restrict__ sRed = lds + NQ * PLANE + NV * NX + NV * NY;

  const Geom& g = a.g;
  const int ti = tid % N1, tj = tid / N1;

  const BlockInfo bi = load_uniform(a.blocks + blk);
  const double gam = g.gamma;
  const double gm1 = gam - 1.0;
  const double igm1 = 1.0 / gm1;
  const double coef = a.beta * dt;
  const int64_t vs = g.vstride;
  const S* __restrict__ in = static_cast<const S*>(a.uin) + (int64_t)blk * g.bstride;
  const S* base = static_cast<const S*>(a.ubase) + (int64_t)blk * g.bstride;
  S* out = static_cast<S*>(a.uout) + (int64_t)blk * g.bstride;
  const int n2 = g.n2, n3 = g.n3;
  const int j = j0 + tj;
  const int fsz = NV * max(max(g.n1 * n2, g.n1 * n3), n2 * n3);  // face slot stride
  double* fbuf = a.fbuf;
  const int32_t* nb27 = a.nbr ? a.nbr + (int64_t)blk * 27 : nullptr;
  // Cells beyond the block (the x halo of interior rows, the y halo rows of
  // the tiles at the block's y faces, the z planes before and after it) are
  // read from the active cells of the same-level face neighbours: the stage
  // kernels keep no ghost zones for same-level faces. A face to a leaf on
  // another level reads this block's ghost zone, which the fill kernel
  // writes. Offsets from this block's cell to the cell read instead:
  auto nbshift = [&](int q, int64_t within) -> int64_t {
    const int32_t nb = nb27 ? load_uniform(nb27 + q) : -1;
    return nb >= 0 ? (int64_t)(nb - blk) * g.bstride + within : 0;
  };
  // the state's row pitch g.p1 (at least N1 + 4; the LDS plane keeps P1)
  const int gp1 = g.p1;
  const int64_t dxl = nbshift(12, N1), dxr = nbshift(14, -N1);
  const int64_t dyl = j0 == 0 ? nbshift(10, (int64_t)n2 * gp1) : 0;
  const int64_t dyh = j0 + TJ == n2 ? nbshift(16, -(int64_t)n2 * gp1) : 0;
  const int64_t dzl = nbshift(4, (int64_t)n3 * g.p2 * gp1), dzh = nbshift(22, -(int64_t)n3 * g.p2 * gp1);
  // offset of plane p (row j0-2) of this block, or of the z neighbour's plane
  auto pofs = [&](int p) -> int64_t {
    return ((int64_t)(p + NG) * g.p2 + j0) * gp1 + (p < 0 ? dzl : (p >= n3 ? dzh : 0));
  };
  const int own = (tj + NG) * P1 + ti + NG;      // this thread's cell in the LDS plane
  const int own_g = (tj + NG) * gp1 + ti + NG;   // and in the state's plane

  FState w[WN];       // z window (column states)
  double uq[UQN][NV];  // predictor: conserved own-cell values awaiting their update
  double dq[QN][NV];  // x/y divergence awaiting the z faces
  double fzp[NV];
  // corrector: half MC z slopes of window cells 1 and 2, each formed once
  // when the cell above it enters the window
  double szp[NV], szc[NV];
  bool bad = false;
  double smax = 0.0;
  const int mask = bi.finer_mask;

#pragma unroll
  for (int s = 0; s < WN; ++s) w[s] = FState{1.0, 0.0, 0.0, 0.0, 1.0, 1.0, 1.0, 1.0};
#pragma unroll
  for (int s = 0; s < QN; ++s)
#pragma unroll
    for (int v = 0; v < NV; ++v) dq[s][v] = 0.0;
#pragma unroll
  for (int s = 0; s < UQN; ++s)
#pragma unroll
    for (int v = 0; v < NV; ++v) uq[s][v] = 0.0;
#pragma unroll
  for (int v = 0; v < NV; ++v) fzp[v] = szp[v] = szc[v] = 0.0;

  // stage one cell's inputs into LDS slot c; returns its state
  auto stage_cell = [&](const double u[NV], int c) {
    FState q;
    double wp[NV];
    bad |= !to_prim(u, gam, wp);
    q.r = wp[0];
    q.v0 = wp[1];
    q.v1 = wp[2];
    q.v2 = wp[3];
    q.p = wp[4];
    sQ[0][c] = q.r;
    sQ[1][c] = q.v0;
    sQ[2][c] = q.v1;
    sQ[3][c] = q.v2;
    sQ[4][c] = q.p;
    if constexpr (!RECON) {
      complete_state(q, gam, igm1);
      sQ[5][c] = q.sr;
      sQ[6][c] = q.c;
      sQ[7][c] = q.h;
    }
    return q;
  };
  // face states of the face between LDS cells cm (lower) and c0 (upper),
  // stride st between neighbours along the face normal
  auto face_states = [&](int c0, int st, FState& L, FState& R) {
    if constexpr (RECON) {
      double wl[NV], wr[NV];
#pragma unroll
      for (int v = 0; v < NV; ++v) {
        const double qm2 = sQ[v][c0 - 2 * st], qm1 = sQ[v][c0 - st], q0 = sQ[v][c0],
                     qp1 = sQ[v][c0 + st];
        wl[v] = qm1 + mc_half(qm1 - qm2, q0 - qm1);
        wr[v] = q0 - mc_half(q0 - qm1, qp1 - q0);
      }
      L = FState{wl[0], wl[1], wl[2], wl[3], wl[4], 0, 0, 0};
      R = FState{wr[0], wr[1], wr[2], wr[3], wr[4], 0, 0, 0};
      complete_state(L, gam, igm1);
      complete_state(R, gam, igm1);
    } else {
      const int cm = c0 - st;
      L = FState{sQ[0][cm], sQ[1][cm], sQ[2][cm], sQ[3][cm], sQ[4][cm], sQ[5][cm], sQ[6][cm], sQ[7][cm]};
      R = FState{sQ[0][c0], sQ[1][c0], sQ[2][c0], sQ[3][c0], sQ[4][c0], sQ[5][c0], sQ[6][c0], sQ[7][c0]};
    }
  };

  // Solve the face of direction D (0: x, 1: y; D < 0: the run-time
  // direction dir, one instruction stream for lanes of both) whose upper
  // cell is LDS slot c0; its flux goes to LDS slot fo, and to the
  // fine-coarse face buffer at slot fsl (if >= 0), offset o, when the face
  // borders a finer leaf. The arithmetic does not depend on D: the
  // pointwise physics rounds the same in every inlined copy.
  auto solve_face = [&](auto dirc, int dir, int c0, int fo, int fsl, int64_t o) {
    constexpr int D = decltype(dirc)::value;
    const int d = D >= 0 ? D : dir;
    FState L, R;
    double fl[NV];
    face_states(c0, d == 0 ? 1 : P1, L, R);
    hlle<D>(L, R, gm1, fl, d);
    double* dstf = d == 0 ? &sFx[0][fo] : &sFy[0][fo];
    const int vstr = d == 0 ? NX : NY;
#pragma unroll
    for (int v = 0; v < NV; ++v) dstf[v * vstr] = fl[v];
    if (fsl >= 0) {
      const int64_t vst = d == 0 ? (int64_t)n3 * n2 : (int64_t)n3 * N1;
#pragma unroll
      for (int v = 0; v < NV; ++v) fbuf[(int64_t)fsl * fsz + v * vst + o] = fl[v];
    }
  };

  // halo cell h of the plane (rows -HW..-1 and TJ..TJ+HW-1 of the tile
  // over the active columns, then the HW cells at each end of the interior
  // rows) -> its LDS slot
  // (pitch: P1 for the LDS plane, gp1 for the state)
  auto hcell_p = [&](int h, int pitch) {
    if (h < 2 * HW * N1) {
      const int r = h / N1, i = h - r * N1;  // r < HW: row r - HW, else row TJ + r - HW
      return (r < HW ? r + NG - HW : TJ + NG + r - HW) * pitch + NG + i;
    }
    const int hh = h - 2 * HW * N1, r = hh / (2 * HW), sc = hh - r * 2 * HW;
    return (r + NG) * pitch + (sc < HW ? sc + NG - HW : N1 + NG + sc - HW);
  };
  auto hcell = [&](int h) { return hcell_p(h, P1); };
  // offset from this block's cell to the one halo cell h is read from. The
  // offsets are captured by value so the per-lane choice is a select: taken
  // by reference, they live in scratch memory and every halo load waits for
  // a pointer load first.
  auto hshift = [dxl, dxr, dyl, dyh](int h) -> int64_t {
    const int64_t sy = h < HW * N1 ? dyl : dyh;
    const int64_t sx = ((h - 2 * HW * N1) % (2 * HW)) < HW ? dxl : dxr;
    return h < 2 * HW * N1 ? sy : sx;
  };
  constexpr int HMAX = PF ? (NHALO + NT - 1) / NT : 1;
  // this lane's halo cells: LDS slot, and offset of the cell read (slot plus
  // neighbour shift), formed once since neither changes from plane to plane
  int hslot[HMAX];
  int64_t hoff[HMAX];
#pragma unroll
  for (int hh = 0; hh < HMAX; ++hh) {
    const int h = min(tid + hh * NT, NHALO - 1);
    hslot[hh] = hcell(h);
    hoff[hh] = hshift(h) + hcell_p(h, gp1);
  }
  // ring of PFD planes in flight: plane p is staged from slot (p - p_first)
  // % PFD, which then receives plane p + PFD; the loop below is unrolled by
  // PFD so every slot index is a compile-time constant
  double pu[PFD][NV], ph[PFD][HMAX][NV];  // own and halo cells of planes ahead
  double ubn[PFD][NV];                    // corrector: U^n of the next updates
  const int p_first = -1 - LAG, p_end = n3 + 1 + LAG;
  // start the loads of plane pn into ring slot sl: the own cell, the halo
  auto prefetch_own = [&](int sl, int pn) {
    if (pn >= p_end) return;
    const S* pl = in + pofs(pn);
#pragma unroll
    for (int v = 0; v < NV; ++v) pu[sl][v] = pl[v * vs + own_g];
  };
  auto prefetch_halo = [&](int sl, int pn) {
    if (pn < 0 || pn >= n3) return;  // the halo is only read on the active planes
    const S* pl = in + pofs(pn);
#pragma unroll
    for (int hh = 0; hh < HMAX; ++hh) {
      const int h = tid + hh * NT;
      if (h < NHALO) {
#pragma unroll
        for (int v = 0; v < NV; ++v) ph[sl][hh][v] = pl[hoff[hh] + v * vs];
      }
    }
  };
  if constexpr (BPF) {
    // the update of cell c happens at plane p_first + 2 + 2 LAG + c
#pragma unroll
    for (int c = 0; c < PFD; ++c) {
      const int64_t oc = ((int64_t)(c + NG) * g.p2 + (j + NG)) * gp1 + ti + NG;
#pragma unroll
      for (int v = 0; v < NV; ++v) ubn[(2 + 2 * LAG + c) % PFD][v] = base[v * vs + oc];
    }
  }
  if constexpr (PF) {
#pragma unroll
    for (int sl = 0; sl < PFD; ++sl) {
      const S* pl = in + pofs(p_first + sl);
#pragma unroll
      for (int v = 0; v < NV; ++v) pu[sl][v] = pl[v * vs + own_g];
      // the halo is only read on the active planes
      const bool act = p_first + sl >= 0 && p_first + sl < n3;
#pragma unroll
      for (int hh = 0; hh < HMAX; ++hh) {
        const int h = tid + hh * NT;
#pragma unroll
        for (int v = 0; v < NV; ++v)
          ph[sl][hh][v] = (act && h < NHALO) ? pl[hoff[hh] + v * vs] : 1.0;
      }
    }
  }

  for (int pb = p_first; pb < p_end; pb += PFD)
#pragma unroll
  for (int sl = 0; sl < PFD; ++sl) {
    const int p = pb + sl;
    if (p >= p_end) break;  // plane count not a multiple of PFD (uniform)
    // --- stage plane p (rows j0-2 .. j0+TJ+1): own cell first, then halo.
    // The predictor takes plane p from registers loaded while plane p-1 was
    // being computed and starts the loads of plane p+1 right away.
    {
      double u[NV];
      if constexpr (PF) {
#pragma unroll
        for (int v = 0; v < NV; ++v) u[v] = pu[sl][v];
      } else {
        const S* pl = in + pofs(p);
#pragma unroll
        for (int v = 0; v < NV; ++v) u[v] = pl[v * vs + own_g];
      }
      const FState q = stage_cell(u, own);
#pragma unroll
      for (int s = 0; s < WN - 1; ++s) w[s] = w[s + 1];
      w[WN - 1] = q;
      if constexpr (RECON) {
        const double a1[NV] = {w[1].r, w[1].v0, w[1].v1, w[1].v2, w[1].p};
        const double a2[NV] = {w[2].r, w[2].v0, w[2].v1, w[2].v2, w[2].p};
        const double a3[NV] = {w[3].r, w[3].v0, w[3].v1, w[3].v2, w[3].p};
#pragma unroll
        for (int v = 0; v < NV; ++v) {
          szp[v] = szc[v];
          szc[v] = mc_half(a2[v] - a1[v], a3[v] - a2[v]);
        }
      }
      if constexpr (!RECON) {
#pragma unroll
        for (int s = 0; s < UQN - 1; ++s)
#pragma unroll
          for (int v = 0; v < NV; ++v) uq[s][v] = uq[s + 1][v];
#pragma unroll
        for (int v = 0; v < NV; ++v) uq[UQN - 1][v] = u[v];
      }
    }
    if constexpr (PF) {
      if (p >= 0 && p < n3) {
#pragma unroll
        for (int hh = 0; hh < HMAX; ++hh) {
          const int h = tid + hh * NT;
          if (h < NHALO) stage_cell(ph[sl][hh], hslot[hh]);
        }
      }
      if (!PKH_PF_LATE) {
        prefetch_own(sl, p + PFD);
        prefetch_halo(sl, p + PFD);
      }
    } else {
      const int64_t po = pofs(p);
      for (int h = tid; h < NHALO && p >= 0 && p < n3; h += NT) {
        double u[NV];
        const int c = hcell(h);
        const int64_t hs = hshift(h) + hcell_p(h, gp1);
#pragma unroll
        for (int v = 0; v < NV; ++v) u[v] = in[po + hs + v * vs];
        stage_cell(u, c);
      }
    }
    __syncthreads();

    // --- z face m between cells m-1 and m, then finish cell m-1
    const int m = p - LAG;
    if (m >= 0 && m <= n3) {
      FState L, R;
      double fz[NV];
      if constexpr (RECON) {
        const double c1[NV] = {w[1].r, w[1].v0, w[1].v1, w[1].v2, w[1].p};
        const double c2[NV] = {w[2].r, w[2].v0, w[2].v1, w[2].v2, w[2].p};
        double wl[NV], wr[NV];
#pragma unroll
        for (int v = 0; v < NV; ++v) {
          wl[v] = c1[v] + szp[v];
          wr[v] = c2[v] - szc[v];
        }
        L = FState{wl[0], wl[1], wl[2], wl[3], wl[4], 0, 0, 0};
        R = FState{wr[0], wr[1], wr[2], wr[3], wr[4], 0, 0, 0};
        complete_state(L, gam, igm1);
        complete_state(R, gam, igm1);
      } else {
        L = w[0];
        R = w[1];
      }
      hlle<2>(L, R, gm1, fz);
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
        const int64_t o = ((int64_t)(k + NG) * g.p2 + (j + NG)) * gp1 + ti + NG;
        double un[NV];
#pragma unroll
        for (int v = 0; v < NV; ++v) {
          const double du = dq[0][v] + (fz[v] - fzp[v]) * bi.idx[2];
          const double ub = RECON ? (BPF ? ubn[sl][v] : base[v * vs + o]) : uq[0][v];
          const S st = static_cast<S>(ub - coef * du);
          out[v * vs + o] = st;
          un[v] = static_cast<double>(st);
        }
        if constexpr (BPF) {
          if (k + PFD < n3) {
#pragma unroll
            for (int v = 0; v < NV; ++v) ubn[sl][v] = base[v * vs + o + (int64_t)PFD * g.p2 * gp1];
          }
        }
        if (a.do_dt) {
          const bool skip = ((mask >> XLO) & 1 && ti == 0) || ((mask >> XHI) & 1 && ti == N1 - 1) ||
                            ((mask >> YLO) & 1 && j == 0) || ((mask >> YHI) & 1 && j == n2 - 1) ||
                            ((mask >> ZLO) & 1 && k == 0) || ((mask >> ZHI) & 1 && k == n3 - 1);
          if (!skip) {
            double wn[NV];
            bad |= !to_prim(un, gam, wn);
            const double cs = fsqrt(gam * wn[4] * frcp(wn[0]));
            const double sv = fmax(fmax((fabs(wn[1]) + cs) * bi.idx[0], (fabs(wn[2]) + cs) * bi.idx[1]),
                                   (fabs(wn[3]) + cs) * bi.idx[2]);
            smax = fmax(smax, sv);
          }
        }
      }
#pragma unroll
      for (int v = 0; v < NV; ++v) fzp[v] = fz[v];
    }
    // Loads of plane p + PFD start here, after the update, so the wait of
    // the update for its U^n values does not also wait for them; they land
    // while the x and y faces are solved.
    if constexpr (PF && PKH_PF_LATE) {
      prefetch_own(sl, p + PFD);
      if (!PKH_PF_SPLIT || p < 0 || p >= n3) prefetch_halo(sl, p + PFD);
    }
    // --- x and y faces of plane p, divergence into the queue.
    if (p >= 0 && p < n3) {
      // Each thread solves the lower x and y faces of its cell. The tile's
      // upper x faces (one per row) and upper y faces (one per column) go to
      // consecutive lanes starting at one wave, rotated with the plane and
      // the workgroup so that no SIMD always gets the extra work. A face
      // shared by two tiles or two blocks gets the same flux bit for bit on
      // both sides, whichever tile shape is used.
      const int wr = (rot + p + 2) % NWAVE;
      const int q = (tid - wr * 64 + NT) % NT;
      solve_face(std::integral_constant<int, 0>{}, 0, own, tj * (N1 + 1) + ti, ti == 0 ? bi.fslot[XLO] : -1,
                 (int64_t)p * n2 + j);
      if constexpr (PF && PKH_PF_LATE && PKH_PF_SPLIT) prefetch_halo(sl, p + PFD);
      solve_face(std::integral_constant<int, 1>{}, 1, own, tj * N1 + ti, j == 0 ? bi.fslot[YLO] : -1,
                 (int64_t)p * N1 + ti);
      if (q < TJ + N1) {
        const bool xf = q < TJ;
        const int iy = q - TJ;
        solve_face(std::integral_constant<int, -1>{}, xf ? 0 : 1,
                   xf ? (q + NG) * P1 + N1 + NG : (TJ + NG) * P1 + iy + NG, xf ? q * (N1 + 1) + N1 : TJ * N1 + iy,
                   xf ? bi.fslot[XHI] : (j0 + TJ == n2 ? bi.fslot[YHI] : -1),
                   xf ? (int64_t)p * n2 + j0 + q : (int64_t)p * N1 + iy);
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
    // no barrier here: the next plane's staging only overwrites the LDS
    // plane, whose last readers (this plane's x/y faces) finished before the
    // barrier above, and the next plane's fluxes are written after its first
    // barrier, which every wave reaches after this divergence
  }

  if (a.do_dt) {
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) smax = fmax(smax, __shfl_xor(smax, off));
    if ((tid & 63) == 0) sRed[tid >> 6] = smax;
    __syncthreads();
    if (tid == 0) {
      double mx = sRed[0];
      for (int q = 1; q < NWAVE; ++q) mx = fmax(mx, sRed[q]);
      reduce_max_speed(a.tm, mx);
    }
  }
  if (bad) atomicOr(&a.tm->err, 1);
}

// Waves per SIMD a stage variant is compiled for. The corrector on 256-thread
// tiles of 16- or 32-cell rows (16 x 16, 32 x 8) runs at three (a 168-VGPR
// cap with a few spilled values): more waves keep more loads in flight per
// CU. Measured at 256^3: in 32^3 blocks 0.722 ms against 0.758 ms at two
// waves with the same tiles and 0.754 ms for 16-row tiles at two; in 16^3
// blocks, on line-aligned rows, 0.722 against 0.789 ms. On 64-cell rows
// (64 x 4) the cap spills 54 registers: 1.33 ms against 0.785 ms at two.
// Everything else at two (the predictor, whose registers allow three
// anyway, is bound by its memory traffic; the other tile shapes spill more;
// four waves spill heavily).
template <int RECON, int N1, int TJ>
constexpr int stage_waves() {
  return (RECON && (N1 == 16 || N1 == 32) && N1 * TJ == 256) ? PKH_CORR_WAVES_256
                                                               : (RECON ? PKH_CORR_WAVES : PKH_PRED_WAVES);
}

// XCD-aware order: workgroups are dealt round-robin to the 8 XCDs; map
// consecutive items (tiles of a block, which share halo rows) to one XCD's L2.
__device__ __forceinline__ int xcd_order(int wg, int nwg) {
  return (nwg & 7) == 0 ? (wg & 7) * (nwg >> 3) + (wg >> 3) : wg;
}

// Occupancy: both stages keep the next plane's loads in flight in registers
// and run at two waves per SIMD.
template <int RECON, int N1, int TJ>
__global__ void __launch_bounds__(N1 * TJ, (stage_waves<RECON, N1, TJ>())) stage_kernel(StageLaunch a) {
  const int ntj = a.g.n2 / TJ;
  const int wg = xcd_order(blockIdx.x, gridDim.x);
  const int blk = wg / ntj;
  if (blk >= a.nblocks) return;
  __shared__ double lds[stage_lds_doubles<RECON, N1, TJ>()];
  stage_tile<RECON, N1, TJ>(a, a.b0 + blk, (wg - blk * ntj) * TJ, wg, a.tm->dt, lds, (int)threadIdx.x);
}

// The same over a state stored in FP32.
template <int RECON, int N1, int TJ>
__global__ void __launch_bounds__(N1 * TJ, (stage_waves<RECON, N1, TJ>())) stage_kernel_f32(StageLaunch a) {
  const int ntj = a.g.n2 / TJ;
  const int wg = xcd_order(blockIdx.x, gridDim.x);
  const int blk = wg / ntj;
  if (blk >= a.nblocks) return;
  __shared__ double lds[stage_lds_doubles<RECON, N1, TJ>()];
  stage_tile<RECON, N1, TJ, float>(a, a.b0 + blk, (wg - blk * ntj) * TJ, wg, a.tm->dt, lds, (int)threadIdx.x);
}

// Grouped launch: the tiles of many independent meshes (same block width
// and tile) in one grid; items[w] names the mesh, block and first row.
template <int RECON, int N1, int TJ>
__global__ void __launch_bounds__(N1 * TJ, (stage_waves<RECON, N1, TJ>())) stage_group_kernel(const StageLaunch* insts,
                                                                 const GroupItem* items, int nitems) {
  const int wg = xcd_order(blockIdx.x, gridDim.x);
  if (wg >= nitems) return;
  const GroupItem it = items[wg];
  __shared__ double lds[stage_lds_doubles<RECON, N1, TJ>()];
  const StageLaunch& a = insts[it.inst];
  stage_tile<RECON, N1, TJ>(a, it.blk, it.j0, wg, a.tm->dt, lds, (int)threadIdx.x);
}

// ---- end of the stage kernels (the persistent batch kernel follows) ----

// ---------------------------------------------------------------------------
// Persistent batch kernel. Each instance is pinned to one XCD; a workgroup
// reads the id of the XCD it runs on and takes tickets from that XCD's
// counter: ticket t is item t % nper of cycle t / nper of the XCD's list,
// whose items are ordered by phase, then instance. An item waits (thread 0,
// bounded) for the previous phase of its instance in the same cycle, or for
// the instance's clock to reach the cycle, i.e. only for items of smaller
// tickets of the same counter, held by running workgroups: no deadlock
// whatever the grid. Visibility: every thread waits for its stores to
// complete, then thread 0 makes them visible at device scope (release)
// before the item is counted, and a consumer's thread 0 acquires at device
// scope after its wait. Pinning an instance to one XCD keeps its blocks in
// one L2 between items; the fences stay device-scope all the same:
// variants whose acquire only dropped the CU's L1 (with the release at
// device scope or only the stores' completion) gave wrong results on
// small instances after a few cycles, so the pinning alone does not make
// an instance's items see each other's stores, and they are not kept.
// ---------------------------------------------------------------------------

__device__ __forceinline__ unsigned int ld_relaxed(const unsigned int* p) {
  return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Id of the XCD (chiplet, own L2) this wave runs on.
__device__ __forceinline__ int xcc_id() {
  unsigned x;
  asm volatile("s_getreg_b32 %0, hwreg(HW_REG_XCC_ID, 0, 4)" : "=s"(x));
  return (int)x;
}

// This thread's global stores are complete (the L1 writes through to the L2).
__device__ __forceinline__ void stores_done() { asm volatile("s_waitcnt vmcnt(0)" ::: "memory"); }

// Release (thread 0, after every thread's stores completed and a barrier):
// the workgroup's stores become visible at device scope before the item is
// counted. Acquire (thread 0, after its wait): later loads of the workgroup
// see what the awaited items stored.
__device__ __forceinline__ void item_release() { __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent"); }
__device__ __forceinline__ void item_acquire() { __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent"); }

// Wait until *p >= target; false when *err is set or wait_ticks of the
// device wall clock pass first.
__device__ bool persistent_wait(const unsigned int* p, unsigned int target, const int* err, long long wait_ticks) {
  if (ld_relaxed(p) >= target) return true;
  const long long t0 = (long long)wall_clock64();
  for (;;) {
    if (__hip_atomic_load(err, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)) return false;
    if ((long long)wall_clock64() - t0 > wait_ticks) return false;
    __builtin_amdgcn_s_sleep(4);
    if (ld_relaxed(p) >= target) return true;
  }
}

// Close a cycle of one instance and open the next (the batched clock with
// no end time): dt_next = CFL / max signal speed, t += dt, cycle + 1,
// dt = dt_next, reduction reset. Every field goes through atomics, which
// are performed in the L2 the instance's workgroups share.
__device__ void persistent_clock(DevTime* tm) {
  const unsigned long long sb = __hip_atomic_load(&tm->smax_bits, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  const double cfl = __hip_atomic_load(&tm->cfl, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  const double t = __hip_atomic_load(&tm->t, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  const double dt = __hip_atomic_load(&tm->dt, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  const long long cyc = __hip_atomic_load(&tm->cycle, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  const double dt_next = cfl / __longlong_as_double((long long)sb);
  __hip_atomic_store(&tm->dt_next, dt_next, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  __hip_atomic_store(&tm->t, t + dt, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  __hip_atomic_store(&tm->cycle, cyc + 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  __hip_atomic_store(&tm->dt, dt_next, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  __hip_atomic_store(&tm->smax_bits, 0ull, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

constexpr int persistent_lds_doubles() {
  return std::max(std::max(stage_lds_doubles<0, 16, 16>(), stage_lds_doubles<1, 16, 16>()),
                  std::max(stage_lds_doubles<0, 32, 8>(), stage_lds_doubles<1, 32, 8>()));
}

template <int W>
__global__ void __launch_bounds__(256, W)
    persistent_kernel(const PInst* __restrict__ insts, int ninst, PSync* sync, const PItem* __restrict__ items,
                      const int32_t* __restrict__ slot_of, PCtl* ctl, int ncycles, long long wait_ticks) {
  __shared__ double lds[persistent_lds_doubles()];
  __shared__ double s_red[4];
  __shared__ unsigned int s_ticket;
  __shared__ double s_dt;
  __shared__ int s_ok;
  const int tid = threadIdx.x;
  const int slot = slot_of[xcc_id() & (PMAX_XCC - 1)];
  if (slot < 0) return;  // no instance lives on this XCD (uniform per workgroup)
  PCtl* q = ctl + slot;
  int* err = &ctl[0].err;
  const unsigned int nper = (unsigned int)q->nper;
  const unsigned int total = nper * (unsigned int)ncycles;
  const PItem* qitems = items + q->off;
  for (;;) {
    if (tid == 0) s_ticket = atomicAdd(&q->ticket, 1u);
    __syncthreads();
    // the item and its instance's records are uniform: kept in SGPRs (a
    // value read from LDS or a generic load would sit in VGPRs, and so would
    // every address derived from it inside the tile)
    const unsigned int tk = __builtin_amdgcn_readfirstlane(s_ticket);
    if (tk >= total) break;  // uniform: every wave of the workgroup leaves
    const unsigned int c = tk / nper;
    const PItem it = load_uniform(qitems + (tk - c * nper));
    const PInst& in = insts[it.inst];
    PSync* ps = sync + it.inst;
    if (tid == 0) {
      int prev = it.phase - 1;
      while (prev >= 0 && in.cnt[prev] == 0) --prev;
      const bool ok = prev < 0 ? persistent_wait(&ps->clock, c, err, wait_ticks)
                               : persistent_wait(&ps->done[prev], (c + 1) * (unsigned int)in.cnt[prev], err,
                                                 wait_ticks);
      if (!ok && atomicCAS(err, 0, 1) == 0) {
        // the first to give up marks every instance's state invalid
        for (int r = 0; r < ninst; ++r) atomicOr(&insts[r].st[0].tm->err, 4);
      }
      item_acquire();
      s_ok = ok;
      s_dt = __hip_atomic_load(&in.st[0].tm->dt, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
    __syncthreads();
    if (__builtin_amdgcn_readfirstlane(s_ok)) {
      const long long dtb = __double_as_longlong(s_dt);
      const double dt = __longlong_as_double(
          ((long long)__builtin_amdgcn_readfirstlane((int)(dtb >> 32)) << 32) |
          (unsigned int)__builtin_amdgcn_readfirstlane((int)dtb));
      const int ph = it.phase;
      if (ph == 0 || ph == 3) {
        const StageLaunch& a = in.st[ph == 3];
        // the thread index as an opaque value: the per-lane set-up of each
        // tile variant is then formed per item instead of being hoisted out
        // of the item loop, where it would hold VGPRs for every variant
        int ltid = tid;
        asm volatile("" : "+v"(ltid));
        const int n1 = in.n1;
        if (n1 == 32) {
          if (a.recon)
            stage_tile<1, 32, 8>(a, it.a, it.b, (int)tk, dt, lds, ltid);
          else
            stage_tile<0, 32, 8>(a, it.a, it.b, (int)tk, dt, lds, ltid);
        } else {
          if (a.recon)
            stage_tile<1, 16, 16>(a, it.a, it.b, (int)tk, dt, lds, ltid);
          else
            stage_tile<0, 16, 16>(a, it.a, it.b, (int)tk, dt, lds, ltid);
        }
      } else if (ph == 1 || ph == 4) {
        const StageLaunch& a = in.st[ph == 4];
        double* u = static_cast<double*>(a.uout);
        flux_correct_item(u, a.blocks, in.ff, in.ff_first, in.cblocks, a.g, a.tm, dt, a.beta, ph == 4, a.fbuf,
                          it.a, it.b, s_red);
      } else {
        const StageLaunch& a = in.st[ph == 5];
        fill_faces_item(static_cast<double*>(a.uout), a.g, a.tm, in.jf, in.plan, it.a, it.b);
      }
      // every thread's stores complete, then one release before the item
      // is counted
      stores_done();
      __syncthreads();
      if (tid == 0) {
        item_release();
        const unsigned int old = atomicAdd(&ps->done[ph], 1u);
        if (ph == in.last && old + 1 == (c + 1) * (unsigned int)in.cnt[ph]) {
          item_acquire();
          persistent_clock(in.st[0].tm);
          stores_done();
          item_release();
          __hip_atomic_store(&ps->clock, c + 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        }
      }
    }
    __syncthreads();  // s_ticket, s_ok and s_dt are rewritten next round
  }
}

__global__ void persistent_reset_kernel(PSync* sync, int ninst, PCtl* ctl, int nslots) {
  const int q = blockIdx.x * blockDim.x + threadIdx.x;
  if (q < ninst) sync[q] = PSync{};
  if (q < nslots) {
    ctl[q].ticket = 0u;
    ctl[q].err = 0;
  }
}

// Each workgroup records the XCD it runs on.
__global__ void xcc_probe_kernel(int32_t* seen) {
  if (threadIdx.x == 0) seen[xcc_id() & (PMAX_XCC - 1)] = 1;
}

// ---- host-side launchers: everything below runs on the host ----

template <int RECON, int N1, int TJ>
static hipError_t launch_group_t(const StageLaunch* insts, const GroupItem* items, int nitems,
                                 hipStream_t s) {
  const int nwg = (nitems + 7) / 8 * 8;
  hipLaunchKernelGGL((stage_group_kernel<RECON, N1, TJ>), dim3((unsigned)nwg), dim3(N1 * TJ), 0, s, insts,
                     items, nitems);
  return hipGetLastError();
}

template <int RECON, int N1, int TJ>
static hipError_t launch_stage_t(const StageLaunch& a, hipStream_t s) {
  const int ntj = a.g.n2 / TJ;
  int64_t nwg = (int64_t)a.nblocks * ntj;
  nwg = (nwg + 7) / 8 * 8;
  hipLaunchKernelGGL((stage_kernel<RECON, N1, TJ>), dim3((unsigned)nwg), dim3(N1 * TJ), 0, s, a);
  return hipGetLastError();
}

template <int RECON, int N1, int TJ>
static hipError_t launch_stage_f32_t(const StageLaunch& a, hipStream_t s) {
  const int ntj = a.g.n2 / TJ;
  int64_t nwg = (int64_t)a.nblocks * ntj;
  nwg = (nwg + 7) / 8 * 8;
  hipLaunchKernelGGL((stage_kernel_f32<RECON, N1, TJ>), dim3((unsigned)nwg), dim3(N1 * TJ), 0, s, a);
  return hipGetLastError();
}

template <int N1, int TJ>
static hipError_t launch_stage_n(const StageLaunch& a, hipStream_t s) {
  return a.recon ? launch_stage_t<1, N1, TJ>(a, s) : launch_stage_t<0, N1, TJ>(a, s);
}

hipError_t launch_stage_group(int recon, int n1, int tj, const StageLaunch* insts,
                              const GroupItem* items, int nitems, hipStream_t s) {
  if (nitems <= 0) return hipSuccess;
#define PKH_G(N1_, TJ_)                                                                 \
  case N1_ * 100 + TJ_:                                                                 \
    return recon ? launch_group_t<1, N1_, TJ_>(insts, items, nitems, s)                 \
                 : launch_group_t<0, N1_, TJ_>(insts, items, nitems, s);
  switch (n1 * 100 + tj) {
    PKH_G(8, 8)
    PKH_G(16, 8)
    PKH_G(16, 16)
    PKH_G(16, 4)
    PKH_G(32, 8)
    PKH_G(32, 4)
    PKH_G(32, 16)
    PKH_G(64, 4)
    PKH_G(64, 2)
    default:
      return hipErrorInvalidValue;
  }
#undef PKH_G
}

hipError_t launch_stage(const StageLaunch& a, hipStream_t s) {
  const int tj = stage_tile_rows(a.g.n1, a.g.n2, a.tj, a.nblocks, a.recon);
  if (a.fp32) {  // FP32 storage: blocks of 16 or 32 cells per row, 8 or 16 rows
    switch (a.g.n1 * 100 + tj) {
      case 1608:
        return a.recon ? launch_stage_f32_t<1, 16, 8>(a, s) : launch_stage_f32_t<0, 16, 8>(a, s);
      case 1616:
        return a.recon ? launch_stage_f32_t<1, 16, 16>(a, s) : launch_stage_f32_t<0, 16, 16>(a, s);
      case 3208:
        return a.recon ? launch_stage_f32_t<1, 32, 8>(a, s) : launch_stage_f32_t<0, 32, 8>(a, s);
      case 3216:
        return a.recon ? launch_stage_f32_t<1, 32, 16>(a, s) : launch_stage_f32_t<0, 32, 16>(a, s);
      default:
        return hipErrorInvalidValue;
    }
  }
  switch (a.g.n1 * 100 + tj) {
    case 808:
      return launch_stage_n<8, 8>(a, s);
    case 1608:
      return launch_stage_n<16, 8>(a, s);
    case 1616:
      return launch_stage_n<16, 16>(a, s);
    case 1604:
      return launch_stage_n<16, 4>(a, s);
    case 3208:
      return launch_stage_n<32, 8>(a, s);
    case 3204:
      return launch_stage_n<32, 4>(a, s);
    case 3216:
      return launch_stage_n<32, 16>(a, s);
    case 6404:
      return launch_stage_n<64, 4>(a, s);
    case 6402:
      return launch_stage_n<64, 2>(a, s);
    default:
      return hipErrorInvalidValue;
  }
}


int persistent_grid(int waves) {
  int dev = 0, ncu = 0, per = 0;
  if (hipGetDevice(&dev) != hipSuccess ||
      hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess)
    return -1;
  hipError_t e = waves == 3
                     ? hipOccupancyMaxActiveBlocksPerMultiprocessor(&per, persistent_kernel<3>, 256, 0)
                     : hipOccupancyMaxActiveBlocksPerMultiprocessor(&per, persistent_kernel<2>, 256, 0);
  if (e != hipSuccess || per < 1) return -1;
  return per * ncu;
}

hipError_t launch_persistent(const PInst* insts, int32_t ninst, PSync* sync, const PItem* items,
                             const int32_t* slot_of, PCtl* ctl, int32_t nslots, int32_t ncycles, int waves,
                             int grid, long long wait_ticks, hipStream_t s) {
  if (ninst < 1 || nslots < 1 || ncycles < 1 || grid < 1) return hipErrorInvalidValue;
  const int nr = std::max<int>(ninst, nslots);
  hipLaunchKernelGGL(persistent_reset_kernel, dim3((nr + 255) / 256), dim3(256), 0, s, sync, (int)ninst, ctl,
                     (int)nslots);
  if (waves == 3)
    hipLaunchKernelGGL(persistent_kernel<3>, dim3(grid), dim3(256), 0, s, insts, (int)ninst, sync, items, slot_of,
                       ctl, (int)ncycles, wait_ticks);
  else
    hipLaunchKernelGGL(persistent_kernel<2>, dim3(grid), dim3(256), 0, s, insts, (int)ninst, sync, items, slot_of,
                       ctl, (int)ncycles, wait_ticks);
  return hipGetLastError();
}

hipError_t probe_xcc(int32_t* dev_buf, int32_t* out_host, hipStream_t s) {
  hipError_t e = hipMemsetAsync(dev_buf, 0, PMAX_XCC * sizeof(int32_t), s);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(xcc_probe_kernel, dim3(4096), dim3(64), 0, s, dev_buf);
  if ((e = hipGetLastError()) != hipSuccess) return e;
  if ((e = hipMemcpyAsync(out_host, dev_buf, PMAX_XCC * sizeof(int32_t), hipMemcpyDeviceToHost, s)) != hipSuccess)
    return e;
  return hipStreamSynchronize(s);
}

}  // namespace pkh
