// pkh_amr.h -- device code of the multilevel parts of the cycle shared by
// the kernels that run them on their own and the persistent batch kernel:
// composite-field lookups (restriction of finer leaves, prolongation from
// coarser ones, wall images), the ghost face fill across level jumps and
// walls, and the fine-coarse flux correction (Parthenon Sec. 3.7).
#pragma once

#include "pkh_device.h"

namespace pkh {

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

// Where the composite value at level L of a global cell J inside the domain
// lives: x the leaf, y the padded index of the cell in it (LOC_CELL bits) —
// the cell of the leaf at level L, or while regridding the containing cell
// of a coarser leaf (injection) — or, with LOC_RESTRICT set, the first of
// the 8 level-(L+1) cells whose mean it is (they lie in one leaf: blocks
// have even edges). x = LOC_NONE when the mesh has no such cell. Bits 29-31
// of y are free for the caller (the image's reflected directions).
constexpr unsigned LOC_NONE = 0xffffffffu, LOC_RESTRICT = 1u << 28, LOC_CELL = LOC_RESTRICT - 1u;

__device__ inline uint2 comp_loc(const BlockInfo* blocks, const LevelMaps& M, const Geom& g, int L, const int J[3]) {
  const int n[3] = {g.n1, g.n2, g.n3};
  const int b[3] = {J[0] / n[0], J[1] / n[1], J[2] / n[2]};
  int32_t id = leaf_at(M, L, b[0], b[1], b[2]);
  if (id >= 0)
    return make_uint2((unsigned)id,
                      (unsigned)pad_index(g, J[0] - b[0] * n[0], J[1] - b[1] * n[1], J[2] - b[2] * n[2]));
  for (int Lc = L - 1; Lc >= 0; --Lc) {
    const int sh = L - Lc;
    id = leaf_at(M, Lc, b[0] >> sh, b[1] >> sh, b[2] >> sh);
    if (id >= 0) {
      const BlockInfo bc = blocks[id];
      return make_uint2((unsigned)id, (unsigned)pad_index(g, (J[0] >> sh) - bc.lx * n[0],
                                                          (J[1] >> sh) - bc.ly * n[1], (J[2] >> sh) - bc.lz * n[2]));
    }
  }
  if (L + 1 > M.maxl) return make_uint2(LOC_NONE, 0u);
  const int F0 = 2 * J[0], F1 = 2 * J[1], F2 = 2 * J[2];
  const int32_t fid = leaf_at(M, L + 1, F0 / n[0], F1 / n[1], F2 / n[2]);
  if (fid < 0) return make_uint2(LOC_NONE, 0u);
  const BlockInfo bf = blocks[fid];
  return make_uint2((unsigned)fid,
                    (unsigned)pad_index(g, F0 - bf.lx * n[0], F1 - bf.ly * n[1], F2 - bf.lz * n[2]) | LOC_RESTRICT);
}

// The five values at a location from comp_loc: the cell's, or the mean of
// the 8 fine cells summed in pairs along x, then y, then z.
__device__ __forceinline__ void comp_gather(const double* u, const Geom& g, uint2 e, double out[NV], int* err) {
  if (e.x == LOC_NONE) {
    *err = 1;
#pragma unroll
    for (int v = 0; v < NV; ++v) out[v] = 0.0;
    return;
  }
  const double* c = u + (int64_t)e.x * g.bstride + (e.y & LOC_CELL);
  if (!(e.y & LOC_RESTRICT)) {
#pragma unroll
    for (int v = 0; v < NV; ++v) out[v] = c[v * g.vstride];
    return;
  }
  const int64_t sx = 1, sy = g.p1, sz = (int64_t)g.p1 * g.p2;
#pragma unroll
  for (int v = 0; v < NV; ++v) {
    const double* f = c + (int64_t)v * g.vstride;
    out[v] = 0.125 * (((f[0] + f[sx]) + (f[sy] + f[sy + sx])) + ((f[sz] + f[sz + sx]) + (f[sz + sy] + f[sz + sy + sx])));
  }
}

// Composite value at level L of a global cell J inside the domain, all five
// variables: leaf value at level L; restriction of the level-(L+1) leaves;
// or, while regridding, the containing coarser cell (injection).
__device__ inline void comp_val_inside(const double* u, const BlockInfo* blocks, const LevelMaps& M, const Geom& g,
                                int L, const int J[3], double out[NV], int* err) {
  comp_gather(u, g, comp_loc(blocks, M, g, L, J), out, err);
}

// Global cell J of level L (at most one domain length outside) brought into
// the domain: wrapped along periodic directions; beyond an outflow face the
// nearest cell inside, beyond a reflecting face the mirror image. Returns
// the reflected directions in bits 0-2 (the image's momentum along them
// changes sign) and bit 3 when J was moved across a wall.
__device__ __forceinline__ int cell_in_domain(const Geom& g, int L, int J[3]) {
  const int n[3] = {g.n1, g.n2, g.n3};
  int code = 0;
#pragma unroll
  for (int d = 0; d < 3; ++d) {
    const int N = (g.nrb[d] * n[d]) << L;
    if (g.bc[2 * d] == BC_PERIODIC) {
      J[d] = wrap_i(J[d], N);
    } else if (J[d] < 0 || J[d] >= N) {
      const int hi = J[d] >= N;
      code |= 8;
      if (g.bc[2 * d + hi] == BC_OUTFLOW) {
        J[d] = hi ? N - 1 : 0;
      } else {
        J[d] = hi ? 2 * N - 1 - J[d] : -1 - J[d];
        code |= 1 << d;
      }
    }
  }
  return code;
}

// Momentum signs of an image reflected along the directions in code.
__device__ __forceinline__ void apply_image_signs(int code, double out[NV]) {
#pragma unroll
  for (int d = 0; d < 3; ++d)
    if ((code >> d) & 1) out[1 + d] = -out[1 + d];
}

// Composite value at level L, global cell J (any integers within a domain
// length; brought into the domain here): beyond a wall, the value of the
// image cell with its momentum signs.
__device__ inline void comp_val(const double* u, const BlockInfo* blocks, const LevelMaps& M, const Geom& g, int L,
                         int J0, int J1, int J2, double out[NV], int* err) {
  int J[3] = {J0, J1, J2};
  const int code = cell_in_domain(g, L, J);
  comp_val_inside(u, blocks, M, g, L, J, out, err);
  apply_image_signs(code, out);
}

// Linear prolongation to fine cell F (level L) from the composite field at
// level L-1 with minmod slopes, all five variables; the fine centre sits a
// quarter coarse width from the coarse centre along each axis.
__device__ inline void prolong_val(const double* u, const BlockInfo* blocks, const LevelMaps& M, const Geom& g, int L,
                            int F0, int F1, int F2, double out[NV], int* err) {
  const int I[3] = {F0 >> 1, F1 >> 1, F2 >> 1};  // F >= 0 here
  const int odd[3] = {F0 & 1, F1 & 1, F2 & 1};
  double c0[NV], t[3][NV];
  comp_val(u, blocks, M, g, L - 1, I[0], I[1], I[2], c0, err);
#pragma unroll
  for (int d = 0; d < 3; ++d) {
    double m[NV], q[NV];
    comp_val(u, blocks, M, g, L - 1, I[0] - (d == 0), I[1] - (d == 1), I[2] - (d == 2), m, err);
    comp_val(u, blocks, M, g, L - 1, I[0] + (d == 0), I[1] + (d == 1), I[2] + (d == 2), q, err);
#pragma unroll
    for (int v = 0; v < NV; ++v) {
      const double sd = minmod(c0[v] - m[v], q[v] - c0[v]);
      t[d][v] = odd[d] ? sd : -sd;
    }
  }
#pragma unroll
  for (int v = 0; v < NV; ++v) out[v] = c0[v] + 0.25 * ((t[0][v] + t[1][v]) + t[2][v]);
}

// Location of the restriction at level L of global cell J (in range): the 8
// level-(L+1) cells below it lie in one fine leaf (blocks have even edges),
// so the leaf is looked up once.
__device__ __forceinline__ uint2 restrict_loc(const BlockInfo* blocks, const LevelMaps& M, const Geom& g, int L,
                                              const int J[3]) {
  const int F[3] = {2 * J[0], 2 * J[1], 2 * J[2]};
  const int32_t fid = leaf_at(M, L + 1, F[0] / g.n1, F[1] / g.n2, F[2] / g.n3);
  if (fid < 0) return make_uint2(LOC_NONE, 0u);
  const BlockInfo bf = blocks[fid];
  return make_uint2((unsigned)fid,
                    (unsigned)pad_index(g, F[0] - bf.lx * g.n1, F[1] - bf.ly * g.n2, F[2] - bf.lz * g.n3) | LOC_RESTRICT);
}

// The face regions (width 2, active transverse extent) listed in jf as
// (leaf, face | wall kind << 3 | coarser << 6) pairs: the faces whose
// neighbour is on another level or beyond a wall, the only ghost cells the
// stage kernels read. Across a level jump, the region across one face is
// one block of the leaf's level, so a face is either wholly inside a
// coarser leaf (bit 6) or wholly refined. Coarser: the 2-deep slab is one
// coarse cell deep and aligned to coarse cells; eight lanes share one
// coarse cell: lane l forms the composite value of stencil point l (the
// cell, then its -x, +x, -y, +y, -z, +z neighbours; lane 7 repeats the
// cell), the lanes swap them by shuffles, and lane o writes fine child o.
// Refined: one thread per ghost cell, restriction of its 8 fine cells.
// Threads per face record: fill_faces_stride(g), 256 per workgroup.

// Thread q of face record f: the level-jump case of the record, the ghost
// cell (coarser: the first of its group's 2x2x2 children) and where the
// value this thread reads lives, as comp_loc encodes it with the image's
// reflected directions in bits 29-31. False for a wall record or a thread
// with no cell.
__device__ inline bool fill_faces_loc(const BlockInfo* blocks, const Geom& g, const LevelMaps& M, int2 rec, int q,
                                      uint2* loc) {
  const int b = rec.x, d = (rec.y & 7) >> 1, hi = rec.y & 1, wall = (rec.y >> 3) & 7;
  if (wall) return false;
  const int n[3] = {g.n1, g.n2, g.n3};
  const int t1 = d == 0 ? 1 : 0, t2 = d == 2 ? 1 : 2;
  const BlockInfo bi = blocks[b];
  const int L = bi.level;
  const int lo[3] = {bi.lx, bi.ly, bi.lz};
  int c[3];
  if ((rec.y >> 6) & 1) {
    const int m1 = n[t1] >> 1, m2 = n[t2] >> 1;
    const int cq = q >> 3, l = q & 7;
    if (cq >= m1 * m2) return false;
    c[t1] = 2 * (cq % m1);
    c[t2] = 2 * (cq / m1);
    c[d] = hi ? n[d] : -NG;
    int J[3];
#pragma unroll
    for (int e = 0; e < 3; ++e) J[e] = wrap_i(lo[e] * n[e] + c[e], (g.nrb[e] * n[e]) << L) >> 1;
    const int se = (l - 1) >> 1, sg = (l & 1) ? -1 : 1;  // lanes 1..6: axis and side
    if (l != 0 && l != 7) J[se] += sg;
    const int code = cell_in_domain(g, L - 1, J);
    const uint2 e = comp_loc(blocks, M, g, L - 1, J);
    *loc = make_uint2(e.x, e.y | (unsigned)(code & 7) << 29);
    return true;
  }
  const int area = n[t1] * n[t2];
  if (q >= 2 * area) return false;
  // x faces: the two layers of a row on neighbouring lanes (one cache line)
  const int s = d == 0 ? (q & 1) : q / area, r = d == 0 ? (q >> 1) : q - s * area;
  c[t1] = r % n[t1];
  c[t2] = r / n[t1];
  c[d] = hi ? n[d] + s : s - NG;
  int J[3];
#pragma unroll
  for (int e = 0; e < 3; ++e) J[e] = wrap_i(lo[e] * n[e] + c[e], (g.nrb[e] * n[e]) << L);
  *loc = restrict_loc(blocks, M, g, L, J);
  return true;
}

// One 256-thread workgroup's share of face record f: cells from 256 x.
// plan: the locations fill_faces_loc gives, fill_faces_stride per record,
// built once per mesh layout, so a thread's reads wait on one load of its
// location instead of a walk through the block list and level maps.
__device__ inline void fill_faces_item(double* u, const Geom& g, DevTime* tm, const int32_t* __restrict__ jf,
                                       const uint2* __restrict__ plan, int x, int f) {
  const int2 rec = reinterpret_cast<const int2*>(jf)[f];
  const int b = rec.x, d = (rec.y & 7) >> 1, hi = rec.y & 1, wall = (rec.y >> 3) & 7;
  const int n[3] = {g.n1, g.n2, g.n3};
  const int t1 = d == 0 ? 1 : 0, t2 = d == 2 ? 1 : 2;
  const int q = x * 256 + (int)threadIdx.x;
  double* ub = u + (int64_t)b * g.bstride;
  if (wall) {
    // a face on the domain boundary: the image of each ghost cell lies in
    // the leaf itself (the nearest layer for outflow, the mirror layer for
    // reflection, normal momentum negated)
    const int area = n[t1] * n[t2];
    if (q >= 2 * area) return;
    // x faces: the two layers of a row on neighbouring lanes (one cache line)
    const int s = d == 0 ? (q & 1) : q / area, r = d == 0 ? (q >> 1) : q - s * area;
    int c[3], src[3];
    c[t1] = src[t1] = r % n[t1];
    c[t2] = src[t2] = r / n[t1];
    c[d] = hi ? n[d] + s : s - NG;
    if (wall == BC_OUTFLOW)
      src[d] = hi ? n[d] - 1 : 0;
    else
      src[d] = hi ? 2 * n[d] - 1 - c[d] : -1 - c[d];
    const double* sp = ub + pad_index(g, src[0], src[1], src[2]);
    double* dp = ub + pad_index(g, c[0], c[1], c[2]);
#pragma unroll
    for (int v = 0; v < NV; ++v) {
      const double x = sp[v * g.vstride];
      dp[v * g.vstride] = (wall == BC_REFLECT && v == 1 + d) ? -x : x;
    }
    return;
  }
  int err = 0;
  if ((rec.y >> 6) & 1) {
    // Uniform per workgroup (one face per item): whole 8-lane groups
    // leave together, so the shuffles below see only live groups.
    const int m1 = n[t1] >> 1, m2 = n[t2] >> 1;
    const int cq = q >> 3, l = q & 7;
    if (cq >= m1 * m2) return;
    int c[3];  // first fine ghost cell of this group's 2x2x2 children, leaf coordinates
    c[t1] = 2 * (cq % m1);
    c[t2] = 2 * (cq / m1);
    c[d] = hi ? n[d] : -NG;
    const uint2 e = plan[(int64_t)f * fill_faces_stride(g) + q];
    double val[NV];
    comp_gather(u, g, e, val, &err);
    apply_image_signs((int)(e.y >> 29), val);
    const int base = threadIdx.x & ~7 & 63;
    const int o = l;
    double outv[NV];
#pragma unroll
    for (int v = 0; v < NV; ++v) {
      const double c0 = __shfl(val[v], base, 64);
      double t[3];
#pragma unroll
      for (int e = 0; e < 3; ++e) {
        const double mv = __shfl(val[v], base + 1 + 2 * e, 64);
        const double pv = __shfl(val[v], base + 2 + 2 * e, 64);
        const double sd = minmod(c0 - mv, pv - c0);
        t[e] = ((o >> e) & 1) ? sd : -sd;
      }
      outv[v] = c0 + 0.25 * ((t[0] + t[1]) + t[2]);
    }
    // c[e] is even in every direction, so child o sits on the odd side
    // along e exactly when bit e of o is set.
    double* dst = ub + pad_index(g, c[0] + (o & 1), c[1] + ((o >> 1) & 1), c[2] + ((o >> 2) & 1));
#pragma unroll
    for (int v = 0; v < NV; ++v) dst[v * g.vstride] = outv[v];
  } else {
    const int area = n[t1] * n[t2];
    if (q >= 2 * area) return;
    // x faces: the two layers of a row on neighbouring lanes (one cache line)
    const int s = d == 0 ? (q & 1) : q / area, r = d == 0 ? (q >> 1) : q - s * area;
    int c[3];
    c[t1] = r % n[t1];
    c[t2] = r / n[t1];
    c[d] = hi ? n[d] + s : s - NG;
    const uint2 e = plan[(int64_t)f * fill_faces_stride(g) + q];
    double val[NV];
    comp_gather(u, g, e, val, &err);
    double* dst = ub + pad_index(g, c[0], c[1], c[2]);
#pragma unroll
    for (int v = 0; v < NV; ++v) dst[v * g.vstride] = val[v];
  }
  if (err) atomicOr(&tm->err, 2);
}

// q-th cell of the outer layer of a block (a coordinate at 0 or n - 1):
// the two z planes, then for each inner plane its two y rows and the two
// x ends of each inner row. False past the last one.
__device__ __forceinline__ bool shell_coord(int q, const Geom& g, int& i, int& j, int& k) {
  const int plane = g.n1 * g.n2;
  if (q < 0) return false;
  if (q < 2 * plane) {
    const bool top = q >= plane;
    k = top ? g.n3 - 1 : 0;
    const int r = top ? q - plane : q;
    j = r / g.n1;
    i = r - j * g.n1;
    return true;
  }
  q -= 2 * plane;
  const int per = 2 * g.n1 + 2 * (g.n2 - 2);
  if (q >= (g.n3 - 2) * per) return false;
  k = 1 + q / per;
  int r = q - (k - 1) * per;
  if (r < 2 * g.n1) {
    const bool top = r >= g.n1;
    j = top ? g.n2 - 1 : 0;
    i = top ? r - g.n1 : r;
    return true;
  }
  r -= 2 * g.n1;
  j = 1 + (r >> 1);
  i = (r & 1) ? g.n1 - 1 : 0;
  return true;
}

// ---------------------------------------------------------------------------
// Flux correction as reflux: on each coarse face bordering finer leaves the
// coarse flux is replaced by the area mean of the 4 fine fluxes,
// U += +-beta*dt/dx * (F_own - F_fine). One thread per outer-layer cell of
// a coarse block that has such faces; a cell on one of them applies all of
// its faces in x, y, z order, then (corrector stage) contributes to the CFL
// reduction the stage kernel skipped for it.
// ---------------------------------------------------------------------------

// One 256-thread workgroup's share: coarse block cblocks[c], shell cells
// from 256 x; dt the stage's timestep, sRed 4 doubles of LDS.
__device__ inline void flux_correct_item(double* u, const BlockInfo* blocks, const FineFace* ff,
                                         const int32_t* ff_first, const int32_t* cblocks, const Geom& g,
                                         DevTime* tm, double dt, double beta, int do_dt, const double* fbuf,
                                         int x, int c, double* sRed) {
  const int b = cblocks[c];
  const BlockInfo bi = blocks[b];
  const int q = x * 256 + (int)threadIdx.x;
  double smax = 0.0;
  bool bad = false;
  int i, j, k;
  if (shell_coord(q, g, i, j, k) &&
      ((((bi.finer_mask >> XLO) & 1) && i == 0) || (((bi.finer_mask >> XHI) & 1) && i == g.n1 - 1) ||
       (((bi.finer_mask >> YLO) & 1) && j == 0) || (((bi.finer_mask >> YHI) & 1) && j == g.n2 - 1) ||
       (((bi.finer_mask >> ZLO) & 1) && k == 0) || (((bi.finer_mask >> ZHI) & 1) && k == g.n3 - 1))) {
    const int fsz = NV * max(max(g.n1 * g.n2, g.n1 * g.n3), g.n2 * g.n3);
    bool touched = false;
    double* cell = u + (int64_t)b * g.bstride + pad_index(g, i, j, k);
    double uc[NV];
#pragma unroll
    for (int v = 0; v < NV; ++v) uc[v] = cell[v * g.vstride];
    const double coef = beta * dt;
    for (int e = ff_first[c]; e < ff_first[c + 1]; ++e) {
      const FineFace rec = ff[e];
      const int d = rec.face >> 1, s = rec.face & 1;
      // normal axis d and the two transverse axes in increasing order, as
      // selects (per-lane indexing of small arrays would put them in
      // scratch memory)
      const int cd = d == 0 ? i : (d == 1 ? j : k);
      const int nd = d == 0 ? g.n1 : (d == 1 ? g.n2 : g.n3);
      if (cd != (s ? nd - 1 : 0)) continue;
      touched = true;
      const int a1 = d == 0 ? j : i, m1 = d == 0 ? g.n2 : g.n1;
      const int a2 = d == 2 ? j : k, m2 = d == 2 ? g.n2 : g.n3;
      const int h1 = a1 >= m1 / 2, h2 = a2 >= m2 / 2;
      const int sub = h1 + 2 * h2;
      const int fs = sub == 0   ? rec.fine_slot[0]
                     : sub == 1 ? rec.fine_slot[1]
                     : sub == 2 ? rec.fine_slot[2]
                                : rec.fine_slot[3];
      const double idd = d == 0 ? bi.idx[0] : (d == 1 ? bi.idx[1] : bi.idx[2]);
      const int f1 = 2 * a1 - h1 * m1, f2 = 2 * a2 - h2 * m2;
      const double sg = s ? 1.0 : -1.0;
      for (int v = 0; v < NV; ++v) {
        const double own = fbuf[(int64_t)rec.own_slot * fsz + ((int64_t)v * m2 + a2) * m1 + a1];
        const double* fb = fbuf + (int64_t)fs * fsz + (int64_t)v * m2 * m1;
        const double fine = 0.25 * ((fb[f2 * m1 + f1] + fb[f2 * m1 + f1 + 1]) +
                                    (fb[(f2 + 1) * m1 + f1] + fb[(f2 + 1) * m1 + f1 + 1]));
        uc[v] += sg * coef * (own - fine) * idd;
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
      reduce_max_speed(tm, mx);
    }
  }
  if (bad) atomicOr(&tm->err, 1);
}

}  // namespace pkh
