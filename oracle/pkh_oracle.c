/*
 * pkh_oracle.c -- CPU FP64 oracle for the block-AMR ideal-gas Euler cycle.
 *
 * TEST INFRASTRUCTURE. Only the test suite, the smoke check and the
 * benchmark's CPU-baseline leg load this library. It shares no source, header,
 * table or helper with the GPU library; it is the plain definition the GPU
 * path is checked against.
 *
 * What it computes (Parthenon paper, arXiv:2202.12309):
 *   - Sec. 4.1 (Parthenon-hydro): a two-stage second-order update of the
 *     Euler equations with piecewise-linear reconstruction and the HLLE
 *     Riemann solver. The paper defers the numerical detail to Athena++; the
 *     readings taken here are the standard ones of that lineage:
 *       * integrator: van Leer / VL2 predictor-corrector (Stone & Gardiner
 *         2009): a donor-cell half step, then a PLM full step from U^n;
 *       * reconstruction on primitive variables with the monotonised-central
 *         (MC) limiter of van Leer (1977);
 *       * HLLE with Einfeldt (1988) wave speeds from Roe averages.
 *   - Sec. 2.1: same-size MeshBlocks as leaves of an oct-tree, one leaf per
 *     point of the domain, levels differing by at most one between
 *     neighbours (2:1).
 *   - Sec. 3.7: ghost zones filled from neighbours: copy at the same level,
 *     restriction from finer, prolongation from coarser; fine-coarse flux
 *     correction.
 *   - Sec. 3.8: periodic derefinement, tree rebuilt on (de)refinement.
 *   - Sec. 3.10: global reductions (the CFL timestep, conserved totals).
 *   - Optional FP32 storage of the state: each stage computes in FP64 from
 *     the stored values and rounds its output once to the nearest binary32
 *     value (the state set by the caller is rounded the same way).
 *   - Boundaries of the domain, per face: periodic, outflow (zero-gradient:
 *     a ghost cell takes the value of the nearest cell inside) or
 *     reflecting (a ghost cell takes the value of its mirror image across
 *     the face with the normal momentum negated). A ghost cell outside the
 *     domain is first mapped to its image inside, then evaluated like any
 *     ghost cell there (copy, restriction or prolongation), so the rule
 *     also covers the coarse cells a prolongation stencil reaches.
 *
 * Ghost values are evaluated as a pure function of the leaves' active data
 * (nothing is cached between stages), so the fill order cannot matter.
 *
 * Build (parity build): gcc -O2 -ffp-contract=off -fopenmp -fPIC -shared
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define NV 5
#define NG 2
#define MAXLEV 8

enum { ORC_OK = 0, ORC_EINVAL = -1, ORC_ETILING = -2, ORC_EBALANCE = -3,
       ORC_ENOMEM = -4, ORC_EPHYS = -6 };
enum { ORC_BC_PERIODIC = 0, ORC_BC_OUTFLOW = 1, ORC_BC_REFLECT = 2 };

typedef struct {
  int n[3];          /* active cells per block along x, y, z */
  int nrb[3];        /* level-0 blocks along x, y, z */
  int maxl;          /* deepest level allowed */
  double xmin[3], xmax[3];
  double gamma, cfl;
  int recon1;        /* stage-1 reconstruction: 0 donor cell, 1 PLM */
  int bc[6];         /* per face x-, x+, y-, y+, z-, z+: ORC_BC_* */
  int fp32;          /* state stored in binary32 (rounded after each stage) */
  int64_t nl;        /* number of leaves */
  int32_t *loc;      /* [nl][4]: level, lx, ly, lz */
  double *U;         /* [nl][5][n3][n2][n1], conserved, active cells */
  int32_t *map[MAXLEV + 1]; /* per level: block location -> leaf id or -1 */
  double t, dt_last;
  int64_t cycle;
  int err;
  /* branch signature (for finite-difference checks of the reverse mode):
     while track is set, every branch the cycle takes -- each MC limiter
     case, each HLLE wave-speed choice, each minmod case of a prolongation
     slope -- is hashed with its position and summed into sig (an
     order-free sum, so the OpenMP schedule cannot change it) */
  int track;
  uint64_t sig;
  int64_t stage_no;
} orc_mesh;

/* ------------------------------------------------------------------ */
/* Small pieces: equation of state, limiter, Riemann solver.          */
/* ------------------------------------------------------------------ */

/* Primitive variables (rho, vx, vy, vz, P) from conserved
   (rho, Mx, My, Mz, E) for an ideal gas: v = M/rho,
   P = (gamma-1) (E - |M|^2 / (2 rho)). */
void orc_prim(const double *u, double gamma, double *w) {
  w[0] = u[0];
  w[1] = u[1] / u[0];
  w[2] = u[2] / u[0];
  w[3] = u[3] / u[0];
  w[4] = (gamma - 1.0) * (u[4] - 0.5 * (u[1] * u[1] + u[2] * u[2] + u[3] * u[3]) / u[0]);
}

/* Monotonised-central limited slope from the two one-sided differences:
   zero at an extremum, else the smallest of 2|dl|, 2|dr|, |dl+dr|/2 with
   the common sign. */
double orc_mc(double dl, double dr) {
  if (dl * dr <= 0.0) return 0.0;
  double a = 2.0 * fabs(dl), b = 2.0 * fabs(dr), c = 0.5 * fabs(dl + dr);
  double m = a;
  if (b < m) m = b;
  if (c < m) m = c;
  return dl > 0.0 ? m : -m;
}

/* minmod limiter used by the prolongation slopes. */
double orc_minmod(double a, double b) {
  if (a * b <= 0.0) return 0.0;
  double m = fabs(a) < fabs(b) ? fabs(a) : fabs(b);
  return a > 0.0 ? m : -m;
}

/* Which case of orc_mc / orc_minmod a pair of differences takes (the same
   comparisons in the same order): MC 0 extremum, 1 2|dl|, 2 2|dr|,
   3 |dl+dr|/2; minmod 0 extremum, 1 a, 2 b. */
int orc_mc_code(double dl, double dr) {
  if (dl * dr <= 0.0) return 0;
  double a = 2.0 * fabs(dl), b = 2.0 * fabs(dr), c = 0.5 * fabs(dl + dr);
  double m = a;
  int k = 1;
  if (b < m) { m = b; k = 2; }
  if (c < m) k = 3;
  return k;
}

int orc_minmod_code(double a, double b) {
  if (a * b <= 0.0) return 0;
  return fabs(a) < fabs(b) ? 1 : 2;
}

static uint64_t mix64(uint64_t x) {
  x += 0x9E3779B97F4A7C15ull;
  x = (x ^ (x >> 30)) * 0xBF58476D1CE4E5B9ull;
  x = (x ^ (x >> 27)) * 0x94D049BB133111EBull;
  return x ^ (x >> 31);
}

/* Per-thread part of the branch signature of the stage being evaluated. */
static uint64_t tl_sig;
#pragma omp threadprivate(tl_sig)

static void track_branch(const orc_mesh *m, uint64_t key, uint64_t word) {
  if (m->track) tl_sig += mix64(mix64(key) ^ (word * 0xD6E8FEB86659FD93ull + 1));
}

static void hlle_impl(const double *wl, const double *wr, int d, double gamma, double *f, int *code);

/* HLLE flux across a face normal to direction d (0=x, 1=y, 2=z) from the
   primitive left/right states. Wave-speed bounds after Einfeldt (1988):
   b+ = max(u_roe + a_roe, u_R + c_R, 0), b- = min(u_roe - a_roe, u_L - c_L, 0),
   with Roe-averaged velocity and enthalpy. F = (b+ F_L - b- F_R +
   b+ b- (U_R - U_L)) / (b+ - b-). Output is the conserved-variable flux in
   (rho, Mx, My, Mz, E) order. */
void orc_hlle(const double *wl, const double *wr, int d, double gamma, double *f) {
  hlle_impl(wl, wr, d, gamma, f, NULL);
}

/* Which wave-speed bounds orc_hlle takes: 3 * (b- case) + (b+ case), with
   case 0 the Roe estimate, 1 the outer side's signal speed, 2 zero. */
int orc_hlle_code(const double *wl, const double *wr, int d, double gamma) {
  double f[5];
  int code = 0;
  hlle_impl(wl, wr, d, gamma, f, &code);
  return code;
}

static void hlle_impl(const double *wl, const double *wr, int d, double gamma, double *f, int *code) {
  double gm1 = gamma - 1.0;
  double rl = wl[0], pl = wl[4], rr = wr[0], pr = wr[4];
  double ul = wl[1 + d], ur = wr[1 + d];
  double v2l = wl[1] * wl[1] + wl[2] * wl[2] + wl[3] * wl[3];
  double v2r = wr[1] * wr[1] + wr[2] * wr[2] + wr[3] * wr[3];
  double el = pl / gm1 + 0.5 * rl * v2l;
  double er = pr / gm1 + 0.5 * rr * v2r;
  double hl = (el + pl) / rl, hr = (er + pr) / rr;
  double cl = sqrt(gamma * pl / rl), cr = sqrt(gamma * pr / rr);
  double sl = sqrt(rl), sr = sqrt(rr);
  double r = sl / (sl + sr);
  double vb[3];
  for (int c = 0; c < 3; ++c) vb[c] = r * wl[1 + c] + (1.0 - r) * wr[1 + c];
  double hb = r * hl + (1.0 - r) * hr;
  double vb2 = vb[0] * vb[0] + vb[1] * vb[1] + vb[2] * vb[2];
  double ab = sqrt(gm1 * (hb - 0.5 * vb2));
  double bp = vb[d] + ab;
  int kp = 0, km = 0;
  if (ur + cr > bp) { bp = ur + cr; kp = 1; }
  if (0.0 > bp) { bp = 0.0; kp = 2; }
  double bm = vb[d] - ab;
  if (ul - cl < bm) { bm = ul - cl; km = 1; }
  if (0.0 < bm) { bm = 0.0; km = 2; }
  if (code) *code = 3 * km + kp;

  double fl[5], fr[5], uL[5], uR[5];
  uL[0] = rl; uR[0] = rr;
  for (int c = 0; c < 3; ++c) { uL[1 + c] = rl * wl[1 + c]; uR[1 + c] = rr * wr[1 + c]; }
  uL[4] = el; uR[4] = er;
  fl[0] = rl * ul; fr[0] = rr * ur;
  for (int c = 0; c < 3; ++c) {
    fl[1 + c] = rl * ul * wl[1 + c];
    fr[1 + c] = rr * ur * wr[1 + c];
  }
  fl[1 + d] += pl;
  fr[1 + d] += pr;
  fl[4] = (el + pl) * ul;
  fr[4] = (er + pr) * ur;
  for (int v = 0; v < 5; ++v)
    f[v] = (bp * fl[v] - bm * fr[v] + bp * bm * (uR[v] - uL[v])) / (bp - bm);
}

/* ------------------------------------------------------------------ */
/* Mesh bookkeeping.                                                   */
/* ------------------------------------------------------------------ */

static int64_t ncell(const orc_mesh *m) { return (int64_t)m->n[0] * m->n[1] * m->n[2]; }
static int64_t nblk_dim(const orc_mesh *m, int L, int d) { return (int64_t)m->nrb[d] << L; }
static int64_t ncel_dim(const orc_mesh *m, int L, int d) { return ((int64_t)m->nrb[d] * m->n[d]) << L; }
static int64_t wrap(int64_t a, int64_t n) { a %= n; return a < 0 ? a + n : a; }

static double dxl(const orc_mesh *m, int L, int d) {
  return (m->xmax[d] - m->xmin[d]) / (double)ncel_dim(m, L, d);
}

static int periodic(const orc_mesh *m, int d) { return m->bc[2 * d] == ORC_BC_PERIODIC; }

/* Block location b of level L brought into the domain: wrapped along
   periodic directions. Returns 0 (and leaves w undefined) when b lies
   outside the domain along a non-periodic direction. */
static int block_in_domain(const orc_mesh *m, int L, const int64_t b[3], int64_t w[3]) {
  for (int d = 0; d < 3; ++d) {
    int64_t nb = nblk_dim(m, L, d);
    if (periodic(m, d)) w[d] = wrap(b[d], nb);
    else if (b[d] < 0 || b[d] >= nb) return 0;
    else w[d] = b[d];
  }
  return 1;
}

/* Leaf id whose block location at level L is b (wrapped along periodic
   directions), or -1 (also outside the domain). */
static int32_t leaf_at(const orc_mesh *m, int L, const int64_t b[3]) {
  if (L < 0 || L > m->maxl) return -1;
  int64_t w[3];
  if (!block_in_domain(m, L, b, w)) return -1;
  return m->map[L][(w[2] * nblk_dim(m, L, 1) + w[1]) * nblk_dim(m, L, 0) + w[0]];
}

/* Leaf at a level below L that contains block location b of level L, or -1.
   Writes its level to *lc. */
static int32_t coarser_leaf(const orc_mesh *m, int L, const int64_t b[3], int *lc) {
  int64_t w[3];
  if (!block_in_domain(m, L, b, w)) return -1;
  for (int Lc = L - 1; Lc >= 0; --Lc) {
    int s = L - Lc;
    int64_t bw[3];
    for (int d = 0; d < 3; ++d) bw[d] = w[d] >> s;
    int32_t id = leaf_at(m, Lc, bw);
    if (id >= 0) { *lc = Lc; return id; }
  }
  return -1;
}

/* Global cell J of level L mapped into the domain: wrapped along periodic
   directions; along the others a cell beyond a face goes to the nearest
   cell inside (outflow) or to its mirror image (reflecting). Returns the
   set of reflected directions as bits (bit d: the momentum along d of the
   image changes sign). */
static int cell_in_domain(const orc_mesh *m, int L, const int64_t Jin[3], int64_t J[3]) {
  int flip = 0;
  for (int d = 0; d < 3; ++d) {
    int64_t N = ncel_dim(m, L, d);
    J[d] = Jin[d];
    if (periodic(m, d)) { J[d] = wrap(J[d], N); continue; }
    int side = J[d] < 0 ? 0 : (J[d] >= N ? 1 : -1);
    if (side < 0) continue;
    if (m->bc[2 * d + side] == ORC_BC_OUTFLOW) {
      J[d] = side ? N - 1 : 0;
    } else {
      J[d] = side ? 2 * N - 1 - J[d] : -1 - J[d];
      flip ^= 1 << d;
    }
  }
  return flip;
}

/* Sign of variable v of an image reflected along the directions in flip. */
static double image_sign(int flip, int v) {
  return (v >= 1 && v <= 3 && ((flip >> (v - 1)) & 1)) ? -1.0 : 1.0;
}

static double uat(const orc_mesh *m, const double *U, int64_t id, int v,
                  int64_t i, int64_t j, int64_t k) {
  return U[(((id * NV + v) * m->n[2] + k) * m->n[1] + j) * m->n[0] + i];
}

/* Restriction: volume average of a 2x2x2 group f[c][b][a] (a along x),
   summed pairwise so that a uniform field restricts exactly. */
static double restrict8(const double f[2][2][2]) {
  return 0.125 * (((f[0][0][0] + f[0][0][1]) + (f[0][1][0] + f[0][1][1])) +
                  ((f[1][0][0] + f[1][0][1]) + (f[1][1][0] + f[1][1][1])));
}

/* Composite field at level L, global cell J of that level (wrapped):
   the leaf value where a level-L leaf covers J; the restriction of the
   composite level-(L+1) field where finer leaves cover it; and the value of
   the containing coarser cell (injection) where a coarser leaf covers it.
   The last case is reached only while regridding. */
static double comp(const orc_mesh *m, const double *U, int L, const int64_t Jin[3], int v) {
  int64_t J[3], b[3];
  const double sg = image_sign(cell_in_domain(m, L, Jin, J), v);
  for (int d = 0; d < 3; ++d) b[d] = J[d] / m->n[d];
  int32_t id = leaf_at(m, L, b);
  if (id >= 0)
    return sg * uat(m, U, id, v, J[0] - b[0] * m->n[0], J[1] - b[1] * m->n[1], J[2] - b[2] * m->n[2]);
  int lc;
  id = coarser_leaf(m, L, b, &lc);
  if (id >= 0) {
    int s = L - lc;
    int64_t Jc[3];
    for (int d = 0; d < 3; ++d) Jc[d] = J[d] >> s;
    const int32_t *lo = m->loc + 4 * id;
    return sg * uat(m, U, id, v, Jc[0] - (int64_t)lo[1] * m->n[0], Jc[1] - (int64_t)lo[2] * m->n[1],
                    Jc[2] - (int64_t)lo[3] * m->n[2]);
  }
  double f[2][2][2];
  for (int c = 0; c < 2; ++c)
    for (int bb = 0; bb < 2; ++bb)
      for (int a = 0; a < 2; ++a) {
        int64_t Jf[3] = {2 * J[0] + a, 2 * J[1] + bb, 2 * J[2] + c};
        f[c][bb][a] = comp(m, U, L + 1, Jf, v);
      }
  return sg * restrict8(f);
}

/* Ghost value at a level-L cell J inside the domain (O6 rules). */
static double ghost_inside(orc_mesh *m, const double *U, int L, const int64_t J[3], int v) {
  int64_t b[3];
  for (int d = 0; d < 3; ++d) b[d] = J[d] / m->n[d];
  int32_t id = leaf_at(m, L, b);
  if (id >= 0)  /* same level: copy */
    return uat(m, U, id, v, J[0] - b[0] * m->n[0], J[1] - b[1] * m->n[1], J[2] - b[2] * m->n[2]);
  int lc;
  id = coarser_leaf(m, L, b, &lc);
  if (id >= 0) {
    if (lc != L - 1) { m->err = ORC_EBALANCE; return NAN; }
    /* coarser: linear prolongation with minmod slopes of the composite
       level-(L-1) field; the fine cell sits a quarter coarse width from the
       coarse centre along each axis. */
    int64_t I[3] = {J[0] >> 1, J[1] >> 1, J[2] >> 1};
    double c0 = comp(m, U, L - 1, I, v);
    double ss[3];
    uint64_t word = 0;
    for (int d = 0; d < 3; ++d) {
      int64_t Im[3] = {I[0], I[1], I[2]}, Ip[3] = {I[0], I[1], I[2]};
      Im[d] -= 1;
      Ip[d] += 1;
      double da = c0 - comp(m, U, L - 1, Im, v), db = comp(m, U, L - 1, Ip, v) - c0;
      double s = orc_minmod(da, db);
      word = 4 * word + (uint64_t)orc_minmod_code(da, db);
      ss[d] = (J[d] & 1) ? s : -s;
    }
    if (m->track) {
      uint64_t key = ((((uint64_t)m->stage_no * 16 + (uint64_t)L) * 8 + (uint64_t)v) << 40) ^
                     (((uint64_t)J[2] & 0x3FFF) << 28) ^ (((uint64_t)J[1] & 0x3FFF) << 14) ^
                     ((uint64_t)J[0] & 0x3FFF);
      track_branch(m, key ^ 0x5555000000000000ull, word);
    }
    return c0 + 0.25 * ((ss[0] + ss[1]) + ss[2]);
  }
  /* finer: restriction of the covering fine cells */
  double f[2][2][2];
  for (int c = 0; c < 2; ++c)
    for (int bb = 0; bb < 2; ++bb)
      for (int a = 0; a < 2; ++a) {
        int64_t Jf[3] = {2 * J[0] + a, 2 * J[1] + bb, 2 * J[2] + c};
        f[c][bb][a] = comp(m, U, L + 1, Jf, v);
      }
  return restrict8(f);
}

/* Value of a ghost cell of a level-L leaf at global level-L cell J: the
   value of its image in the domain (the cell itself where it lies inside),
   times the image's momentum signs. */
static double ghost_value(orc_mesh *m, const double *U, int L, const int64_t Jin[3], int v) {
  int64_t J[3];
  const double sg = image_sign(cell_in_domain(m, L, Jin, J), v);
  return sg * ghost_inside(m, U, L, J, v);
}

/* Padded copy [5][n3+4][n2+4][n1+4] of leaf id: active cells from U, ghost
   cells from ghost_value. */
static void fill_padded(orc_mesh *m, const double *U, int64_t id, double *P) {
  const int n1 = m->n[0], n2 = m->n[1], n3 = m->n[2];
  const int p1 = n1 + 2 * NG, p2 = n2 + 2 * NG, p3 = n3 + 2 * NG;
  const int32_t *lo = m->loc + 4 * id;
  int L = lo[0];
  for (int v = 0; v < NV; ++v)
    for (int k = -NG; k < n3 + NG; ++k)
      for (int j = -NG; j < n2 + NG; ++j)
        for (int i = -NG; i < n1 + NG; ++i) {
          double val;
          if (i >= 0 && i < n1 && j >= 0 && j < n2 && k >= 0 && k < n3) {
            val = uat(m, U, id, v, i, j, k);
          } else {
            int64_t J[3] = {(int64_t)lo[1] * n1 + i, (int64_t)lo[2] * n2 + j,
                            (int64_t)lo[3] * n3 + k};
            val = ghost_value(m, U, L, J, v);
          }
          P[(((int64_t)v * p3 + (k + NG)) * p2 + (j + NG)) * p1 + (i + NG)] = val;
        }
  (void)p3;
}

/* ------------------------------------------------------------------ */
/* One stage: fluxes of every leaf, flux correction, update.           */
/* ------------------------------------------------------------------ */

/* Flux arrays per leaf and direction d: [5][.][.][.] with extent n_d + 1
   along d (face f lies between cells f-1 and f). */
static int64_t fsize(const orc_mesh *m, int d) {
  return (int64_t)NV * (m->n[0] + (d == 0)) * (m->n[1] + (d == 1)) * (m->n[2] + (d == 2));
}
static int64_t fidx(const orc_mesh *m, int d, int v, int64_t i, int64_t j, int64_t k) {
  int64_t e0 = m->n[0] + (d == 0), e1 = m->n[1] + (d == 1), e2 = m->n[2] + (d == 2);
  return (((int64_t)v * e2 + k) * e1 + j) * e0 + i;
}

/* Face fluxes of one leaf along d from its padded primitives Wp. */
static void leaf_fluxes(const orc_mesh *m, int64_t blk, const double *Wp, int recon, int d, double *F) {
  const int n1 = m->n[0], n2 = m->n[1], n3 = m->n[2];
  const int64_t p1 = n1 + 2 * NG, p2 = n2 + 2 * NG, p3 = n3 + 2 * NG;
  const int64_t cstride = p1 * p2 * p3;
  const int64_t step = d == 0 ? 1 : (d == 1 ? p1 : p1 * p2);
  int e0 = n1 + (d == 0), e1 = n2 + (d == 1), e2 = n3 + (d == 2);
  for (int k = 0; k < e2; ++k)
    for (int j = 0; j < e1; ++j)
      for (int i = 0; i < e0; ++i) {
        /* cell "i" of the face is the upper neighbour; "i-1" the lower */
        int64_t c = ((int64_t)(k + NG) * p2 + (j + NG)) * p1 + (i + NG);
        double wl[5], wr[5], f[5];
        uint64_t word = 0;
        for (int v = 0; v < NV; ++v) {
          const double *q = Wp + v * cstride;
          double qm2 = q[c - 2 * step], qm1 = q[c - step], q0 = q[c], qp1 = q[c + step];
          if (recon == 0) {
            wl[v] = qm1;
            wr[v] = q0;
          } else {
            wl[v] = qm1 + 0.5 * orc_mc(qm1 - qm2, q0 - qm1);
            wr[v] = q0 - 0.5 * orc_mc(q0 - qm1, qp1 - q0);
            if (m->track) word = 16 * word + 4 * (uint64_t)orc_mc_code(qm1 - qm2, q0 - qm1) +
                                 (uint64_t)orc_mc_code(q0 - qm1, qp1 - q0);
          }
        }
        int hc = 0;
        hlle_impl(wl, wr, d, m->gamma, f, &hc);
        if (m->track) {
          /* with identical face states (outflow walls copy the cell beside
             them) both wave-speed bounds of a pair coincide in exact
             arithmetic and the flux is F(U) whatever they are: its
             derivative does not depend on the bound taken, so such a face
             records no wave-speed case */
          int same = 1;
          for (int v = 0; v < NV; ++v) same &= wl[v] == wr[v];
          if (same) hc = 15;
          uint64_t key = (((((uint64_t)m->stage_no * 4 + (uint64_t)d) << 24) ^ (uint64_t)blk) << 32) ^
                         (((uint64_t)k & 0x7FF) << 22) ^ (((uint64_t)j & 0x7FF) << 11) ^ ((uint64_t)i & 0x7FF);
          track_branch(m, key, 16 * word + (uint64_t)hc);
        }
        for (int v = 0; v < NV; ++v) F[fidx(m, d, v, i, j, k)] = f[v];
      }
}

/* On every face of a leaf that borders finer leaves, the leaf's flux is
   replaced by the area average of the four covering fine-face fluxes. */
static void flux_correct(orc_mesh *m, double **F) {
  for (int64_t b = 0; b < m->nl; ++b) {
    const int32_t *lo = m->loc + 4 * b;
    int L = lo[0];
    if (L >= m->maxl) continue;
    for (int d = 0; d < 3; ++d)
      for (int s = 0; s < 2; ++s) {
        int64_t nb0[3] = {lo[1], lo[2], lo[3]}, nb[3];
        nb0[d] += s ? 1 : -1;
        if (!block_in_domain(m, L, nb0, nb)) continue; /* domain boundary */
        if (leaf_at(m, L, nb) >= 0) continue;
        int lc;
        if (coarser_leaf(m, L, nb, &lc) >= 0) continue;
        int t1 = d == 0 ? 1 : 0, t2 = d == 2 ? 1 : 2;
        int nt1 = m->n[t1], nt2 = m->n[t2];
        for (int c2 = 0; c2 < nt2; ++c2)
          for (int c1 = 0; c1 < nt1; ++c1) {
            int h1 = c1 >= nt1 / 2, h2 = c2 >= nt2 / 2;
            int64_t ch[3];
            ch[d] = 2 * nb[d] + (s ? 0 : 1);
            ch[t1] = 2 * nb[t1] + h1;
            ch[t2] = 2 * nb[t2] + h2;
            int32_t fid = leaf_at(m, L + 1, ch);
            if (fid < 0) { m->err = ORC_EBALANCE; return; }
            int64_t ff = s ? 0 : m->n[d];
            for (int v = 0; v < NV; ++v) {
              double g[2][2];
              for (int b2 = 0; b2 < 2; ++b2)
                for (int b1 = 0; b1 < 2; ++b1) {
                  int64_t ix[3];
                  ix[d] = ff;
                  ix[t1] = 2 * c1 - (h1 ? nt1 : 0) + b1;
                  ix[t2] = 2 * c2 - (h2 ? nt2 : 0) + b2;
                  g[b2][b1] = F[fid * 3 + d][fidx(m, d, v, ix[0], ix[1], ix[2])];
                }
              double avg = 0.25 * ((g[0][0] + g[0][1]) + (g[1][0] + g[1][1]));
              int64_t ic[3];
              ic[d] = s ? m->n[d] : 0;
              ic[t1] = c1;
              ic[t2] = c2;
              F[b * 3 + d][fidx(m, d, v, ic[0], ic[1], ic[2])] = avg;
            }
          }
      }
  }
}

/* Uout = Ubase - coef * D(Uin), D = sum_d (F_d(+1/2) - F_d(-1/2)) / dx_d with
   the fluxes of Uin after flux correction. Uout may alias Ubase. */
static int stage(orc_mesh *m, const double *Uin, const double *Ubase, double *Uout, int recon,
                 double coef) {
  const int n1 = m->n[0], n2 = m->n[1], n3 = m->n[2];
  const int64_t psz = (int64_t)NV * (n1 + 2 * NG) * (n2 + 2 * NG) * (n3 + 2 * NG);
  double **F = (double **)calloc((size_t)(m->nl * 3), sizeof(double *));
  if (!F) return ORC_ENOMEM;
  for (int64_t q = 0; q < m->nl * 3; ++q) {
    F[q] = (double *)malloc(sizeof(double) * (size_t)fsize(m, (int)(q % 3)));
    if (!F[q]) return ORC_ENOMEM;
  }
  int bad = 0;
  m->stage_no += 1;
#pragma omp parallel
  {
    tl_sig = 0;
    double *P = (double *)malloc(sizeof(double) * (size_t)psz);
    double *W = (double *)malloc(sizeof(double) * (size_t)psz);
    int64_t cs = psz / NV;
#pragma omp for schedule(dynamic, 1)
    for (int64_t b = 0; b < m->nl; ++b) {
      fill_padded(m, Uin, b, P);
      for (int64_t c = 0; c < cs; ++c) {
        double u[5], w[5];
        for (int v = 0; v < NV; ++v) u[v] = P[v * cs + c];
        orc_prim(u, m->gamma, w);
        if (!(w[0] > 0.0) || !(w[4] > 0.0) || !isfinite(w[1] + w[2] + w[3])) {
#pragma omp atomic write
          bad = 1;
        }
        for (int v = 0; v < NV; ++v) W[v * cs + c] = w[v];
      }
      for (int d = 0; d < 3; ++d) leaf_fluxes(m, b, W, recon, d, F[b * 3 + d]);
    }
    free(P);
    free(W);
    if (m->track) {
#pragma omp atomic
      m->sig += tl_sig;
    }
  }
  flux_correct(m, F);
#pragma omp parallel for schedule(static)
  for (int64_t b = 0; b < m->nl; ++b) {
    int L = m->loc[4 * b];
    double dx = dxl(m, L, 0), dy = dxl(m, L, 1), dz = dxl(m, L, 2);
    const double *Fx = F[b * 3], *Fy = F[b * 3 + 1], *Fz = F[b * 3 + 2];
    for (int v = 0; v < NV; ++v)
      for (int k = 0; k < n3; ++k)
        for (int j = 0; j < n2; ++j)
          for (int i = 0; i < n1; ++i) {
            double div = (Fx[fidx(m, 0, v, i + 1, j, k)] - Fx[fidx(m, 0, v, i, j, k)]) / dx +
                         (Fy[fidx(m, 1, v, i, j + 1, k)] - Fy[fidx(m, 1, v, i, j, k)]) / dy;
            div += (Fz[fidx(m, 2, v, i, j, k + 1)] - Fz[fidx(m, 2, v, i, j, k)]) / dz;
            int64_t o = (((b * NV + v) * n3 + k) * n2 + j) * n1 + i;
            Uout[o] = Ubase[o] - coef * div;
            if (m->fp32) Uout[o] = (double)(float)Uout[o];
          }
  }
  for (int64_t q = 0; q < m->nl * 3; ++q) free(F[q]);
  free(F);
  if (bad) m->err = ORC_EPHYS;
  return m->err;
}

/* CFL timestep: cfl * min over leaf active cells and directions of
   dx_d / (|v_d| + c). Returns a negative value on an unphysical state. */
static double cfl_dt(orc_mesh *m, const double *U) {
  double best = INFINITY;
  int bad = 0;
#pragma omp parallel for reduction(min : best) reduction(| : bad)
  for (int64_t b = 0; b < m->nl; ++b) {
    int L = m->loc[4 * b];
    double dx[3] = {dxl(m, L, 0), dxl(m, L, 1), dxl(m, L, 2)};
    for (int64_t c = 0; c < ncell(m); ++c) {
      double u[5], w[5];
      for (int v = 0; v < NV; ++v) u[v] = U[(b * NV + v) * ncell(m) + c];
      orc_prim(u, m->gamma, w);
      if (!(w[0] > 0.0) || !(w[4] > 0.0) || !isfinite(w[1] + w[2] + w[3])) { bad |= 1; continue; }
      double cs = sqrt(m->gamma * w[4] / w[0]);
      for (int d = 0; d < 3; ++d) {
        double q = dx[d] / (fabs(w[1 + d]) + cs);
        if (q < best) best = q;
      }
    }
  }
  if (bad) { m->err = ORC_EPHYS; return -1.0; }
  return m->cfl * best;
}

/* ------------------------------------------------------------------ */
/* Public interface.                                                   */
/* ------------------------------------------------------------------ */

static uint64_t spread3(uint64_t x) {
  uint64_t r = 0;
  for (int bit = 0; bit < 21; ++bit) r |= ((x >> bit) & 1ull) << (3 * bit);
  return r;
}

static uint64_t morton_key(const orc_mesh *m, const int32_t *lo) {
  int s = m->maxl - lo[0];
  return spread3((uint64_t)lo[1] << s) | (spread3((uint64_t)lo[2] << s) << 1) |
         (spread3((uint64_t)lo[3] << s) << 2);
}

static const orc_mesh *g_sort_mesh;
static int cmp_loc(const void *a, const void *b) {
  const int32_t *la = (const int32_t *)a, *lb = (const int32_t *)b;
  uint64_t ka = morton_key(g_sort_mesh, la), kb = morton_key(g_sort_mesh, lb);
  if (ka != kb) return ka < kb ? -1 : 1;
  return la[0] - lb[0];
}

/* Rebuild the per-level location maps; validates the tiling and 2:1. */
static int build_maps(orc_mesh *m) {
  for (int L = 0; L <= MAXLEV; ++L) { free(m->map[L]); m->map[L] = NULL; }
  for (int L = 0; L <= m->maxl; ++L) {
    int64_t sz = nblk_dim(m, L, 0) * nblk_dim(m, L, 1) * nblk_dim(m, L, 2);
    m->map[L] = (int32_t *)malloc(sizeof(int32_t) * (size_t)sz);
    if (!m->map[L]) return ORC_ENOMEM;
    for (int64_t q = 0; q < sz; ++q) m->map[L][q] = -1;
  }
  /* occupancy at the deepest level: every unit covered exactly once */
  int64_t f0 = nblk_dim(m, m->maxl, 0), f1 = nblk_dim(m, m->maxl, 1), f2 = nblk_dim(m, m->maxl, 2);
  unsigned char *occ = (unsigned char *)calloc((size_t)(f0 * f1 * f2), 1);
  if (!occ) return ORC_ENOMEM;
  int rc = ORC_OK;
  for (int64_t b = 0; b < m->nl && rc == ORC_OK; ++b) {
    const int32_t *lo = m->loc + 4 * b;
    int L = lo[0];
    if (L < 0 || L > m->maxl) { rc = ORC_EINVAL; break; }
    for (int d = 0; d < 3; ++d)
      if (lo[1 + d] < 0 || lo[1 + d] >= nblk_dim(m, L, d)) rc = ORC_EINVAL;
    if (rc) break;
    m->map[L][((int64_t)lo[3] * nblk_dim(m, L, 1) + lo[2]) * nblk_dim(m, L, 0) + lo[1]] = (int32_t)b;
    int s = m->maxl - L;
    for (int64_t z = (int64_t)lo[3] << s; z < ((int64_t)lo[3] + 1) << s; ++z)
      for (int64_t y = (int64_t)lo[2] << s; y < ((int64_t)lo[2] + 1) << s; ++y)
        for (int64_t x = (int64_t)lo[1] << s; x < ((int64_t)lo[1] + 1) << s; ++x) {
          unsigned char *o = &occ[(z * f1 + y) * f0 + x];
          if (*o) rc = ORC_ETILING;
          *o = 1;
        }
  }
  if (rc == ORC_OK)
    for (int64_t q = 0; q < f0 * f1 * f2; ++q)
      if (!occ[q]) { rc = ORC_ETILING; break; }
  free(occ);
  if (rc) return rc;
  /* 2:1 balance over all 26 neighbour directions */
  for (int64_t b = 0; b < m->nl; ++b) {
    const int32_t *lo = m->loc + 4 * b;
    int L = lo[0];
    for (int dz = -1; dz <= 1; ++dz)
      for (int dy = -1; dy <= 1; ++dy)
        for (int dx = -1; dx <= 1; ++dx) {
          if (!dx && !dy && !dz) continue;
          int64_t nb0[3] = {lo[1] + dx, lo[2] + dy, lo[3] + dz}, nb[3];
          if (!block_in_domain(m, L, nb0, nb)) continue; /* beyond the domain boundary */
          if (leaf_at(m, L, nb) >= 0) continue;
          int lc;
          if (coarser_leaf(m, L, nb, &lc) >= 0) {
            if (lc < L - 1) return ORC_EBALANCE;
            continue;
          }
          int del[3] = {dx, dy, dz};
          for (int c = 0; c < 8; ++c) {
            int o[3] = {c & 1, (c >> 1) & 1, (c >> 2) & 1};
            int touch = 1;
            for (int e = 0; e < 3; ++e)
              if ((del[e] < 0 && o[e] == 0) || (del[e] > 0 && o[e] == 1)) touch = 0;
            if (!touch) continue;
            int64_t ch[3] = {2 * nb[0] + o[0], 2 * nb[1] + o[1], 2 * nb[2] + o[2]};
            if (L + 1 > m->maxl || leaf_at(m, L + 1, ch) < 0) return ORC_EBALANCE;
          }
        }
  }
  return ORC_OK;
}

void orc_destroy(void *h) {
  orc_mesh *m = (orc_mesh *)h;
  if (!m) return;
  for (int L = 0; L <= MAXLEV; ++L) free(m->map[L]);
  free(m->loc);
  free(m->U);
  free(m);
}

/* Create a mesh from a leaf list [nl][4] = (level, lx, ly, lz). Leaves are
   stored in Morton order of their deepest-level corner. */
int orc_create(const int32_t *n, const int32_t *nrb, int32_t maxl, const double *xmin,
               const double *xmax, double gamma, double cfl, int32_t recon1,
               const int32_t *bc, const int32_t *locs, int64_t nl, void **out) {
  *out = NULL;
  if (maxl < 0 || maxl > MAXLEV || nl <= 0) return ORC_EINVAL;
  for (int f = 0; f < 6; ++f) {
    int k = bc ? bc[f] : ORC_BC_PERIODIC;
    if (k < ORC_BC_PERIODIC || k > ORC_BC_REFLECT) return ORC_EINVAL;
    /* a periodic direction is periodic on both faces */
    if ((k == ORC_BC_PERIODIC) != ((bc ? bc[f ^ 1] : ORC_BC_PERIODIC) == ORC_BC_PERIODIC)) return ORC_EINVAL;
  }
  for (int d = 0; d < 3; ++d) {
    if (n[d] < 2 || nrb[d] < 1 || (n[d] & 1)) return ORC_EINVAL;
    if (maxl > 0 && n[d] < 8) return ORC_EINVAL;
    if (!(xmax[d] > xmin[d])) return ORC_EINVAL;
  }
  orc_mesh *m = (orc_mesh *)calloc(1, sizeof(orc_mesh));
  if (!m) return ORC_ENOMEM;
  for (int d = 0; d < 3; ++d) {
    m->n[d] = n[d];
    m->nrb[d] = nrb[d];
    m->xmin[d] = xmin[d];
    m->xmax[d] = xmax[d];
  }
  m->maxl = maxl;
  m->gamma = gamma;
  m->cfl = cfl;
  m->recon1 = recon1;
  for (int f = 0; f < 6; ++f) m->bc[f] = bc ? bc[f] : ORC_BC_PERIODIC;
  m->nl = nl;
  m->loc = (int32_t *)malloc(sizeof(int32_t) * 4 * (size_t)nl);
  m->U = (double *)calloc((size_t)(nl * NV * ncell(m)), sizeof(double));
  if (!m->loc || !m->U) { orc_destroy(m); return ORC_ENOMEM; }
  memcpy(m->loc, locs, sizeof(int32_t) * 4 * (size_t)nl);
  g_sort_mesh = m;
  qsort(m->loc, (size_t)nl, 4 * sizeof(int32_t), cmp_loc);
  int rc = build_maps(m);
  if (rc) { orc_destroy(m); return rc; }
  *out = m;
  return ORC_OK;
}

int64_t orc_nleaves(void *h) { return ((orc_mesh *)h)->nl; }
void orc_leaves(void *h, int32_t *out) {
  orc_mesh *m = (orc_mesh *)h;
  memcpy(out, m->loc, sizeof(int32_t) * 4 * (size_t)m->nl);
}
void orc_set_state(void *h, const double *U) {
  orc_mesh *m = (orc_mesh *)h;
  memcpy(m->U, U, sizeof(double) * (size_t)(m->nl * NV * ncell(m)));
  if (m->fp32)
    for (int64_t q = 0; q < m->nl * NV * ncell(m); ++q) m->U[q] = (double)(float)m->U[q];
}

/* Store the state in binary32 from now on (rounds the current state). */
void orc_set_fp32(void *h, int32_t on) {
  orc_mesh *m = (orc_mesh *)h;
  m->fp32 = on ? 1 : 0;
  if (m->fp32)
    for (int64_t q = 0; q < m->nl * NV * ncell(m); ++q) m->U[q] = (double)(float)m->U[q];
}
void orc_get_state(void *h, double *U) {
  orc_mesh *m = (orc_mesh *)h;
  memcpy(U, m->U, sizeof(double) * (size_t)(m->nl * NV * ncell(m)));
}
void orc_set_time(void *h, double t, int64_t cycle) {
  orc_mesh *m = (orc_mesh *)h;
  m->t = t;
  m->cycle = cycle;
}
int orc_error(void *h) { return ((orc_mesh *)h)->err; }

/* Ghost-filled copy of leaf b, [5][n3+4][n2+4][n1+4]. */
int orc_padded(void *h, int64_t b, double *out) {
  orc_mesh *m = (orc_mesh *)h;
  if (b < 0 || b >= m->nl) return ORC_EINVAL;
  fill_padded(m, m->U, b, out);
  return m->err;
}

/* The timestep the next cycle would take (before any t_end clamp). */
double orc_dt(void *h) {
  orc_mesh *m = (orc_mesh *)h;
  return cfl_dt(m, m->U);
}

/* One stage applied to the current state (test hook): U <- U - coef*D(U). */
int orc_stage_inplace(void *h, int32_t recon, double coef) {
  orc_mesh *m = (orc_mesh *)h;
  size_t sz = (size_t)(m->nl * NV * ncell(m));
  double *tmp = (double *)malloc(sizeof(double) * sz);
  if (!tmp) return ORC_ENOMEM;
  int rc = stage(m, m->U, m->U, tmp, recon, coef);
  memcpy(m->U, tmp, sizeof(double) * sz);
  free(tmp);
  return rc;
}

/* n full cycles. Each cycle: dt from the current state (clamped so that
   t does not pass t_end when t_end is finite), predictor
   U* = U^n - dt/2 D_{stage-1 recon}(U^n), corrector
   U^{n+1} = U^n - dt D_PLM(U*). */
int orc_step(void *h, int32_t ncycles, double t_end) {
  orc_mesh *m = (orc_mesh *)h;
  size_t sz = (size_t)(m->nl * NV * ncell(m));
  double *Us = (double *)malloc(sizeof(double) * sz);
  if (!Us) return ORC_ENOMEM;
  int rc = ORC_OK;
  for (int c = 0; c < ncycles; ++c) {
    double dt = cfl_dt(m, m->U);
    if (dt < 0.0) { rc = m->err; break; }
    if (isfinite(t_end) && dt > t_end - m->t) dt = t_end - m->t;
    rc = stage(m, m->U, m->U, Us, m->recon1, 0.5 * dt);
    if (rc) break;
    rc = stage(m, Us, m->U, m->U, 1, dt);
    if (rc) break;
    m->t += dt;
    m->dt_last = dt;
    m->cycle += 1;
  }
  free(Us);
  return rc;
}

/* n full cycles with the given timesteps dts[0..n) instead of the CFL
   timestep (the map a reverse mode with frozen timesteps differentiates). */
int orc_step_dts(void *h, int32_t ncycles, const double *dts) {
  orc_mesh *m = (orc_mesh *)h;
  size_t sz = (size_t)(m->nl * NV * ncell(m));
  double *Us = (double *)malloc(sizeof(double) * sz);
  if (!Us) return ORC_ENOMEM;
  int rc = ORC_OK;
  for (int c = 0; c < ncycles; ++c) {
    double dt = dts[c];
    rc = stage(m, m->U, m->U, Us, m->recon1, 0.5 * dt);
    if (rc) break;
    rc = stage(m, Us, m->U, m->U, 1, dt);
    if (rc) break;
    m->t += dt;
    m->dt_last = dt;
    m->cycle += 1;
  }
  free(Us);
  return rc;
}

/* Start (on = 1, signature reset to 0) or stop recording the branch
   signature of the stages that follow. */
void orc_track_branches(void *h, int32_t on) {
  orc_mesh *m = (orc_mesh *)h;
  m->track = on ? 1 : 0;
  m->sig = 0;
  m->stage_no = 0;
}

uint64_t orc_branch_signature(void *h) { return ((orc_mesh *)h)->sig; }

void orc_time(void *h, double *t, double *dt_last, int64_t *cycle) {
  orc_mesh *m = (orc_mesh *)h;
  *t = m->t;
  *dt_last = m->dt_last;
  *cycle = m->cycle;
}

/* Conserved totals sum U_v dV over leaf active cells, Neumaier-compensated,
   plus the sums of |U_v| dV (the scale relative errors are quoted against). */
void orc_totals(void *h, double *out, double *absout) {
  orc_mesh *m = (orc_mesh *)h;
  for (int v = 0; v < NV; ++v) {
    double s = 0.0, comp_ = 0.0, a = 0.0;
    for (int64_t b = 0; b < m->nl; ++b) {
      int L = m->loc[4 * b];
      double dV = dxl(m, L, 0) * dxl(m, L, 1) * dxl(m, L, 2);
      for (int64_t c = 0; c < ncell(m); ++c) {
        double x = m->U[(b * NV + v) * ncell(m) + c] * dV;
        double t = s + x;
        if (fabs(s) >= fabs(x)) comp_ += (s - t) + x;
        else comp_ += (x - t) + s;
        s = t;
        a += fabs(x);
      }
    }
    out[v] = s + comp_;
    absout[v] = a;
  }
}

/* ------------------------------------------------------------------ */
/* Regridding from per-leaf flags (-1 derefine, 0 keep, +1 refine).     */
/* ------------------------------------------------------------------ */

/* Leaf covering block location nb of level L at a level below L, else -1. */
static int32_t cover_coarser(const orc_mesh *m, int L, const int64_t nb[3], int *lc) {
  return coarser_leaf(m, L, nb, lc);
}

int orc_regrid(void *h, const int8_t *flags, int64_t nflags) {
  orc_mesh *m = (orc_mesh *)h;
  if (nflags != m->nl) return ORC_EINVAL;
  int64_t nl = m->nl;
  char *ref = (char *)calloc((size_t)nl, 1);
  char *der = (char *)calloc((size_t)nl, 1);
  if (!ref || !der) return ORC_ENOMEM;
  for (int64_t b = 0; b < nl; ++b) ref[b] = flags[b] > 0 && m->loc[4 * b] < m->maxl;
  /* a leaf that refines forces every touching coarser leaf to refine */
  for (int changed = 1; changed;) {
    changed = 0;
    for (int64_t b = 0; b < nl; ++b) {
      if (!ref[b]) continue;
      const int32_t *lo = m->loc + 4 * b;
      for (int dz = -1; dz <= 1; ++dz)
        for (int dy = -1; dy <= 1; ++dy)
          for (int dx = -1; dx <= 1; ++dx) {
            if (!dx && !dy && !dz) continue;
            int64_t nb[3] = {lo[1] + dx, lo[2] + dy, lo[3] + dz};
            int lc;
            int32_t c = cover_coarser(m, lo[0], nb, &lc);
            if (c >= 0 && !ref[c]) { ref[c] = 1; changed = 1; }
          }
    }
  }
  /* derefinement: complete sibling groups, all flagged -1, none refining,
     and the merged parent keeps 2:1 against the refined mesh */
  for (int64_t b = 0; b < nl; ++b) {
    const int32_t *lo = m->loc + 4 * b;
    int L = lo[0];
    if (L == 0 || (lo[1] & 1) || (lo[2] & 1) || (lo[3] & 1)) continue;
    int ok = 1;
    int32_t sib[8];
    for (int c = 0; c < 8 && ok; ++c) {
      int64_t ch[3] = {lo[1] + (c & 1), lo[2] + ((c >> 1) & 1), lo[3] + ((c >> 2) & 1)};
      sib[c] = leaf_at(m, L, ch);
      if (sib[c] < 0 || flags[sib[c]] >= 0 || ref[sib[c]]) ok = 0;
    }
    if (!ok) continue;
    int64_t p[3] = {lo[1] >> 1, lo[2] >> 1, lo[3] >> 1};
    for (int dz = -1; dz <= 1 && ok; ++dz)
      for (int dy = -1; dy <= 1 && ok; ++dy)
        for (int dx = -1; dx <= 1 && ok; ++dx) {
          if (!dx && !dy && !dz) continue;
          int64_t q0[3] = {p[0] + dx, p[1] + dy, p[2] + dz}, q[3];
          if (!block_in_domain(m, L - 1, q0, q)) continue;
          int32_t id = leaf_at(m, L - 1, q);
          int lc;
          if (id >= 0 || cover_coarser(m, L - 1, q, &lc) >= 0) continue;
          int del[3] = {dx, dy, dz};
          for (int c = 0; c < 8 && ok; ++c) {
            int o[3] = {c & 1, (c >> 1) & 1, (c >> 2) & 1};
            int touch = 1;
            for (int e = 0; e < 3; ++e)
              if ((del[e] < 0 && o[e] == 0) || (del[e] > 0 && o[e] == 1)) touch = 0;
            if (!touch) continue;
            int64_t ch[3] = {2 * q[0] + o[0], 2 * q[1] + o[1], 2 * q[2] + o[2]};
            int32_t cid = leaf_at(m, L, ch);
            if (cid < 0 || ref[cid]) ok = 0;
          }
        }
    if (ok)
      for (int c = 0; c < 8; ++c) der[sib[c]] = (char)(c == 0 ? 2 : 1);
  }
  /* new leaf list and data */
  int64_t nn = 0;
  for (int64_t b = 0; b < nl; ++b) nn += ref[b] ? 8 : (der[b] == 1 ? 0 : 1);
  int32_t *nloc = (int32_t *)malloc(sizeof(int32_t) * 4 * (size_t)nn);
  int64_t *tag = (int64_t *)malloc(sizeof(int64_t) * 2 * (size_t)nn); /* source leaf, kind */
  if (!nloc || !tag) return ORC_ENOMEM;
  int64_t q = 0;
  for (int64_t b = 0; b < nl; ++b) {
    const int32_t *lo = m->loc + 4 * b;
    if (ref[b]) {
      for (int c = 0; c < 8; ++c) {
        nloc[4 * q] = lo[0] + 1;
        nloc[4 * q + 1] = 2 * lo[1] + (c & 1);
        nloc[4 * q + 2] = 2 * lo[2] + ((c >> 1) & 1);
        nloc[4 * q + 3] = 2 * lo[3] + ((c >> 2) & 1);
        tag[2 * q] = b;
        tag[2 * q + 1] = 1;
        ++q;
      }
    } else if (der[b] == 2) {
      nloc[4 * q] = lo[0] - 1;
      nloc[4 * q + 1] = lo[1] >> 1;
      nloc[4 * q + 2] = lo[2] >> 1;
      nloc[4 * q + 3] = lo[3] >> 1;
      tag[2 * q] = b;
      tag[2 * q + 1] = 2;
      ++q;
    } else if (der[b] == 0) {
      memcpy(nloc + 4 * q, lo, 4 * sizeof(int32_t));
      tag[2 * q] = b;
      tag[2 * q + 1] = 0;
      ++q;
    }
  }
  /* sort new leaves (with their tags) into Morton order */
  int32_t *rec = (int32_t *)malloc(sizeof(int32_t) * 8 * (size_t)nn);
  for (int64_t r = 0; r < nn; ++r) {
    memcpy(rec + 8 * r, nloc + 4 * r, 4 * sizeof(int32_t));
    memcpy(rec + 8 * r + 4, tag + 2 * r, 2 * sizeof(int64_t));
  }
  g_sort_mesh = m;
  qsort(rec, (size_t)nn, 8 * sizeof(int32_t), cmp_loc);
  const int n1 = m->n[0], n2 = m->n[1], n3 = m->n[2];
  double *NU = (double *)malloc(sizeof(double) * (size_t)(nn * NV * ncell(m)));
  if (!NU) return ORC_ENOMEM;
  for (int64_t r = 0; r < nn; ++r) {
    const int32_t *lo = rec + 8 * r;
    int64_t src, kind;
    memcpy(&src, rec + 8 * r + 4, sizeof(int64_t));
    memcpy(&kind, rec + 8 * r + 6, sizeof(int64_t));
    for (int v = 0; v < NV; ++v)
      for (int k = 0; k < n3; ++k)
        for (int j = 0; j < n2; ++j)
          for (int i = 0; i < n1; ++i) {
            double val;
            int64_t J[3] = {(int64_t)lo[1] * n1 + i, (int64_t)lo[2] * n2 + j, (int64_t)lo[3] * n3 + k};
            if (kind == 0) {
              val = uat(m, m->U, src, v, i, j, k);
            } else if (kind == 1) {
              /* new child: prolongation of the composite field at the
                 parent's level on the old mesh */
              int Lp = lo[0] - 1;
              int64_t I[3] = {J[0] >> 1, J[1] >> 1, J[2] >> 1};
              double c0 = comp(m, m->U, Lp, I, v);
              double ss[3];
              for (int d = 0; d < 3; ++d) {
                int64_t Im[3] = {I[0], I[1], I[2]}, Ip[3] = {I[0], I[1], I[2]};
                Im[d] -= 1;
                Ip[d] += 1;
                double s = orc_minmod(c0 - comp(m, m->U, Lp, Im, v), comp(m, m->U, Lp, Ip, v) - c0);
                ss[d] = (J[d] & 1) ? s : -s;
              }
              val = c0 + 0.25 * ((ss[0] + ss[1]) + ss[2]);
            } else {
              /* new parent: restriction of the children */
              double f[2][2][2];
              for (int c = 0; c < 2; ++c)
                for (int bb = 0; bb < 2; ++bb)
                  for (int a = 0; a < 2; ++a) {
                    int64_t Jf[3] = {2 * J[0] + a, 2 * J[1] + bb, 2 * J[2] + c};
                    f[c][bb][a] = comp(m, m->U, lo[0] + 1, Jf, v);
                  }
              val = restrict8(f);
            }
            NU[(((r * NV + v) * n3 + k) * n2 + j) * n1 + i] = val;
          }
  }
  free(m->U);
  m->U = NU;
  free(m->loc);
  m->loc = (int32_t *)malloc(sizeof(int32_t) * 4 * (size_t)nn);
  for (int64_t r = 0; r < nn; ++r) memcpy(m->loc + 4 * r, rec + 8 * r, 4 * sizeof(int32_t));
  m->nl = nn;
  free(rec);
  free(nloc);
  free(tag);
  free(ref);
  free(der);
  return build_maps(m);
}

/* Number of OpenMP threads the oracle's parallel loops use. */
#include <omp.h>
int orc_threads(void) { return omp_get_max_threads(); }
