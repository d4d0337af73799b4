// pkh_hostcheck.cpp -- host build of the pointwise physics and its
// hand-written adjoints, and of the tile-shape choice, exported for the CPU
// unit tests (finite-difference checks of the reverse mode, launch shapes).
// Not used by the GPU path.
#include "pkh_physics.h"
#include "pkh_tiles.h"

using namespace pkh;

namespace {
FState make(const double* w, double gam, double igm1) {
  FState q{w[0], w[1], w[2], w[3], w[4], 0, 0, 0};
  complete_state(q, gam, igm1);
  return q;
}

// PLM face states of the face between cells 1 and 2 of q[4][5] (primitives).
void plm_states(const double* q, double* wl, double* wr) {
  for (int v = 0; v < NVAR; ++v) {
    const double qm2 = q[v], qm1 = q[5 + v], q0 = q[10 + v], qp1 = q[15 + v];
    wl[v] = qm1 + 0.5 * mc_slope(qm1 - qm2, q0 - qm1);
    wr[v] = q0 - 0.5 * mc_slope(q0 - qm1, qp1 - q0);
  }
}
}  // namespace

extern "C" {

int pkhc_tile_rows(int n1, int n2, int tj, long long nblocks, int recon) {
  return stage_tile_rows(n1, n2, tj, nblocks, recon);
}

void pkhc_prim(const double* u, double gam, double* w) { to_prim(u, gam, w); }

void pkhc_prim_rev(const double* u, double gam, const double* gw, double* gu) { prim_rev(u, gam, gw, gu); }

double pkhc_mc(double dl, double dr) { return mc_slope(dl, dr); }

double pkhc_mc_half(double dl, double dr) { return mc_half(dl, dr); }

// HLLE flux from primitive face states; d = 0, 1, 2.
void pkhc_hlle(const double* wl, const double* wr, int d, double gam, double* f) {
  const double igm1 = 1.0 / (gam - 1.0);
  hlle<-1>(make(wl, gam, igm1), make(wr, gam, igm1), gam - 1.0, f, d);
}

// Adjoint of pkhc_hlle w.r.t. the primitive face states.
void pkhc_hlle_rev(const double* wl, const double* wr, int d, double gam, const double* mu, double* gwl,
                   double* gwr) {
  const double igm1 = 1.0 / (gam - 1.0);
  const FState L = make(wl, gam, igm1), R = make(wr, gam, igm1);
  double gL[8] = {0}, gR[8] = {0};
  hlle_rev<-1>(L, R, gam - 1.0, mu, gL, gR, d);
  for (int v = 0; v < NVAR; ++v) gwl[v] = gwr[v] = 0.0;
  complete_state_rev(L, gam, igm1, gL, gwl);
  complete_state_rev(R, gam, igm1, gR, gwr);
}

// PLM + HLLE flux of the face between cells 1 and 2 of four primitive
// states q[4][5].
void pkhc_face_plm(const double* q, int d, double gam, double* f) {
  double wl[5], wr[5];
  plm_states(q, wl, wr);
  pkhc_hlle(wl, wr, d, gam, f);
}

// Adjoint of pkhc_face_plm w.r.t. q[4][5].
void pkhc_face_plm_rev(const double* q, int d, double gam, const double* mu, double* gq) {
  double wl[5], wr[5], gwl[5], gwr[5];
  plm_states(q, wl, wr);
  pkhc_hlle_rev(wl, wr, d, gam, mu, gwl, gwr);
  for (int k = 0; k < 20; ++k) gq[k] = 0.0;
  for (int v = 0; v < NVAR; ++v) {
    const double qm2 = q[v], qm1 = q[5 + v], q0 = q[10 + v], qp1 = q[15 + v];
    double ga, gb;
    // wl = qm1 + S(qm1 - qm2, q0 - qm1) / 2
    mc_branch(qm1 - qm2, q0 - qm1, ga, gb);
    gq[5 + v] += gwl[v] * (1.0 + 0.5 * ga - 0.5 * gb);
    gq[v] -= gwl[v] * 0.5 * ga;
    gq[10 + v] += gwl[v] * 0.5 * gb;
    // wr = q0 - S(q0 - qm1, qp1 - q0) / 2
    mc_branch(q0 - qm1, qp1 - q0, ga, gb);
    gq[10 + v] += gwr[v] * (1.0 - 0.5 * ga + 0.5 * gb);
    gq[5 + v] += gwr[v] * 0.5 * ga;
    gq[15 + v] -= gwr[v] * 0.5 * gb;
  }
}
}
