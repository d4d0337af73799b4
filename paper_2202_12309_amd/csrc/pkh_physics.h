// pkh_physics.h -- pointwise physics of the Euler cycle, for the gfx950
// kernels and (compiled for the host) for the CPU unit tests of the
// hand-written reverse-mode derivatives.
//
// Parthenon Sec. 4.1: piecewise-linear reconstruction (MC limiter, van Leer
// 1977) on primitive variables and HLLE fluxes (Einfeldt 1988 wave speeds
// from Roe averages) for the ideal-gas Euler equations.
#pragma once

#include <math.h>

#if defined(__HIP_DEVICE_COMPILE__)
#define PKH_HD __host__ __device__ __forceinline__
#elif defined(__HIPCC__)
#define PKH_HD __host__ __device__ inline
#else
#define PKH_HD inline
#endif

namespace pkh {

constexpr int NVAR = 5;  // rho, M1, M2, M3, E (conserved) / rho, v1, v2, v3, P (primitive)

// Reciprocal, reciprocal square root and square root from the hardware
// estimates (v_rcp_f64 / v_rsq_f64, relative error ~5e-8 on gfx950) refined
// by one Newton step (relative error below 5e-15, measured over 4M
// arguments spanning 1e-3..1e3). Arguments are positive and normal here
// (densities, pressures, squared sound speeds), so the IEEE special-case
// sequences are not needed; the results enter fluxes whose parity
// tolerance is 1e-12.
PKH_HD double hw_rcp(double x) {
#if defined(__HIP_DEVICE_COMPILE__)
  return __builtin_amdgcn_rcp(x);
#else
  return 1.0 / x;
#endif
}
PKH_HD double hw_rsq(double x) {
#if defined(__HIP_DEVICE_COMPILE__)
  return __builtin_amdgcn_rsq(x);
#else
  return 1.0 / sqrt(x);
#endif
}

PKH_HD double frcp(double x) {
  const double r = hw_rcp(x);
  return fma(r, fma(-x, r, 1.0), r);
}

PKH_HD double frsq(double x) {
  const double r = hw_rsq(x);
  return fma(r, fma(-x * r, 0.5 * r, 0.5), r);
}

PKH_HD double fsqrt(double x) { return x * frsq(x); }

// The pointwise functions below are written with explicit fused
// multiply-adds and with contraction off, so that every inlined copy rounds
// the same way: a kernel may solve the faces of one direction in several
// places, and a face shared by two tiles must get the same flux from both.
PKH_HD bool to_prim(const double u[NVAR], double gam, double w[NVAR]) {
#pragma clang fp contract(off)
  const double ir = frcp(u[0]);
  w[0] = u[0];
  w[1] = u[1] * ir;
  w[2] = u[2] * ir;
  w[3] = u[3] * ir;
  const double mv = fma(u[3], w[3], fma(u[2], w[2], u[1] * w[1]));  // M.v = 2 x kinetic energy
  w[4] = (gam - 1.0) * fma(-0.5, mv, u[4]);
  return (w[0] > 0.0) && (w[4] > 0.0);  // false also for NaN
}

// Monotonised-central limited slope (van Leer 1977), branch free: with
// s = sign(dl), s*MC = max(0, min(2|dl|, 2 s dr, s (dl+dr)/2)); a zero or
// opposite-signed dr gives 0.
PKH_HD double mc_slope(double dl, double dr) {
  const double s = copysign(1.0, dl);
  const double m = fmin(fmin(fabs(dl), s * dr) * 2.0, s * (dl + dr) * 0.5);
  return s * fmax(m, 0.0);
}

// Half the MC slope, MC(dl, dr)/2 = s*max(0, min(|dl|, s dr, s (dl+dr)/4)),
// the offset of a face value from its cell's value. Scaling by powers of two
// is exact, so this equals 0.5 * mc_slope(dl, dr) bit for bit (outside the
// subnormal range) with one multiplication less and the sign applied by a
// bit copy.
PKH_HD double mc_half(double dl, double dr) {
#pragma clang fp contract(off)
  const double s = copysign(1.0, dl);
  const double m = fmin(fmin(fabs(dl), s * dr), copysign(0.25, dl) * (dl + dr));
  return copysign(fmax(m, 0.0), dl);
}

PKH_HD double minmod(double a, double b) {
  const double m = fmin(fabs(a), fabs(b));
  return (a * b > 0.0) ? copysign(m, a) : 0.0;
}

// Face state for the HLLE solver: primitives plus the derived quantities
// the solver needs (sqrt(rho), sound speed, total enthalpy).
struct FState {
  double r, v0, v1, v2, p, sr, c, h;
};

// Derived quantities of a state from its primitives.
PKH_HD void complete_state(FState& q, double gam, double igm1) {
#pragma clang fp contract(off)
  const double is = frsq(q.r);     // 1/sqrt(rho)
  const double ir = is * is;
  q.sr = q.r * is;
  q.c = fsqrt(gam * q.p * ir);
  const double v2 = fma(q.v2, q.v2, fma(q.v1, q.v1, q.v0 * q.v0));
  const double e = fma(0.5 * q.r, v2, q.p * igm1);
  q.h = (e + q.p) * ir;
}

// HLLE flux normal to direction D; Einfeldt (1988) bounds
// b+ = max(u_roe + a_roe, u_R + c_R, 0), b- = min(u_roe - a_roe, u_L - c_L, 0)
// from Roe averages (weights sqrt(rho)). D < 0: the direction is the
// run-time argument drt (one instruction stream for mixed x/y jobs).
template <int D>
PKH_HD void hlle(const FState& L, const FState& R, double gm1, double f[NVAR],
                                     int drt = 0) {
#pragma clang fp contract(off)
  const int d = D >= 0 ? D : drt;
  const double r = L.sr * frcp(L.sr + R.sr), r1 = 1.0 - r;
  const double vb0 = fma(r, L.v0, r1 * R.v0);
  const double vb1 = fma(r, L.v1, r1 * R.v1);
  const double vb2 = fma(r, L.v2, r1 * R.v2);
  const double hb = fma(r, L.h, r1 * R.h);
  const double kb = fma(vb2, vb2, fma(vb1, vb1, vb0 * vb0));
  const double ab = fsqrt(gm1 * fma(-0.5, kb, hb));
  const double vbn = d == 0 ? vb0 : (d == 1 ? vb1 : vb2);
  const double ul = d == 0 ? L.v0 : (d == 1 ? L.v1 : L.v2);
  const double ur = d == 0 ? R.v0 : (d == 1 ? R.v1 : R.v2);
  const double bp = fmax(fmax(vbn + ab, ur + R.c), 0.0);
  const double bm = fmin(fmin(vbn - ab, ul - L.c), 0.0);
  const double ib = frcp(bp - bm);
  const double bpm = bp * bm;
  const double ml = L.r * ul, mr = R.r * ur;  // mass fluxes
  f[0] = fma(bpm, R.r - L.r, fma(bp, ml, -(bm * mr))) * ib;
  const double vl[3] = {L.v0, L.v1, L.v2}, vr[3] = {R.v0, R.v1, R.v2};
#pragma unroll
  for (int c = 0; c < 3; ++c) {
    const double fl = c == d ? fma(ml, vl[c], L.p) : ml * vl[c];
    const double fr = c == d ? fma(mr, vr[c], R.p) : mr * vr[c];
    const double du = fma(R.r, vr[c], -(L.r * vl[c]));
    f[1 + c] = fma(bpm, du, fma(bp, fl, -(bm * fr))) * ib;
  }
  // energy: E = rho h - P, energy flux (E + P) u = m h
  const double el = fma(L.r, L.h, -L.p), er = fma(R.r, R.h, -R.p);
  f[4] = fma(bpm, er - el, fma(bp * ml, L.h, -((bm * mr) * R.h))) * ib;
}


// ---------------------------------------------------------------------------
// Reverse mode (adjoints). Branches of max/min and of the limiter are the
// ones the forward pass takes at the same state; at a tie the first argument
// attaining the extremum (in the order written in the forward) is taken,
// and an MC slope at an extremum (dl*dr <= 0) has zero derivative.
// ---------------------------------------------------------------------------

// Derivative of the MC slope w.r.t. (dl, dr) on the branch the forward takes.
PKH_HD void mc_branch(double dl, double dr, double& ga, double& gb) {
  ga = 0.0;
  gb = 0.0;
  if (!(dl * dr > 0.0)) return;
  const double a = 2.0 * fabs(dl), b = 2.0 * fabs(dr), c = 0.5 * fabs(dl + dr);
  if (a <= b && a <= c) {
    ga = 2.0;
  } else if (b <= c) {
    gb = 2.0;
  } else {
    ga = 0.5;
    gb = 0.5;
  }
}

// Adjoint of complete_state: g = adjoints of (r, v0, v1, v2, p, sr, c, h);
// accumulates the primitive adjoint into gw.
PKH_HD void complete_state_rev(const FState& q, double gam, double igm1, const double g[8],
                               double gw[NVAR]) {
  const double ir = frcp(q.r);
  const double v2 = q.v0 * q.v0 + q.v1 * q.v1 + q.v2 * q.v2;
  const double e = q.p * igm1 + 0.5 * q.r * v2;
  double gr = g[0], gp = g[4], gir = 0.0;
  double gv[3] = {g[1], g[2], g[3]};
  // h = (e + p) / r
  const double ge = g[7] * ir;
  gp += g[7] * ir;
  gir += g[7] * (e + q.p);
  // c = sqrt(gam p / r)
  const double hc = 0.5 * frcp(q.c);
  gp += g[6] * gam * ir * hc;
  gir += g[6] * gam * q.p * hc;
  // e = p/(gam-1) + r |v|^2 / 2
  gp += ge * igm1;
  gr += ge * 0.5 * v2;
  gv[0] += ge * q.r * q.v0;
  gv[1] += ge * q.r * q.v1;
  gv[2] += ge * q.r * q.v2;
  // sr = sqrt(r), ir = 1/r
  gr += g[5] * 0.5 * frcp(q.sr);
  gr -= gir * ir * ir;
  gw[0] += gr;
  gw[1] += gv[0];
  gw[2] += gv[1];
  gw[3] += gv[2];
  gw[4] += gp;
}

// Adjoint of hlle<D>: given mu = dL/dF, accumulate the adjoints of the two
// face states' fields (r, v0, v1, v2, p, sr, c, h) into gL and gR.
template <int D>
PKH_HD void hlle_rev(const FState& L, const FState& R, double gm1, const double mu[NVAR],
                     double gL[8], double gR[8], int drt = 0) {
  const int d = D >= 0 ? D : drt;
  // forward recomputation
  const double isum = frcp(L.sr + R.sr);
  const double r = L.sr * isum, r1 = 1.0 - r;
  const double vl[3] = {L.v0, L.v1, L.v2}, vr[3] = {R.v0, R.v1, R.v2};
  double vb[3];
  for (int c = 0; c < 3; ++c) vb[c] = r * vl[c] + r1 * vr[c];
  const double hb = r * L.h + r1 * R.h;
  const double q = hb - 0.5 * (vb[0] * vb[0] + vb[1] * vb[1] + vb[2] * vb[2]);
  const double ab = fsqrt(gm1 * q);
  const double vbn = vb[d], ul = vl[d], ur = vr[d];
  const double a1 = vbn + ab, a2 = ur + R.c;
  const int kp = (a1 >= a2 && a1 >= 0.0) ? 0 : (a2 >= 0.0 ? 1 : 2);
  const double bp = kp == 0 ? a1 : (kp == 1 ? a2 : 0.0);
  const double b1 = vbn - ab, b2 = ul - L.c;
  const int km = (b1 <= b2 && b1 <= 0.0) ? 0 : (b2 <= 0.0 ? 1 : 2);
  const double bm = km == 0 ? b1 : (km == 1 ? b2 : 0.0);
  const double ib = frcp(bp - bm);
  const double bpm = bp * bm;
  const double ml = L.r * ul, mr = R.r * ur;
  const double el = L.r * L.h - L.p, er = R.r * R.h - R.p;
  double N[NVAR];
  N[0] = bp * ml - bm * mr + bpm * (R.r - L.r);
  for (int c = 0; c < 3; ++c)
    N[1 + c] = bp * (ml * vl[c] + (c == d ? L.p : 0.0)) - bm * (mr * vr[c] + (c == d ? R.p : 0.0)) +
               bpm * (R.r * vr[c] - L.r * vl[c]);
  N[4] = bp * ml * L.h - bm * mr * R.h + bpm * (er - el);
  // reverse
  double gib = 0.0;
  for (int v = 0; v < NVAR; ++v) gib += mu[v] * N[v];
  double gbp = -gib * ib * ib, gbm = gib * ib * ib, gbpm = 0.0, gml = 0.0, gmr = 0.0;
  double t = mu[0] * ib;
  gbp += t * ml;
  gbm -= t * mr;
  gbpm += t * (R.r - L.r);
  gml += t * bp;
  gmr -= t * bm;
  gR[0] += t * bpm;
  gL[0] -= t * bpm;
  for (int c = 0; c < 3; ++c) {
    t = mu[1 + c] * ib;
    const double FL = ml * vl[c] + (c == d ? L.p : 0.0), FR = mr * vr[c] + (c == d ? R.p : 0.0);
    gbp += t * FL;
    gbm -= t * FR;
    gbpm += t * (R.r * vr[c] - L.r * vl[c]);
    gml += t * bp * vl[c];
    gL[1 + c] += t * (bp * ml - bpm * L.r);
    gmr -= t * bm * vr[c];
    gR[1 + c] += t * (bpm * R.r - bm * mr);
    gR[0] += t * bpm * vr[c];
    gL[0] -= t * bpm * vl[c];
    if (c == d) {
      gL[4] += t * bp;
      gR[4] -= t * bm;
    }
  }
  t = mu[4] * ib;
  gbp += t * ml * L.h;
  gbm -= t * mr * R.h;
  gbpm += t * (er - el);
  gml += t * bp * L.h;
  gL[7] += t * bp * ml;
  gmr -= t * bm * R.h;
  gR[7] -= t * bm * mr;
  const double ger = t * bpm, gel = -t * bpm;
  // e = r h - p
  gR[0] += ger * R.h;
  gR[7] += ger * R.r;
  gR[4] -= ger;
  gL[0] += gel * L.h;
  gL[7] += gel * L.r;
  gL[4] -= gel;
  // bpm = bp bm
  gbp += gbpm * bm;
  gbm += gbpm * bp;
  // mass fluxes
  gL[0] += gml * ul;
  double gul = gml * L.r;
  gR[0] += gmr * ur;
  double gur = gmr * R.r;
  // wave-speed bounds on the frozen branches
  double gvbn = 0.0, gab = 0.0;
  if (kp == 0) {
    gvbn += gbp;
    gab += gbp;
  } else if (kp == 1) {
    gur += gbp;
    gR[6] += gbp;
  }
  if (km == 0) {
    gvbn += gbm;
    gab -= gbm;
  } else if (km == 1) {
    gul += gbm;
    gL[6] -= gbm;
  }
  // ab = sqrt(gm1 q)
  const double gq = gab * gm1 * 0.5 * frcp(ab);
  const double ghb = gq;
  double gvb[3];
  for (int c = 0; c < 3; ++c) gvb[c] = -gq * vb[c];
  gvb[d] += gvbn;
  // Roe averages
  double gr = ghb * (L.h - R.h);
  gL[7] += ghb * r;
  gR[7] += ghb * r1;
  for (int c = 0; c < 3; ++c) {
    gr += gvb[c] * (vl[c] - vr[c]);
    gL[1 + c] += gvb[c] * r;
    gR[1 + c] += gvb[c] * r1;
  }
  gL[1 + d] += gul;
  gR[1 + d] += gur;
  gL[5] += gr * R.sr * isum * isum;
  gR[5] -= gr * L.sr * isum * isum;
}

// Adjoint of the primitive recovery: gw (adjoint of rho, v, P) -> gu
// (adjoint of rho, M, E) at the conserved state u.
PKH_HD void prim_rev(const double u[NVAR], double gam, const double gw[NVAR], double gu[NVAR]) {
  const double ir = frcp(u[0]);
  const double v0 = u[1] * ir, v1 = u[2] * ir, v2 = u[3] * ir;
  const double g1 = (gam - 1.0) * gw[4];
  gu[0] = gw[0] - (gw[1] * v0 + gw[2] * v1 + gw[3] * v2) * ir + g1 * 0.5 * (v0 * v0 + v1 * v1 + v2 * v2);
  gu[1] = gw[1] * ir - g1 * v0;
  gu[2] = gw[2] * ir - g1 * v1;
  gu[3] = gw[3] * ir - g1 * v2;
  gu[4] = g1;
}

}  // namespace pkh
