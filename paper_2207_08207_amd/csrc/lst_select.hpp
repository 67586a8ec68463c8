// Device-side selections of the Line Segment Tracking chain (arXiv:2207.08207,
// Sections 2.2-2.5) for gfx950.
//
// Numerics: built with -ffp-contract=off and correctly rounded f32 divide and
// sqrt, no denormal flushing.  Every expression below is evaluated as one IEEE
// binary32 operation per + - * / sqrt, in the parenthesised order written, so
// a decision taken here is the decision the same formula takes on any IEEE
// host.  Transcendentals never feed a cut: the pT-threshold windows that need
// asin are per-module constants (module_windows, f64, series asin), arc
// lengths use the asin(x)/x Maclaurin series, angles are compared through
// cross and dot products.  atan2f only produces the reported segment angles.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace lst {

// ---- physics constants (B = 3.8 T, pT threshold 0.8 GeV, Section 2.2) ----
// (The transverse impact-parameter bound d0 of the selections is a parameter
// of the detector description, DevGeom::d0max: 0.1 cm by default, wider for
// displaced tracks.)
constexpr double kCurvD = 0.299792458 * 3.8 / 100.0;  // |kappa| = kCurvD / pT  [1/cm, GeV]
constexpr double kPtMinD = 0.8;
constexpr double kZLumD = 20.0;   // luminous-region half length [cm]

constexpr float kCurv = (float)kCurvD;
constexpr float kHalfKmax = (float)(kCurvD / kPtMinD / 2.0);
constexpr float kKmaxCut = (float)(kCurvD / kPtMinD * 1.01);
constexpr float kZLum = (float)kZLumD;
constexpr float kTau = (float)0.8;        // bound on sin(track-to-radial angle), endcap x-y error
constexpr float kXT3 = (float)10.0;       // T3 r-z chi2
// T5 chi2 cuts: per quintuplet category, DevGeom::t5cut (t5_category below).
constexpr float kXPxy3 = (float)50.0, kXPxy5 = (float)80.0;
constexpr float kXPrz3 = (float)50.0, kXPrz5 = (float)80.0;
constexpr float kBoxXY = (float)1.0;      // seed window at the first anchor, x-y [cm]
constexpr float kBoxZ0 = (float)3.0;      // seed window at the first anchor, z base [cm]
constexpr float kSeedDpt = (float)0.02;   // relative seed curvature resolution
constexpr float kSeedDdir = (float)0.001; // seed direction resolution [rad]
constexpr float kDpT3 = (float)0.02, kDT5 = (float)0.02, kDpLS = (float)0.05;  // eta-phi proximity
constexpr float kXSeriesMax = (float)0.7;
constexpr float kC1 = (float)(1.0 / 6.0), kC2 = (float)0.075, kC3 = (float)(5.0 / 112.0),
                kC4 = (float)(35.0 / 1152.0), kC5 = (float)(63.0 / 2816.0);
constexpr float kThird = (float)(1.0 / 3.0);
constexpr float kMargin = (float)1.001, kEps = (float)1e-6;

// Half pitches of a module type (0 PS, 1 2S): r-phi and long coordinate [cm].
__device__ __forceinline__ float half_rphi(int type2s) { return type2s ? (float)0.0045 : (float)0.005; }
__device__ __forceinline__ float half_long(int type2s) { return type2s ? (float)2.5 : (float)0.075; }

// Module info word: bit 0 = 2S, bit 1 = endcap.
struct ModInfo {
  int bits;
  __device__ __forceinline__ int is2s() const { return bits & 1; }
  __device__ __forceinline__ int endcap() const { return (bits >> 1) & 1; }
  __device__ __forceinline__ float hphi() const { return half_rphi(bits & 1); }
  __device__ __forceinline__ float hlong() const { return half_long(bits & 1); }
  // x-y position error transverse to the track
  __device__ __forceinline__ float sig_t() const { return endcap() ? hphi() + kTau * hlong() : hphi(); }
  // z error for a track of slope lam = dz/ds
  __device__ __forceinline__ float sig_z(float lam) const {
    return endcap() ? hlong() * fabsf(lam) + (float)0.01 : hlong();
  }
  // long-coordinate error that enters as a z error (barrel) / as a radius error (endcap)
  __device__ __forceinline__ float ez() const { return endcap() ? 0.0f : hlong(); }
  __device__ __forceinline__ float er() const { return endcap() ? hlong() : 0.0f; }
};

// asin(x)/x, Maclaurin series through x^8 (a lower bound of it).
__device__ __forceinline__ float arc_over_chord(float x) {
  float x2 = x * x;
  return 1.0f + x2 * (kC1 + x2 * (kC2 + x2 * (kC3 + x2 * kC4)));
}

// ------------------------------------------------------------------ windows
// asin in double from its Maclaurin series (+ * / only, fixed order).
__device__ __forceinline__ double series_asin(double x) {
  double x2 = x * x, term = x, acc = x;
  for (int n = 0; n < 200; ++n) {
    term = term * x2;
    term = term * (double)((2 * n + 1) * (2 * n + 1));
    term = term / (double)((2 * n + 2) * (2 * n + 3));
    acc = acc + term;
  }
  return acc;
}

// Mini-doublet windows of one module (Section 2.2), in double.
//  W  bound on |sin(azimuth change)| between the two hits;
//  PS barrel: |z_up - A1 z_lo| <= A2 + A3 |z_lo|;  PS endcap: -A2 <= r_up - r_lo <= A1 r_lo + A2.
__device__ inline void module_windows(int endcap, int type2s, double p_lo, double p_up, double l_min, double l_max,
                                      double d0, double w[4]) {
  const double km = kCurvD / kPtMinD;
  const double hp = type2s ? 0.0045 : 0.005;
  const double hl = type2s ? 2.5 : 0.075;
  double W, A1 = 0.0, A2 = 0.0, A3 = 0.0;
  if (!endcap) {
    const double r1 = p_lo, r2 = p_up;
    const double a1 = series_asin(km * r1 / 2.0), a2 = series_asin(km * r2 / 2.0);
    const double dphi = (a2 - a1) + d0 * (1.0 / r1 - 1.0 / r2) + hp / r1 + hp / r2;
    W = dphi * (1.0 + 1e-3) + 1e-6;
    if (!type2s) {
      const double a = r2 / r1;
      const double s1 = 2.0 * a1 / km, s2 = 2.0 * a2 / km;
      const double ap = s2 / s1;
      A1 = a;
      A2 = ((ap - 1.0) * kZLumD + hl * (1.0 + a) + (ap - a) * hl) * (1.0 + 1e-3);
      A3 = (ap - a) * (1.0 + 1e-3);
    }
  } else {
    const double z1 = p_lo, z2 = p_up, rmin = l_min, rmax = l_max;
    const double xg = km * (rmax + hl) / 2.0;
    const double gmax = series_asin(xg) / xg;
    const double k = (z2 - z1) * gmax / (z1 - kZLumD);
    const double b1 = series_asin(km * rmax / 2.0), b2 = series_asin(km * rmax * (1.0 + k) / 2.0);
    const double dphi = (b2 - b1) + d0 * k / rmin + 2.0 * hp / rmin;
    W = dphi * (1.0 + 1e-3) + 1e-6;
    if (!type2s) {
      A1 = k * (1.0 + 1e-3);
      A2 = (2.0 * hl + k * hl) * (1.0 + 1e-3);
    }
  }
  w[0] = W; w[1] = A1; w[2] = A2; w[3] = A3;
}

// -------------------------------------------------------------- MD (S2.2)
// Hit pair (lower i, upper j) of one module.  hi/hj = (x, y, z, r).
__device__ __forceinline__ bool md_pass(const float4 &hi, const float4 &hj, const float4 &win, ModInfo mi) {
  const float c = hi.x * hj.y - hi.y * hj.x;
  const float d = hi.x * hj.x + hi.y * hj.y;
  if (!(d > 0.0f)) return false;
  bool ok = fabsf(c) <= win.x * (hi.w * hj.w);
  if (!mi.is2s()) {
    if (!mi.endcap()) {
      const float t = hj.z - win.y * hi.z;
      ok &= fabsf(t) <= win.z + win.w * fabsf(hi.z);
    } else {
      const float dr = hj.w - hi.w;
      ok &= -dr <= win.z;
      ok &= dr <= win.y * hi.w + win.z;
    }
  }
  return ok;
}

// Stub of an MD: tangential displacement between its hits, seen from the
// lower hit, and its separation along the sensor normal (radius in the
// barrel, |z| in the endcap).
__device__ __forceinline__ float2 md_stub(const float4 &hi, const float4 &hj, ModInfo mi) {
  const float tau = (hi.x * hj.y - hi.y * hj.x) / hi.w;
  const float dl = mi.endcap() ? fabsf(hj.z) - fabsf(hi.z) : hj.w - hi.w;
  return make_float2(tau, dl);
}

// -------------------------------------------------------------- LS (S2.2)
// Reported angles of a segment: the chord AB against the radial direction at A
// and at B.
__device__ __forceinline__ float2 ls_beta(const float4 &A, const float4 &B) {
  const float sx = B.x - A.x, sy = B.y - A.y;
  return make_float2(atan2f(A.x * sy - A.y * sx, A.x * sx + A.y * sy), atan2f(B.x * sy - B.y * sx, B.x * sx + B.y * sy));
}

// One MD's stub direction against the chord AB (stub st = (tangential
// displacement, sensor separation), sn = sine of the chord's angle to the
// radial direction used for it, rp its radius).
__device__ __forceinline__ bool ls_stub_ok(float2 st, ModInfo m, float sn, float rp, float Ls, float adz, float eang,
                                           float d0) {
  float pred, err;
  if (!m.endcap()) {
    const float cs2 = 1.0f - sn * sn;
    if (!(cs2 > 0.0f)) return false;
    pred = (st.y * sn) / sqrtf(cs2);
    err = 2.0f * m.hphi() + (2.0f * st.y) * (eang + d0 / rp);
  } else {
    if (!(adz > 0.0f)) return false;
    const float ds = (st.y * Ls) / adz;
    pred = ds * sn;
    err = (2.0f * m.hphi() + (float)0.03 * fabsf(pred)) + ds * (eang + d0 / rp);
  }
  const float dt = st.x - pred;
  return fabsf(dt) <= err * kMargin + kEps;
}

// MDs a (anchor A, stub sa, module ma) and b (B, sb, mb), the modules linked
// by the map.  x-y azimuth window from the beam line, r-z pointing to the
// luminous region, and each stub's direction against the origin-constrained
// chord.  Returns the reported angles in *beta.
__device__ __forceinline__ bool ls_pass(const float4 &A, const float4 &B, float2 sa, float2 sb, ModInfo ma,
                                        ModInfo mb, float2 *beta, float d0) {
  const float dr = B.w - A.w;
  if (!(dr > 0.0f)) return false;
  const float ea = ma.er(), eb = mb.er();
  const float c = A.x * B.y - A.y * B.x;
  const float d = A.x * B.x + A.y * B.y;
  if (!(d > 0.0f)) return false;
  const float ub = kHalfKmax * (B.w + eb);
  const float ua = kHalfKmax * (A.w - ea);
  const float w = (((ub - ua) / sqrtf(1.0f - ub * ub) + (d0 * dr) / (A.w * B.w)) + ma.hphi() / A.w) +
                  mb.hphi() / B.w;
  const float Wn = w * kMargin + kEps;
  bool ok = fabsf(c) <= Wn * (A.w * B.w);
  // r-z: z0 of the chord over the arc-length ratios allowed by the threshold
  const float xa = kHalfKmax * A.w, xb = kHalfKmax * B.w;
  const float xb2 = xb * xb;
  float x10 = xb2 * xb2;
  x10 = (x10 * x10) * xb2;
  const float ghi = arc_over_chord(xb) + (kC5 * x10) / (1.0f - xb2);
  const float t_hi = A.w / B.w;
  const float t_lo = (A.w * arc_over_chord(xa)) / (B.w * ghi);
  const float z0a = (A.z - t_lo * B.z) / (1.0f - t_lo);
  const float z0b = (A.z - t_hi * B.z) / (1.0f - t_hi);
  const float zlo = z0a < z0b ? z0a : z0b;
  const float zhi = z0a < z0b ? z0b : z0a;
  const float Ez = (ma.ez() + t_hi * mb.ez()) / (1.0f - t_hi);
  const float dz = B.z - A.z;
  const float Er = ((B.w * ea + A.w * eb) * fabsf(dz)) / (dr * dr);
  const float L = (kZLum + (Ez + Er)) * kMargin;
  ok &= zlo <= L;
  ok &= -zhi <= L;
  // stub directions against the chord through the beam line
  const float sx = B.x - A.x, sy = B.y - A.y;
  const float Ls = sqrtf(sx * sx + sy * sy);
  const float s_out = (B.x * sy - B.y * sx) / (B.w * Ls);
  const float s_in = (A.x * sy - A.y * sx) / (A.w * Ls);
  const float adz = fabsf(dz);
  const float ea2 = ma.endcap() ? ma.hlong() : ma.hphi();
  const float eb2 = mb.endcap() ? mb.hlong() : mb.hphi();
  const float eang = (ea2 + eb2) / Ls;
  ok &= ls_stub_ok(sa, ma, s_out, A.w, Ls, adz, eang, d0);
  ok &= ls_stub_ok(sb, mb, s_in, B.w, Ls, adz, eang, d0);
  if (ok) *beta = ls_beta(A, B);
  return ok;
}

// The inner MD's stub check of ls_pass on its own, with the same operations in
// the same order: a candidate failing it fails ls_pass.
__device__ __forceinline__ bool ls_inner_stub_ok(const float4 &A, const float4 &B, float2 sa, ModInfo ma, ModInfo mb,
                                                 float d0) {
  const float dz = B.z - A.z;
  const float sx = B.x - A.x, sy = B.y - A.y;
  const float Ls = sqrtf(sx * sx + sy * sy);
  const float s_out = (B.x * sy - B.y * sx) / (B.w * Ls);
  const float adz = fabsf(dz);
  const float ea2 = ma.endcap() ? ma.hlong() : ma.hphi();
  const float eb2 = mb.endcap() ? mb.hlong() : mb.hphi();
  const float eang = (ea2 + eb2) / Ls;
  return ls_stub_ok(sa, ma, s_out, A.w, Ls, adz, eang, d0);
}

// Azimuth linear in z over three anchors P, Q, R (Section 2.3 pointing for a
// helix from the beam line): sin(phiQ-phiP)(zR-zQ) = sin(phiR-phiQ)(zQ-zP).
__device__ __forceinline__ bool phiz_pass(const float4 &P, const float4 &Q, const float4 &R, ModInfo mp, ModInfo mq,
                                          ModInfo mr, float d0) {
  const float su = (P.x * Q.y - P.y * Q.x) / (P.w * Q.w);
  const float sv = (Q.x * R.y - Q.y * R.x) / (Q.w * R.w);
  const float dzpq = Q.z - P.z, dzqr = R.z - Q.z;
  const float res = su * dzqr - sv * dzpq;
  const float iP = 1.0f / P.w, iQ = 1.0f / Q.w, iR = 1.0f / R.w;
  const float dpq = iP - iQ, dqr = iQ - iR;
  const float ePQ = (mp.hphi() * iP + mq.hphi() * iQ) + d0 * fabsf(dpq);
  const float eQR = (mq.hphi() * iQ + mr.hphi() * iR) + d0 * fabsf(dqr);
  const float au = fabsf(su), av = fabsf(sv), adpq = fabsf(dzpq), adqr = fabsf(dzqr);
  const float nl = (au * au + av * av) * kThird;
  const float tol = ((adqr * ePQ + adpq * eQR) + (au * (mq.ez() + mr.ez()) + av * (mp.ez() + mq.ez()))) +
                    nl * (au * adqr + av * adpq);
  return fabsf(res) <= tol * kMargin + kEps;
}

// Weighted straight line z = alpha + lambda s over N points; returns chi2.
template <int N>
__device__ __forceinline__ float line_chi2(const float *s, const float *z, const float *w, float *lam_out) {
  float S = 0.0f, Ss = 0.0f, Sz = 0.0f;
#pragma unroll
  for (int i = 0; i < N; ++i) {
    S = S + w[i];
    Ss = Ss + w[i] * s[i];
    Sz = Sz + w[i] * z[i];
  }
  const float sbar = Ss / S, zbar = Sz / S;
  float Sss = 0.0f, Ssz = 0.0f;
#pragma unroll
  for (int i = 0; i < N; ++i) {
    const float ds = s[i] - sbar, dzz = z[i] - zbar;
    Sss = Sss + (w[i] * ds) * ds;
    Ssz = Ssz + (w[i] * ds) * dzz;
  }
  const float lam = Ssz / Sss;
  float chi2 = 0.0f;
#pragma unroll
  for (int i = 0; i < N; ++i) {
    const float r = (z[i] - zbar) - lam * (s[i] - sbar);
    chi2 = chi2 + (w[i] * r) * r;
  }
  *lam_out = lam;
  return chi2;
}

// -------------------------------------------------------------- T3 (S2.3)
// Anchors A, B, C of LS (a,b) + LS (b,c).  out = (kappa, dkappa, chi2_rz, lambda).
__device__ __forceinline__ bool t3_pass(const float4 &A, const float4 &B, const float4 &C, ModInfo mA, ModInfo mB,
                                        ModInfo mC, float4 *out, float d0) {
  const float ux = B.x - A.x, uy = B.y - A.y, wx = C.x - A.x, wy = C.y - A.y, tx = C.x - B.x, ty = C.y - B.y;
  const float k = ux * wy - uy * wx;
  const float Lu = sqrtf(ux * ux + uy * uy), Lw = sqrtf(wx * wx + wy * wy), Lt = sqrtf(tx * tx + ty * ty);
  const float kap = (2.0f * k) / ((Lu * Lw) * Lt);
  const float dk = (4.0f * ((mA.sig_t() + 2.0f * mB.sig_t()) + mC.sig_t())) / (Lw * Lw);
  if (!(fabsf(kap) <= kKmaxCut + dk)) return false;
  if (!phiz_pass(A, B, C, mA, mB, mC, d0)) return false;
  const float xa = (kap * Lu) * 0.5f, xb = (kap * Lt) * 0.5f;
  if (!(fabsf(xa) <= kXSeriesMax) || !(fabsf(xb) <= kXSeriesMax)) return false;
  float s[3], z[3], w[3];
  s[0] = 0.0f;
  s[1] = Lu * arc_over_chord(xa);
  s[2] = s[1] + Lt * arc_over_chord(xb);
  z[0] = A.z; z[1] = B.z; z[2] = C.z;
  const float lam0 = (C.z - A.z) / s[2];
  const ModInfo mm[3] = {mA, mB, mC};
#pragma unroll
  for (int i = 0; i < 3; ++i) {
    const float sg = mm[i].sig_z(lam0);
    w[i] = 1.0f / (sg * sg);
  }
  float lam;
  const float chi2 = line_chi2<3>(s, z, w, &lam);
  if (!(chi2 <= kXT3)) return false;
  *out = make_float4(kap, dk, chi2, lam);
  return true;
}

// -------------------------------------------------------------- T5 (S2.3)
// Category of a quintuplet (Section 2.3 sets its chi2 cuts per category):
// the ordered kinds of the five anchor modules, innermost first, kind = the
// module info word (2 * endcap + 2S), index sum_i kind_i 4^i in [0, 1024).
__device__ __forceinline__ int t5_category(const ModInfo *M) {
  return (((M[4].bits * 4 + M[3].bits) * 4 + M[2].bits) * 4 + M[1].bits) * 4 + M[0].bits;
}

// Anchors P[0..4]; tin/tout = (kappa, dkappa, ...) of the two triplets;
// cuts = (chi2_xy, chi2_rz) bounds of each category.
// out[0..7] = kappa5, chi2_xy, chi2_rz, lambda, kappa_in, kappa_out, dir_x, dir_y.
__device__ __forceinline__ bool t5_pass(const float4 *P, const ModInfo *M, float4 tin, float4 tout, float *out,
                                        float d0, const float2 *__restrict__ cuts) {
  const float dkk = tin.x - tout.x;
  if (!(fabsf(dkk) <= tin.y + tout.y)) return false;
  if (!phiz_pass(P[0], P[2], P[4], M[0], M[2], M[4], d0)) return false;
  // circle v = a + b u + c (u^2 + v^2) in the frame of the chord from P0 to P4, unit = chord
  const float ex = P[4].x - P[0].x, ey = P[4].y - P[0].y;
  const float L = sqrtf(ex * ex + ey * ey);
  const float ux = ex / L, uy = ey / L;
  float u[5], v[5], q[5], w[5];
#pragma unroll
  for (int i = 0; i < 5; ++i) {
    const float dx = P[i].x - P[0].x, dy = P[i].y - P[0].y;
    u[i] = (dx * ux + dy * uy) / L;
    v[i] = (dy * ux - dx * uy) / L;
    q[i] = u[i] * u[i] + v[i] * v[i];
    const float t = L / M[i].sig_t();
    w[i] = t * t;
  }
  float S0 = 0.0f, S1 = 0.0f, S2 = 0.0f, S11 = 0.0f, S12 = 0.0f, S22 = 0.0f, T0 = 0.0f, T1 = 0.0f, T2 = 0.0f;
#pragma unroll
  for (int i = 0; i < 5; ++i) {
    S0 = S0 + w[i];
    S1 = S1 + w[i] * u[i];
    S2 = S2 + w[i] * q[i];
    S11 = S11 + (w[i] * u[i]) * u[i];
    S12 = S12 + (w[i] * u[i]) * q[i];
    S22 = S22 + (w[i] * q[i]) * q[i];
    T0 = T0 + w[i] * v[i];
    T1 = T1 + (w[i] * u[i]) * v[i];
    T2 = T2 + (w[i] * q[i]) * v[i];
  }
  const float m00 = S11 * S22 - S12 * S12;
  const float m01 = S1 * S22 - S12 * S2;
  const float m02 = S1 * S12 - S11 * S2;
  const float det = (S0 * m00 - S1 * m01) + S2 * m02;
  if (!(det > 0.0f)) return false;
  const float n1 = T1 * S22 - S12 * T2;
  const float n2 = T1 * S12 - S11 * T2;
  const float n3 = S1 * T2 - T1 * S2;
  const float deta = (T0 * m00 - S1 * n1) + S2 * n2;
  const float detb = (S0 * n1 - T0 * m01) + S2 * n3;
  const float detc = (S0 * (S11 * T2 - T1 * S12) - S1 * n3) + T0 * m02;
  const float fa = deta / det, fb = detb / det, fc = detc / det;
  float chi2xy = 0.0f;
#pragma unroll
  for (int i = 0; i < 5; ++i) {
    const float r = v[i] - ((fa + fb * u[i]) + fc * q[i]);
    chi2xy = chi2xy + (w[i] * r) * r;
  }
  const float2 cut = cuts[t5_category(M)];
  if (!(chi2xy <= cut.x)) return false;
  const float disc = (1.0f + fb * fb) - (4.0f * fa) * fc;
  if (!(disc > 0.0f)) return false;
  const float k5 = (2.0f * fc) / (L * sqrtf(disc));
  // r-z line over the arc lengths along the anchors with the mean triplet curvature
  const float kb = (tin.x + tout.x) * 0.5f;
  float s[5], z[5];
  s[0] = 0.0f;
#pragma unroll
  for (int i = 1; i < 5; ++i) {
    const float dx = P[i].x - P[i - 1].x, dy = P[i].y - P[i - 1].y;
    const float Lc = sqrtf(dx * dx + dy * dy);
    const float xs = (kb * Lc) * 0.5f;
    if (!(fabsf(xs) <= kXSeriesMax)) return false;
    s[i] = s[i - 1] + Lc * arc_over_chord(xs);
  }
#pragma unroll
  for (int i = 0; i < 5; ++i) z[i] = P[i].z;
  const float lam0 = (P[4].z - P[0].z) / s[4];
#pragma unroll
  for (int i = 0; i < 5; ++i) {
    const float sg = M[i].sig_z(lam0);
    w[i] = 1.0f / (sg * sg);
  }
  float lam;
  const float chi2rz = line_chi2<5>(s, z, w, &lam);
  if (!(chi2rz <= cut.y)) return false;
  const float nb = sqrtf(1.0f + fb * fb);
  const float cx = (ux - fb * uy) / nb, cy = (uy + fb * ux) / nb;
  out[0] = k5; out[1] = chi2xy; out[2] = chi2rz; out[3] = lam;
  out[4] = tin.x; out[5] = tout.x;
  out[6] = cx + k5 * P[0].y;
  out[7] = cy - k5 * P[0].x;
  return true;
}

// ------------------------------------------------- track extensions (S2.5)
// A candidate's MD chain lengthened by one triplet (its last one or two MDs
// shared) is tested with the quintuplet's fits widened to the n = 4..7
// anchors of the chain: the circle in x-y (chi2 <= 10 per degree of freedom,
// N - 3) and the straight line in (arc length, z) (chi2 <= 20/3 per degree
// of freedom, N - 2), arc lengths taken with the fitted circle's curvature.
// out = (chi2_xy, chi2_rz, kappa).
constexpr double kXExtXyD = 10.0, kXExtRzD = 20.0 / 3.0;

// Room for the longest chain (a five-MD candidate plus two MDs); a chain of
// n < kExtMax anchors occupies P[0..n) and every sum skips the slots past it,
// so each term enters in the order a fit over exactly n anchors adds it.
constexpr int kExtMax = 7;

__device__ __forceinline__ bool ext_fit(const float4 *P, const ModInfo *M, int n, float3 *out) {
  float4 PL = P[0];
#pragma unroll
  for (int i = 1; i < kExtMax; ++i)
    if (i == n - 1) PL = P[i];
  const float ex = PL.x - P[0].x, ey = PL.y - P[0].y;
  const float L = sqrtf(ex * ex + ey * ey);
  const float ux = ex / L, uy = ey / L;
  float u[kExtMax], v[kExtMax], q[kExtMax], w[kExtMax];
#pragma unroll
  for (int i = 0; i < kExtMax; ++i) {
    const float dx = P[i].x - P[0].x, dy = P[i].y - P[0].y;
    u[i] = (dx * ux + dy * uy) / L;
    v[i] = (dy * ux - dx * uy) / L;
    q[i] = u[i] * u[i] + v[i] * v[i];
    const float t = L / M[i].sig_t();
    w[i] = t * t;
  }
  float S0 = 0.0f, S1 = 0.0f, S2 = 0.0f, S11 = 0.0f, S12 = 0.0f, S22 = 0.0f, T0 = 0.0f, T1 = 0.0f, T2 = 0.0f;
#pragma unroll
  for (int i = 0; i < kExtMax; ++i) {
    if (i < n) {
      S0 = S0 + w[i];
      S1 = S1 + w[i] * u[i];
      S2 = S2 + w[i] * q[i];
      S11 = S11 + (w[i] * u[i]) * u[i];
      S12 = S12 + (w[i] * u[i]) * q[i];
      S22 = S22 + (w[i] * q[i]) * q[i];
      T0 = T0 + w[i] * v[i];
      T1 = T1 + (w[i] * u[i]) * v[i];
      T2 = T2 + (w[i] * q[i]) * v[i];
    }
  }
  const float m00 = S11 * S22 - S12 * S12;
  const float m01 = S1 * S22 - S12 * S2;
  const float m02 = S1 * S12 - S11 * S2;
  const float det = (S0 * m00 - S1 * m01) + S2 * m02;
  if (!(det > 0.0f)) return false;
  const float n1 = T1 * S22 - S12 * T2;
  const float n2 = T1 * S12 - S11 * T2;
  const float n3 = S1 * T2 - T1 * S2;
  const float deta = (T0 * m00 - S1 * n1) + S2 * n2;
  const float detb = (S0 * n1 - T0 * m01) + S2 * n3;
  const float detc = (S0 * (S11 * T2 - T1 * S12) - S1 * n3) + T0 * m02;
  const float fa = deta / det, fb = detb / det, fc = detc / det;
  float chi2xy = 0.0f;
#pragma unroll
  for (int i = 0; i < kExtMax; ++i) {
    const float r = v[i] - ((fa + fb * u[i]) + fc * q[i]);
    if (i < n) chi2xy = chi2xy + (w[i] * r) * r;
  }
  const float disc = (1.0f + fb * fb) - (4.0f * fa) * fc;
  if (!(disc > 0.0f)) return false;
  const float kap = (2.0f * fc) / (L * sqrtf(disc));
  if (!(chi2xy <= (float)(kXExtXyD * (double)(n - 3)))) return false;
  float s[kExtMax];
  s[0] = 0.0f;
  bool series_ok = true;
#pragma unroll
  for (int i = 1; i < kExtMax; ++i) {
    const float dx = P[i].x - P[i - 1].x, dy = P[i].y - P[i - 1].y;
    const float Lc = sqrtf(dx * dx + dy * dy);
    const float xs = (kap * Lc) * 0.5f;
    if (i < n && !(fabsf(xs) <= kXSeriesMax)) series_ok = false;
    s[i] = s[i - 1] + Lc * arc_over_chord(xs);
  }
  if (!series_ok) return false;
  float sL = s[0];
#pragma unroll
  for (int i = 1; i < kExtMax; ++i)
    if (i == n - 1) sL = s[i];
  const float lam0 = (PL.z - P[0].z) / sL;
  float S = 0.0f, Ss = 0.0f, Sz = 0.0f;
#pragma unroll
  for (int i = 0; i < kExtMax; ++i) {
    const float sg = M[i].sig_z(lam0);
    w[i] = 1.0f / (sg * sg);
    if (i < n) {
      S = S + w[i];
      Ss = Ss + w[i] * s[i];
      Sz = Sz + w[i] * P[i].z;
    }
  }
  const float sbar = Ss / S, zbar = Sz / S;
  float Sss = 0.0f, Ssz = 0.0f;
#pragma unroll
  for (int i = 0; i < kExtMax; ++i) {
    const float ds = s[i] - sbar, dzz = P[i].z - zbar;
    if (i < n) {
      Sss = Sss + (w[i] * ds) * ds;
      Ssz = Ssz + (w[i] * ds) * dzz;
    }
  }
  const float lam = Ssz / Sss;
  float chi2rz = 0.0f;
#pragma unroll
  for (int i = 0; i < kExtMax; ++i) {
    const float r = (P[i].z - zbar) - lam * (s[i] - sbar);
    if (i < n) chi2rz = chi2rz + (w[i] * r) * r;
  }
  if (!(chi2rz <= (float)(kXExtRzD * (double)(n - 2)))) return false;
  *out = make_float3(chi2xy, chi2rz, kap);
  return true;
}

// ------------------------------------------------------- pT3 / pT5 (S2.4)
// Seed: sd = (pT, cx, cy, lambda, kappa, x0, y0, z0).  Anchors P[0..K-1].
struct Seed {
  float pt, cx, cy, lam, ks, x0, y0, z0;
};

// window around the seed hypothesis at the first anchor (part of the selection)
__device__ __forceinline__ bool seed_box(const Seed &sd, float ax, float ay) {
  const float hk = sd.ks * 0.5f;
  const float dx = ax - sd.x0, dy = ay - sd.y0;
  const float u1 = dx * sd.cx + dy * sd.cy, v1 = dy * sd.cx - dx * sd.cy;
  const float r1 = v1 - hk * (u1 * u1 + v1 * v1);
  return (u1 > 0.0f) && (fabsf(r1) <= kBoxXY);
}

// The first-anchor part of pt_pass on its own (the same operations in the
// same order: seed window, arc-length series validity, z window), so that a
// candidate failing it is known to fail pt_pass before its other anchors are read.
__device__ __forceinline__ bool pt_first_anchor(const Seed &sd, float4 A, ModInfo m) {
  if (!seed_box(sd, A.x, A.y)) return false;
  const float hk = sd.ks * 0.5f;
  const float ddx = A.x - sd.x0, ddy = A.y - sd.y0;
  const float Lc = sqrtf(ddx * ddx + ddy * ddy);
  const float xs = hk * Lc;
  if (!(fabsf(xs) <= kXSeriesMax)) return false;
  const float s = 0.0f + Lc * arc_over_chord(xs);
  const float sz = m.sig_z(sd.lam);
  const float rz = A.z - (sd.z0 + sd.lam * s);
  return fabsf(rz) <= kBoxZ0 + 2.0f * sz;
}

template <int K>
__device__ __forceinline__ bool pt_pass(const Seed &sd, const float4 *P, const ModInfo *M, float kT, float dkT,
                                        float4 *out) {
  const float hk = sd.ks * 0.5f;
  const float sk = kSeedDpt * fabsf(sd.ks);
  if (!seed_box(sd, P[0].x, P[0].y)) return false;
  float s = 0.0f, px = sd.x0, py = sd.y0, chi_xy = 0.0f, chi_rz = 0.0f;
#pragma unroll
  for (int i = 0; i < K; ++i) {
    const float ddx = P[i].x - px, ddy = P[i].y - py;
    const float Lc = sqrtf(ddx * ddx + ddy * ddy);
    const float xs = hk * Lc;
    if (!(fabsf(xs) <= kXSeriesMax)) return false;
    s = s + Lc * arc_over_chord(xs);
    px = P[i].x; py = P[i].y;
    const float ex = P[i].x - sd.x0, ey = P[i].y - sd.y0;
    const float u = ex * sd.cx + ey * sd.cy, v = ey * sd.cx - ex * sd.cy;
    const float qq = u * u + v * v;
    const float r = v - hk * qq;
    const float st = M[i].sig_t();
    const float sa = (sk * qq) * 0.5f, sb = kSeedDdir * u;
    const float var = (st * st + sa * sa) + sb * sb;
    chi_xy = chi_xy + (r * r) / var;
    const float sz = M[i].sig_z(sd.lam);
    const float rz = P[i].z - (sd.z0 + sd.lam * s);
    if (i == 0 && !(fabsf(rz) <= kBoxZ0 + 2.0f * sz)) return false;
    chi_rz = chi_rz + (rz * rz) / (sz * sz);
  }
  if (!(chi_xy <= (K == 3 ? kXPxy3 : kXPxy5))) return false;
  if (!(chi_rz <= (K == 3 ? kXPrz3 : kXPrz5))) return false;
  const float dks = sd.ks - kT;
  if (!(fabsf(dks) <= 3.0f * sk + dkT)) return false;
  *out = make_float4(chi_xy, chi_rz, chi_xy + chi_rz, 0.0f);
  return true;
}

// ---------------------------------------------------- proximity (S2.5)
// Direction at the beam line (d) and slope of an object.
struct Dir {
  float dx, dy, lam;
};
__device__ __forceinline__ Dir seed_dir(const Seed &sd) {
  Dir d;
  d.dx = sd.cx + sd.ks * sd.y0;
  d.dy = sd.cy - sd.ks * sd.x0;
  d.lam = sd.lam;
  return d;
}
// same hemisphere and sin^2(dphi) + dlambda^2 / (1 + mean lambda^2) < D^2
__device__ __forceinline__ bool near_dir(const Dir &a, const Dir &b, float D) {
  const float dot = a.dx * b.dx + a.dy * b.dy;
  if (!(dot > 0.0f)) return false;
  const float cr = a.dx * b.dy - a.dy * b.dx;
  const float na = a.dx * a.dx + a.dy * a.dy, nb = b.dx * b.dx + b.dy * b.dy;
  const float dl = a.lam - b.lam, lm = (a.lam + b.lam) * 0.5f;
  const float dr2 = (cr * cr) / (na * nb) + (dl * dl) / (1.0f + lm * lm);
  return dr2 < D * D;
}

}  // namespace lst
