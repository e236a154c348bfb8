// Device-side helpers: boundary reflection, element loads and the per-voxel
// eigen / FA / cylindrical-angle epilogue.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "st_internal.h"

namespace st {

// Half-sample symmetric reflection of index m into [0, n): -1 -> 0, n -> n-1,
// folded with period 2n for indices farther out.  Positions are 32-bit (every
// size is below 2^31), so with wave-uniform arguments the compares run on the
// scalar unit, which has no 64-bit signed compare.
__device__ __forceinline__ int reflect_lane(int m, int n) {
  if (m >= 0 && m < n) return m;
  const int p = 2 * n;
  m %= p;
  if (m < 0) m += p;
  return m < n ? m : p - 1 - m;
}

// Entry of a grouped launch that block b belongs to: the last e with
// first[e] <= b (b is wave-uniform, so the search runs on the scalar unit).
__device__ __forceinline__ int group_entry(const int64_t* __restrict__ first, int count, int64_t b) {
  int lo = 0, hi = count - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (first[mid] <= b) lo = mid; else hi = mid - 1;
  }
  return lo;
}

__device__ __forceinline__ float load_as_float(const uint16_t* p) { return static_cast<float>(*p); }
__device__ __forceinline__ float load_as_float(const float* p) { return *p; }

// Polynomial kernels fitted for this library: near-minimax in relative error,
// found with Lawson's iteratively reweighted least squares (C. L. Lawson,
// 1961) on 8000 Chebyshev-distributed points, leading term fixed at 1.
// atan(t) = t + t^3 P(t^2) on [0, 1]: relative error below 1.7e-8.
__device__ __forceinline__ float atan_unit(float t) {
  const float u = t * t;
  float q = 0.0029206906f;
  q = fmaf(q, u, -0.016367922f);
  q = fmaf(q, u, 0.043211852f);
  q = fmaf(q, u, -0.075522136f);
  q = fmaf(q, u, 0.10666004f);
  q = fmaf(q, u, -0.14211055f);
  q = fmaf(q, u, 0.19993773f);
  q = fmaf(q, u, -0.33333153f);
  return fmaf(t * u, q, t);
}

// atan2(y, x) for x >= 0, in [-pi/2, pi/2] (0 for x = y = 0): the octant
// reduction atan(y/x) = pi/2 - atan(x/y) keeps the polynomial argument in [0, 1].
__device__ __forceinline__ float atan2_right(float y, float x) {
  const float ay = fabsf(y);
  const float hi = fmaxf(ay, x), lo = fminf(ay, x);
  const float t = hi > 0.f ? lo * __builtin_amdgcn_rcpf(hi) : 0.f;
  float a = atan_unit(fminf(t, 1.f));
  a = ay > x ? 1.5707963705062866f - a : a;
  return y < 0.f ? -a : a;
}

// asin(x) = x + x^3 Q(x^2) on [0, sqrt(1/2)]: relative error below 1.6e-8.
__device__ __forceinline__ float asin_half(float x) {
  const float u = x * x;
  float q = 0.11124149f;
  q = fmaf(q, u, -0.092497088f);
  q = fmaf(q, u, 0.076894834f);
  q = fmaf(q, u, 0.016413327f);
  q = fmaf(q, u, 0.046498492f);
  q = fmaf(q, u, 0.074885110f);
  q = fmaf(q, u, 0.16666905f);
  return fmaf(x * u, q, x);
}

// Helix and intrusion angles of the unit fibre vector v at voxel (pz, py, px)
// in the cylindrical frame about the axis through c with unit direction a
// (all (z, y, x)).  With q_perp the component of (p - c) normal to the axis
// (length r), e_r = q_perp / r and e_t = a x e_r (right-handed (x, y, z)
// order); f_* = v . e_*, HA = atan2(f_a sgn f_t, |f_t|) and
// IA = atan2(f_r sgn f_t, |f_t|) with sgn(0) = +1.  f_r and f_t are formed
// from the unnormalised q_perp and a x q_perp (both scaled by r), so only HA
// needs r itself.  Returns true (ha = ia = 0) when the voxel lies on the axis.
__device__ __forceinline__ bool fibre_angles(double vz, double vy, double vx, const double c[3],
                                             const double a[3], double pz, double py, double px,
                                             float& ha, float& ia) {
  const double qz = pz - c[0], qy = py - c[1], qx = px - c[2];
  const double qa = qz * a[0] + qy * a[1] + qx * a[2];
  const double ez = qz - qa * a[0], ey = qy - qa * a[1], ex = qx - qa * a[2];
  const double r2 = ez * ez + ey * ey + ex * ex;
  if (r2 < 1e-18) {
    ha = 0.f;
    ia = 0.f;
    return true;
  }
  const float fz = static_cast<float>(ez), fy = static_cast<float>(ey), fx = static_cast<float>(ex);
  const float az = static_cast<float>(a[0]), ay = static_cast<float>(a[1]), ax = static_cast<float>(a[2]);
  // a x q_perp taken in right-handed (x, y, z) order, stored (z, y, x)
  const float tz = ax * fy - ay * fx;
  const float ty = az * fx - ax * fz;
  const float tx = ay * fz - az * fy;
  const float uz = static_cast<float>(vz), uy = static_cast<float>(vy), ux = static_cast<float>(vx);
  const float f_r = uz * fz + uy * fy + ux * fx;   // r * (v . e_r)
  const float f_t = uz * tz + uy * ty + ux * tx;   // r * (v . e_t)
  const float f_a = uz * az + uy * ay + ux * ax;   // v . a
  const float r = __builtin_amdgcn_sqrtf(static_cast<float>(r2));
  const float den = fabsf(f_t);
  const float sg = f_t >= 0.f ? 1.f : -1.f;
  ha = atan2_right(f_a * r * sg, den);
  ia = atan2_right(f_r * sg, den);
  return false;
}

// Null vector of A - mu I (A symmetric, components zz, zy, zx, yy, yx, xx):
// the largest of the three cross products of pairs of its rows (Kopp 2008).
// Returns it unnormalised with its squared length.
__device__ __forceinline__ void null_vector(double zz, double zy, double zx, double yy, double yx,
                                            double xx, double mu, double& vz, double& vy,
                                            double& vx, double& nn) {
  const double a = zz - mu, b = yy - mu, c = xx - mu;
  const double c0z = zy * yx - zx * b, c0y = zx * zy - a * yx, c0x = a * b - zy * zy;  // r0 x r1
  const double c1z = zy * c - zx * yx, c1y = zx * zx - a * c, c1x = a * yx - zy * zx;  // r0 x r2
  const double c2z = b * c - yx * yx, c2y = yx * zx - zy * c, c2x = zy * yx - b * zx;  // r1 x r2
  const double n0 = c0z * c0z + c0y * c0y + c0x * c0x;
  const double n1 = c1z * c1z + c1y * c1y + c1x * c1x;
  const double n2 = c2z * c2z + c2y * c2y + c2x * c2x;
  vz = c0z; vy = c0y; vx = c0x; nn = n0;
  if (n1 > nn) { vz = c1z; vy = c1y; vx = c1x; nn = n1; }
  if (n2 > nn) { vz = c2z; vy = c2y; vx = c2x; nn = n2; }
}

// sin and cos of x in [0, pi/3] by their Taylor series through x^11 / x^12
// (truncation error below 1e-9, under float32 rounding).
__device__ __forceinline__ void sincos_small(float x, float& s, float& c) {
  const float x2 = x * x;
  s = x * (1.f + x2 * (-1.f / 6.f + x2 * (1.f / 120.f + x2 * (-1.f / 5040.f +
          x2 * (1.f / 362880.f + x2 * (-1.f / 39916800.f))))));
  c = 1.f + x2 * (-0.5f + x2 * (1.f / 24.f + x2 * (-1.f / 720.f + x2 * (1.f / 40320.f +
          x2 * (-1.f / 3628800.f + x2 * (1.f / 479001600.f))))));
}

// Reciprocal square root in float64: the hardware estimate refined by two
// Newton-Raphson steps (each squares the relative error).
__device__ __forceinline__ double rsq64(double a) {
  double y = __builtin_amdgcn_rsq(a);
  const double h = 0.5 * a;
  y = y * fma(-h * y, y, 1.5);
  return y * fma(-h * y, y, 1.5);
}

struct EigOut {
  double vz, vy, vx;  // unit e3, canonical sign
  float l1, l2, l3;   // lambda1 >= lambda2 >= lambda3
  float fa;
  bool degenerate;    // trace <= 0 or (lambda2 - lambda3) / trace < 1e-3
};

// Smallest-eigenvalue eigenvector of one symmetric 3x3 tensor (float64
// components), its eigenvalues, FA and the degeneracy test.
//
// The invariants of the deviatoric part D = S - mI (m = tr/3, q = |D|_F^2 / 6,
// r = det(D) / (2 q^(3/2))) are formed in float64, and the eigen-angle
// phi = acos(r)/3 of the trigonometric solution of the characteristic cubic
// (O. K. Smith, "Eigenvalues of a symmetric 3x3 matrix", CACM 1961;
// mu_k = 2 sqrt(q) cos(phi + 2 pi k / 3)) is taken as (2/3) asin(sqrt((1 - |r|)/2))
// (or pi/3 minus that for r < 0), which keeps full relative accuracy where
// acos(r) is ill-conditioned (|r| -> 1).  That float32-accurate mu_3 gets one
// float64 Newton step on the deviatoric characteristic polynomial
// mu^3 - (|D|_F^2 / 2) mu - det D, which squares its relative error, and the
// eigenvector is the largest cross product of two rows of D - mu_3 I
// (J. Kopp, "Efficient numerical diagonalization of hermitian 3x3 matrices",
// 2008).  FA = sqrt(3/2 |D|_F^2 / |S|_F^2), the eigenvalue form rewritten in
// invariants, is finished in float32 once the two float64 norms are formed.
__device__ __forceinline__ void eig_smallest(const double s6[6], EigOut& o) {
  const double zz = s6[0], zy = s6[1], zx = s6[2], yy = s6[3], yx = s6[4], xx = s6[5];
  const double tr = zz + yy + xx;
  const double m = tr * (1.0 / 3.0);
  o.vz = 1.0; o.vy = 0.0; o.vx = 0.0;
  o.degenerate = true;
  o.fa = 0.f;
  o.l1 = o.l2 = o.l3 = static_cast<float>(m);
  if (!(tr > 0.0)) return;
  const double dz = zz - m, dy = yy - m, dx = xx - m;
  const double off = zy * zy + zx * zx + yx * yx;
  const double p2 = dz * dz + dy * dy + dx * dx + 2.0 * off;  // |D|_F^2
  const double f2 = zz * zz + yy * yy + xx * xx + 2.0 * off;  // |S|_F^2
  {
    double rf = __builtin_amdgcn_rcp(f2);
    rf = fma(rf, fma(-f2, rf, 1.0), rf);
    o.fa = fminf(1.f, __builtin_amdgcn_sqrtf(static_cast<float>(1.5 * p2 * rf)));
  }
  if (!(p2 > 1e-28 * tr * tr)) return;  // isotropic to working precision
  const double det = dz * (dy * dx - yx * yx) - zy * (zy * dx - yx * zx) + zx * (zy * yx - dy * zx);
  const double q = p2 * (1.0 / 6.0);
  const double iq = rsq64(q);                          // 1 / sqrt(q)
  double r = 0.5 * det * (iq * iq * iq);               // det / (2 q^(3/2))
  r = fmin(1.0, fmax(-1.0, r));
  const float h = static_cast<float>(0.5 * (1.0 - fabs(r)));
  const float a = (2.f / 3.f) * asin_half(__builtin_amdgcn_sqrtf(h));
  const float phi = r >= 0.0 ? a : 1.0471975511965976f - a;  // pi/3 - a
  float sf, cf;
  sincos_small(phi, sf, cf);
  const double k3 = 1.7320508075688772;  // sqrt(3)
  const double sq = q * iq;              // sqrt(q)
  const double cs = cf, sn = sf;
  double mu = -sq * (cs + k3 * sn);      // smallest root
  const double mu1 = 2.0 * sq * cs;      // largest root
  const double gap = 2.0 * k3 * sq * sn; // mu_2 - mu_3
  {
    const double j2 = 0.5 * p2;
    const double f = fma(mu, fma(mu, mu, -j2), -det);
    const double fp = fma(3.0 * mu, mu, -j2);  // (mu - mu_1)(mu - mu_2) >= 0 at mu_3
    const double step = f * __builtin_amdgcn_rcp(fp);
    if (fp > 0.0 && fabs(step) < 0.25 * gap) mu -= step;
  }
  o.l1 = static_cast<float>(m + mu1);
  o.l3 = static_cast<float>(m + mu);
  o.l2 = static_cast<float>(m - mu1 - mu);
  o.degenerate = gap < 1e-3 * tr;

  double vz, vy, vx, nn;
  null_vector(dz, zy, zx, dy, yx, dx, mu, vz, vy, vx, nn);
  if (!(nn > 0.0)) return;
  const double inv = rsq64(nn);
  vz *= inv; vy *= inv; vx *= inv;
  // canonical sign: largest |component| positive, ties to the lower axis (z, then y)
  const double az = fabs(vz), ay = fabs(vy), ax = fabs(vx);
  const double lead = (az >= ay && az >= ax) ? vz : (ay >= ax ? vy : vx);
  if (lead < 0.0) { vz = -vz; vy = -vy; vx = -vx; }
  o.vz = vz; o.vy = vy; o.vx = vx;
}

}  // namespace st
