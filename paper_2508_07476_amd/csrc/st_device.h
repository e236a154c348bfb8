// Device-side helpers: boundary reflection, element loads and the per-voxel
// eigen / FA / cylindrical-angle epilogue.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "st_internal.h"

namespace st {

// Half-sample symmetric reflection of index m into [0, n): -1 -> 0, n -> n-1,
// folded with period 2n for indices farther out.  Called with wave-uniform
// arguments, so it runs on the scalar unit.
__device__ __forceinline__ int64_t reflect(int64_t m, int64_t n) {
  if (m >= 0 && m < n) return m;
  const int64_t p = 2 * n;
  m %= p;
  if (m < 0) m += p;
  return m < n ? m : p - 1 - m;
}

// Per-lane variant for small |m| excursions (x-axis halos).
__device__ __forceinline__ int reflect_lane(int m, int n) {
  if (m >= 0 && m < n) return m;
  const int p = 2 * n;
  m %= p;
  if (m < 0) m += p;
  return m < n ? m : p - 1 - m;
}

__device__ __forceinline__ float load_as_float(const uint16_t* p) { return static_cast<float>(*p); }
__device__ __forceinline__ float load_as_float(const float* p) { return *p; }

// Helix and intrusion angles of the fibre vector v (any length) at voxel
// (pz, py, px) in the cylindrical frame about the axis through c with unit
// direction a (all (z, y, x)): e_r is the unit radial vector, e_t = a x e_r
// taken in right-handed (x, y, z) order, and with f_* = v . e_*,
// HA = atan2(f_a sgn f_t, |f_t|), IA = atan2(f_r sgn f_t, |f_t|), sgn(0) = +1.
// Returns true (and leaves ha = ia = 0) when the voxel lies on the axis.
__device__ __forceinline__ bool fibre_angles(double vz, double vy, double vx, const double c[3],
                                             const double a[3], double pz, double py, double px,
                                             float& ha, float& ia) {
  const double qz = pz - c[0], qy = py - c[1], qx = px - c[2];
  const double qa = qz * a[0] + qy * a[1] + qx * a[2];
  const double ez = qz - qa * a[0], ey = qy - qa * a[1], ex = qx - qa * a[2];
  const double rr = sqrt(ez * ez + ey * ey + ex * ex);
  if (rr < 1e-9) {
    ha = 0.f;
    ia = 0.f;
    return true;
  }
  const double ir = 1.0 / rr;
  const double erz = ez * ir, ery = ey * ir, erx = ex * ir;
  const double etz = a[2] * ery - a[1] * erx;
  const double ety = a[0] * erx - a[2] * erz;
  const double etx = a[1] * erz - a[0] * ery;
  const double f_r = vz * erz + vy * ery + vx * erx;
  const double f_t = vz * etz + vy * ety + vx * etx;
  const double f_a = vz * a[0] + vy * a[1] + vx * a[2];
  const double sg = f_t >= 0.0 ? 1.0 : -1.0;
  const float den = static_cast<float>(fabs(f_t));
  ha = atan2f(static_cast<float>(f_a * sg), den);
  ia = atan2f(static_cast<float>(f_r * sg), den);
  return false;
}

struct VoxelOut {
  float e3[3];
  float ev[3];
  float fa, ha, ia;
  uint32_t flags;
};

// Eigen-decomposition of one symmetric 3x3 tensor (float32 components, solved in
// float64), fractional anisotropy, degeneracy test and -- if an axis is given --
// helix and intrusion angles in the cylindrical frame at voxel (pz, py, px).
//
// Eigenvalues: trigonometric closed form for the characteristic cubic of the
// deviatoric tensor (O. K. Smith, "Eigenvalues of a symmetric 3x3 matrix",
// CACM 1961): with m = tr/3, p = sqrt(|S - mI|_F^2 / 6), r = det((S - mI)/p)/2
// and phi = acos(r)/3, the roots are m + 2p cos(phi + 2 pi k / 3).
// Eigenvector of lambda3: the largest cross product of two rows of S - lambda3 I
// (J. Kopp, "Efficient numerical diagonalization of hermitian 3x3 matrices",
// 2008), normalised and given the canonical sign.
// FA = sqrt(3/2 * |S - mI|_F^2 / |S|_F^2), identical to the eigenvalue form.
__device__ __forceinline__ void solve_voxel(const float s6[6], bool has_axis,
                                            const double c[3], const double a[3],
                                            double pz, double py, double px, VoxelOut& o) {
  const double szz = s6[0], szy = s6[1], szx = s6[2], syy = s6[3], syx = s6[4], sxx = s6[5];
  const double tr = szz + syy + sxx;
  const double m = tr * (1.0 / 3.0);
  const double dz = szz - m, dy = syy - m, dx = sxx - m;
  const double off = szy * szy + szx * szx + syx * syx;
  const double p2 = dz * dz + dy * dy + dx * dx + 2.0 * off;
  const double f2 = szz * szz + syy * syy + sxx * sxx + 2.0 * off;

  double l1 = m, l2 = m, l3 = m, gap = 0.0;
  double vz = 1.0, vy = 0.0, vx = 0.0;
  if (p2 > 1e-30 * f2 && p2 > 0.0) {
    const double p = sqrt(p2 * (1.0 / 6.0));
    const double ip = 1.0 / p;
    const double bzz = dz * ip, byy = dy * ip, bxx = dx * ip;
    const double bzy = szy * ip, bzx = szx * ip, byx = syx * ip;
    const double det = bzz * (byy * bxx - byx * byx) - bzy * (bzy * bxx - byx * bzx) +
                       bzx * (bzy * byx - byy * bzx);
    const double r = fmin(1.0, fmax(-1.0, 0.5 * det));
    const double phi = acos(r) * (1.0 / 3.0);
    double sn, cs;
    sincos(phi, &sn, &cs);
    const double k3 = 1.7320508075688772;  // sqrt(3)
    l1 = m + 2.0 * p * cs;
    l2 = m - p * (cs - k3 * sn);
    l3 = m - p * (cs + k3 * sn);
    gap = 2.0 * k3 * p * sn;

    const double r0z = szz - l3, r0y = szy, r0x = szx;
    const double r1z = szy, r1y = syy - l3, r1x = syx;
    const double r2z = szx, r2y = syx, r2x = sxx - l3;
    const double az0 = r0y * r1x - r0x * r1y, ay0 = r0x * r1z - r0z * r1x, ax0 = r0z * r1y - r0y * r1z;
    const double az1 = r0y * r2x - r0x * r2y, ay1 = r0x * r2z - r0z * r2x, ax1 = r0z * r2y - r0y * r2z;
    const double az2 = r1y * r2x - r1x * r2y, ay2 = r1x * r2z - r1z * r2x, ax2 = r1z * r2y - r1y * r2z;
    const double n0 = az0 * az0 + ay0 * ay0 + ax0 * ax0;
    const double n1 = az1 * az1 + ay1 * ay1 + ax1 * ax1;
    const double n2 = az2 * az2 + ay2 * ay2 + ax2 * ax2;
    double nb = n0, bz = az0, by = ay0, bx = ax0;
    if (n1 > nb) { nb = n1; bz = az1; by = ay1; bx = ax1; }
    if (n2 > nb) { nb = n2; bz = az2; by = ay2; bx = ax2; }
    if (nb > 0.0) {
      const double inv = 1.0 / sqrt(nb);
      vz = bz * inv; vy = by * inv; vx = bx * inv;
    }
  }
  // canonical sign: largest |component| positive, ties to the lower axis (z, then y)
  {
    const double az = fabs(vz), ay = fabs(vy), ax = fabs(vx);
    const double lead = (az >= ay && az >= ax) ? vz : (ay >= ax ? vy : vx);
    if (lead < 0.0) { vz = -vz; vy = -vy; vx = -vx; }
  }
  uint32_t flags = 0;
  if (!(tr > 0.0) || gap < 1e-3 * tr) flags |= ST_FLAG_DEGENERATE;

  float ha = 0.f, ia = 0.f;
  if (has_axis && fibre_angles(vz, vy, vx, c, a, pz, py, px, ha, ia)) flags |= ST_FLAG_ON_AXIS;
  o.e3[0] = static_cast<float>(vz);
  o.e3[1] = static_cast<float>(vy);
  o.e3[2] = static_cast<float>(vx);
  o.ev[0] = static_cast<float>(l1);
  o.ev[1] = static_cast<float>(l2);
  o.ev[2] = static_cast<float>(l3);
  o.fa = f2 > 0.0 ? static_cast<float>(sqrt(1.5 * p2 / f2)) : 0.f;
  o.ha = ha;
  o.ia = ia;
  o.flags = flags;
}

}  // namespace st
