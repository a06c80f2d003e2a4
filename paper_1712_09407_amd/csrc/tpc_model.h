// Track model of the Kalman filter: exact helix steps in a sector's local
// frame with their analytic Jacobian, the Kalman update with a (y, z)
// measurement, the three-point seed and the rotation into a neighbouring
// sector's frame (section 1: tracklets are fit with a Kalman filter and
// extrapolated to adjacent rows; section 5: global tracking continues in the
// neighbour's coordinate system).
//
// State (y, z, sin phi, tan lambda, q/pT) at the x of a pad row, in FP32.
// The covariance and the Kalman gain are FP64: the filter starts from a
// diffuse prior (variance 100 on q/pT against about 1e-3 at the end of a
// low-pT track), and the covariance form of the filter then subtracts
// nearly equal numbers in both the transport J C J^T and the update
// C - K H C.  In FP32 that cancellation leaves errors of 1e-3 relative in
// the q/pT of low-pT tracks.  In FP64 they fall below 1e-4, while the state,
// the Jacobian and the measurements stay FP32.  FP64 fused multiply-adds
// issue at the rate of non-packed FP32 ones on CDNA, so the cost is registers,
// not issue slots.
//
// Every function is __host__ __device__: the CPU tests compile this header
// for the host and run the same arithmetic beside the FP64 oracle.
#pragma once

#include <hip/hip_runtime.h>
#include <math.h>

#include "tpc_internal.h"

namespace tpc {

// Reciprocal and square roots: the hardware instructions on the device
// (about 1 ulp), correctly rounded operations on the host.
__host__ __device__ __forceinline__ float frcp(float x) {
#if defined(__HIP_DEVICE_COMPILE__)
  return __builtin_amdgcn_rcpf(x);
#else
  return 1.f / x;
#endif
}
__host__ __device__ __forceinline__ float fsqrt(float x) {
#if defined(__HIP_DEVICE_COMPILE__)
  return __builtin_amdgcn_sqrtf(x);
#else
  return sqrtf(x);
#endif
}
__host__ __device__ __forceinline__ float frsq(float x) {
#if defined(__HIP_DEVICE_COMPILE__)
  return __builtin_amdgcn_rsqf(x);
#else
  return 1.f / sqrtf(x);
#endif
}

// Lower-triangular packed symmetric 5x5 covariance (FP64).
struct Cov {
  double c00, c10, c11, c20, c21, c22, c30, c31, c32, c33, c40, c41, c42, c43, c44;
};

struct KState {
  float x, y, z, sp, tl, qpt;
  Cov C;
};

__host__ __device__ __forceinline__ void reset_cov(Cov& C, const KParams& kp) {
  C.c00 = kp.sy2;
  C.c11 = kp.sz2;
  C.c22 = kp.prior_sinphi;
  C.c33 = kp.prior_tanl;
  C.c44 = kp.prior_qpt;
  C.c10 = C.c20 = C.c21 = C.c30 = C.c31 = C.c32 = C.c40 = C.c41 = C.c42 = C.c43 = 0.0;
}

// asin(u)/u and its derivative; series below |u| = 0.1 (next term < 1e-9).
__host__ __device__ __forceinline__ float asinc(float u) {
  const float u2 = u * u;
  if (u2 < 0.01f) return 1.f + u2 * (1.f / 6.f + u2 * (3.f / 40.f + u2 * (5.f / 112.f)));
  return asinf(u) * frcp(u);
}
__host__ __device__ __forceinline__ float asinc_d(float u, float isq) {
  const float u2 = u * u;
  if (u2 < 0.01f) return u * (1.f / 3.f + u2 * (3.f / 10.f + u2 * (15.f / 56.f)));
  return (u * isq - asinf(u)) * frcp(u2);
}

// Exact helix step to x2 with the analytic Jacobian.  Returns false, leaving
// the state unchanged, if |sin phi| would pass max_sinphi.
__host__ __device__ __forceinline__ bool propagate(KState& s, float x2, const KParams& kp) {
  const float k = kp.k_curv;
  const float dx = x2 - s.x;
  const float kap = k * s.qpt;
  const float s1 = s.sp, s2 = s1 - kap * dx;
  if (fabsf(s1) > kp.max_sinphi || fabsf(s2) > kp.max_sinphi) return false;
  const float ic1 = frsq((1.f - s1) * (1.f + s1)), ic2 = frsq((1.f - s2) * (1.f + s2));
  const float c1 = (1.f - s1) * (1.f + s1) * ic1, c2 = (1.f - s2) * (1.f + s2) * ic2;
  const float T = (s1 + s2) * frcp(c1 + c2);
  const float Q2 = 1.f + T * T;
  const float iQ = frsq(Q2);
  const float Q = Q2 * iQ;
  const float u = 0.5f * kap * dx * Q;
  const float isq = frsq(1.f - u * u);
  const float h = asinc(u);
  const float ds = dx * Q * h;
  const float dT_ds1 = 0.5f * Q2 * (ic1 + ic2);
  const float dT_dk = -0.5f * Q2 * dx * ic2;
  const float TQ = T * iQ;
  const float dds_ds1 = dx * TQ * dT_ds1 * isq;
  const float dds_dk = dx * (TQ * dT_dk * isq + 0.5f * Q2 * dx * asinc_d(u, isq));
  // the Jacobian's non-trivial entries, widened for the covariance transport
  const double a = dx * dT_ds1;        // dy/dsinphi
  const double bq = dx * dT_dk * k;    // dy/dqpt
  const double c = s.tl * dds_ds1;     // dz/dsinphi
  const double d = ds;                 // dz/dtanl
  const double ee = s.tl * dds_dk * k; // dz/dqpt
  const double f = -dx * k;            // dsinphi/dqpt
  Cov& C = s.C;
  // T = J C (rows 0..2 differ from C)
  const double t00 = C.c00 + a * C.c20 + bq * C.c40;
  const double t02 = C.c20 + a * C.c22 + bq * C.c42;
  const double t04 = C.c40 + a * C.c42 + bq * C.c44;
  const double t10 = C.c10 + c * C.c20 + d * C.c30 + ee * C.c40;
  const double t11 = C.c11 + c * C.c21 + d * C.c31 + ee * C.c41;
  const double t12 = C.c21 + c * C.c22 + d * C.c32 + ee * C.c42;
  const double t13 = C.c31 + c * C.c32 + d * C.c33 + ee * C.c43;
  const double t14 = C.c41 + c * C.c42 + d * C.c43 + ee * C.c44;
  const double t20 = C.c20 + f * C.c40;
  const double t21 = C.c21 + f * C.c41;
  const double t22 = C.c22 + f * C.c42;
  const double t23 = C.c32 + f * C.c43;
  const double t24 = C.c42 + f * C.c44;
  Cov N;
  N.c00 = t00 + a * t02 + bq * t04;
  N.c10 = t10 + a * t12 + bq * t14;
  N.c11 = t11 + c * t12 + d * t13 + ee * t14;
  N.c20 = t20 + a * t22 + bq * t24;
  N.c21 = t21 + c * t22 + d * t23 + ee * t24;
  N.c22 = t22 + f * t24;
  N.c30 = C.c30 + a * C.c32 + bq * C.c43;
  N.c31 = C.c31 + c * C.c32 + d * C.c33 + ee * C.c43;
  N.c32 = C.c32 + f * C.c43;
  N.c33 = C.c33;
  N.c40 = C.c40 + a * C.c42 + bq * C.c44;
  N.c41 = C.c41 + c * C.c42 + d * C.c43 + ee * C.c44;
  N.c42 = C.c42 + f * C.c44;
  N.c43 = C.c43;
  N.c44 = C.c44;
  C = N;
  s.y += dx * T;
  s.z += s.tl * ds;
  s.sp = s2;
  s.x = x2;
  return true;
}

// Kalman update with the measurement (my, mz); returns its chi^2.  The gain
// is computed in FP64 from the FP64 covariance, so that the plain update
// C -= K H C stays consistent with it.
__host__ __device__ __forceinline__ float kf_update(KState& s, float my, float mz,
                                                    const KParams& kp) {
  Cov& C = s.C;
  const double S00 = C.c00 + (double)kp.sy2, S01 = C.c10, S11 = C.c11 + (double)kp.sz2;
  const double idet = 1.0 / (S00 * S11 - S01 * S01);
  const double i00 = S11 * idet, i01 = -S01 * idet, i11 = S00 * idet;
  const double ry = my - s.y, rz = mz - s.z;
  const double chi2 = ry * ry * i00 + 2.0 * ry * rz * i01 + rz * rz * i11;
  // K = C H^T S^-1 (columns 0 and 1 of C)
  const double k00 = C.c00 * i00 + C.c10 * i01, k01 = C.c00 * i01 + C.c10 * i11;
  const double k10 = C.c10 * i00 + C.c11 * i01, k11 = C.c10 * i01 + C.c11 * i11;
  const double k20 = C.c20 * i00 + C.c21 * i01, k21 = C.c20 * i01 + C.c21 * i11;
  const double k30 = C.c30 * i00 + C.c31 * i01, k31 = C.c30 * i01 + C.c31 * i11;
  const double k40 = C.c40 * i00 + C.c41 * i01, k41 = C.c40 * i01 + C.c41 * i11;
  s.y += (float)(k00 * ry + k01 * rz);
  s.z += (float)(k10 * ry + k11 * rz);
  s.sp += (float)(k20 * ry + k21 * rz);
  s.tl += (float)(k30 * ry + k31 * rz);
  s.qpt += (float)(k40 * ry + k41 * rz);
  // C -= K (H C): rows 0 and 1 of the old C
  const double h00 = C.c00, h01 = C.c10, h02 = C.c20, h03 = C.c30, h04 = C.c40;
  const double h10 = C.c10, h11 = C.c11, h12 = C.c21, h13 = C.c31, h14 = C.c41;
  C.c00 -= k00 * h00 + k01 * h10;
  C.c10 -= k10 * h00 + k11 * h10;
  C.c11 -= k10 * h01 + k11 * h11;
  C.c20 -= k20 * h00 + k21 * h10;
  C.c21 -= k20 * h01 + k21 * h11;
  C.c22 -= k20 * h02 + k21 * h12;
  C.c30 -= k30 * h00 + k31 * h10;
  C.c31 -= k30 * h01 + k31 * h11;
  C.c32 -= k30 * h02 + k31 * h12;
  C.c33 -= k30 * h03 + k31 * h13;
  C.c40 -= k40 * h00 + k41 * h10;
  C.c41 -= k40 * h01 + k41 * h11;
  C.c42 -= k40 * h02 + k41 * h12;
  C.c43 -= k40 * h03 + k41 * h13;
  C.c44 -= k40 * h04 + k41 * h14;
  return (float)chi2;
}

// Seed from chain clusters a (first), b (middle) and e (last of the seed
// window): the circle through them in (x, y) gives curvature and direction at
// a; tan lambda is the z rise over the arc a -> e.
__host__ __device__ __forceinline__ void seed3(KState& s, float xa, float ya, float za, float xb,
                                               float yb, float xe, float ye, float ze,
                                               const KParams& kp) {
  const float d1x = xb - xa, d1y = yb - ya, d2x = xe - xa, d2y = ye - ya;
  float kappa = 0.f;
  if (kp.bz != 0.f) {
    const float cross = d1x * d2y - d1y * d2x;
    const float den = sqrtf(d1x * d1x + d1y * d1y) * sqrtf(d2x * d2x + d2y * d2y) *
                      sqrtf((d2x - d1x) * (d2x - d1x) + (d2y - d1y) * (d2y - d1y));
    kappa = den > 0.f ? -2.f * cross / den : 0.f;
  }
  const float L = sqrtf(d2x * d2x + d2y * d2y);
  float u = 0.5f * kappa * L;
  u = fminf(fmaxf(u, -1.f), 1.f);
  s.x = xa;
  s.y = ya;
  s.z = za;
  s.sp = (d2y / L) * sqrtf(1.f - u * u) + (d2x / L) * u;
  s.tl = (ze - za) / (L * asinc(u));
  s.qpt = kp.bz != 0.f ? kappa / kp.k_curv : 0.f;
  reset_cov(s.C, kp);
}

// Rotation of the local frame by the angle whose cosine and sine are (ca, sa):
// the point and the direction stay, x becomes the rotated x.  A change of y
// at fixed x is carried along the track onto the new reference plane:
// dy'/dy = cos(phi)/cos(phi'), dz'/dy = -sin(d) tan(lambda)/cos(phi'),
// dsin(phi')/dy = kappa sin(d), dsin(phi')/dsin(phi) = cos(phi')/cos(phi).
// False (state unchanged) if the direction would not point along +x'.
__host__ __device__ __forceinline__ bool rotate(KState& s, float ca, float sa, const KParams& kp) {
  const float sp = s.sp, cp = fsqrt((1.f - sp) * (1.f + sp));
  const float sp2 = sp * ca - cp * sa, cp2 = cp * ca + sp * sa;
  if (!(cp2 > 0.f)) return false;
  const double j00 = cp / cp2, j10 = -sa * s.tl / cp2, j20 = kp.k_curv * s.qpt * sa;
  const double j22 = cp2 / cp;
  Cov& C = s.C;
  // rows of J C: row 1 = j10 (C row 0) + (C row 1), row 2 = j20 (C row 0) + j22 (C row 2)
  const double b0 = j10 * C.c00 + C.c10, b1 = j10 * C.c10 + C.c11;
  const double b3 = j10 * C.c30 + C.c31, b4 = j10 * C.c40 + C.c41;
  const double a0 = j20 * C.c00 + j22 * C.c20, a1 = j20 * C.c10 + j22 * C.c21;
  const double a2 = j20 * C.c20 + j22 * C.c22, a3 = j20 * C.c30 + j22 * C.c32;
  const double a4 = j20 * C.c40 + j22 * C.c42;
  Cov N;
  N.c00 = j00 * j00 * C.c00;
  N.c10 = j00 * b0;
  N.c11 = b0 * j10 + b1;
  N.c20 = j00 * a0;
  N.c21 = a0 * j10 + a1;
  N.c22 = a0 * j20 + a2 * j22;
  N.c30 = j00 * C.c30;
  N.c31 = b3;
  N.c32 = a3;
  N.c33 = C.c33;
  N.c40 = j00 * C.c40;
  N.c41 = b4;
  N.c42 = a4;
  N.c43 = C.c43;
  N.c44 = C.c44;
  C = N;
  const float x2 = s.x * ca + s.y * sa, y2 = -s.x * sa + s.y * ca;
  s.x = x2;
  s.y = y2;
  s.sp = sp2;
  return true;
}

// The helix parameters alone, stepped to x2 with the same formulas as
// propagate (no Jacobian): for checks along a path whose covariance is
// needed only at its end.
struct HelixPar {
  float x, y, z, sp, tl, qpt;
};
__host__ __device__ __forceinline__ bool step_par(HelixPar& h, float x2, const KParams& kp) {
  const float dx = x2 - h.x;
  const float kap = kp.k_curv * h.qpt;
  const float s1 = h.sp, s2 = s1 - kap * dx;
  if (fabsf(s1) > kp.max_sinphi || fabsf(s2) > kp.max_sinphi) return false;
  const float c1 = (1.f - s1) * (1.f + s1) * frsq((1.f - s1) * (1.f + s1));
  const float c2 = (1.f - s2) * (1.f + s2) * frsq((1.f - s2) * (1.f + s2));
  const float T = (s1 + s2) * frcp(c1 + c2);
  const float Q2 = 1.f + T * T;
  const float Q = Q2 * frsq(Q2);
  const float u = 0.5f * kap * dx * Q;
  h.y += dx * T;
  h.z += h.tl * dx * Q * asinc(u);
  h.sp = s2;
  h.x = x2;
  return true;
}

}  // namespace tpc
